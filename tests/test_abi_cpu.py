"""Host-only checks of the C ABI: the library loads, exports every function
declared in include/rsfde.h, and rejects bad arguments before touching a GPU."""

import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "rsfde.h")
# RSFDE_LIBRARY: the host-sanitised build (tests/test_sanitize_cpu.py runs this
# module's host checks against it)
LIB = os.environ.get("RSFDE_LIBRARY") or os.path.join(ROOT, "paper_2102_11576_amd", "librsfde.so")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rsfde_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librsfde.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"rsfde_setup", "rsfde_matvec", "rsfde_precond_apply", "rsfde_step",
            "rsfde_adjoint_step", "rsfde_destroy", "rsfde_strerror"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rsfde_\w+)", out))
    assert set(names) <= exported


def test_strerror(lib):
    lib.rsfde_strerror.restype = C.c_char_p
    assert lib.rsfde_strerror(0) == b"ok"
    assert lib.rsfde_strerror(-1) == b"invalid argument"
    assert lib.rsfde_strerror(-4).startswith(b"iteration cap")
    assert lib.rsfde_strerror(12345) == b"unknown error"


def test_host_validation_fails_fast(lib):
    from paper_2102_11576_amd._lib import rsfde_grid, rsfde_solver_opts, rsfde_stats
    P = C.c_void_p
    lib.rsfde_setup.argtypes = [C.POINTER(P), C.POINTER(rsfde_grid), C.c_double, C.c_double,
                                C.c_double, C.c_double, P, C.c_double, C.c_double, C.c_int32, P]
    h = P()
    fake = P(0x1000)  # never dereferenced: validation rejects first
    g = rsfde_grid(15, 15, 0.0, 1.0, 0.0, 1.0)
    assert lib.rsfde_setup(None, C.byref(g), 1.5, 1.5, 1.0, 1.0, fake, 1e-6, 0.1, 20, None) == -1
    assert lib.rsfde_setup(C.byref(h), None, 1.5, 1.5, 1.0, 1.0, fake, 1e-6, 0.1, 20, None) == -1
    for a1, a2, kx, ky, eta, dt in ((2.5, 1.5, 1, 1, 1e-6, .1), (1.5, 1.0, 1, 1, 1e-6, .1),
                                    (1.5, 1.5, -1, 1, 1e-6, .1), (1.5, 1.5, 1, 1, 0.0, .1),
                                    (1.5, 1.5, 1, 1, 1e-6, -0.1), (1.5, 1.5, 1, float("nan"), 1e-6, .1)):
        assert lib.rsfde_setup(C.byref(h), C.byref(g), a1, a2, kx, ky, fake, eta, dt, 20, None) == -1
        assert h.value is None
    bad = rsfde_grid(0, 15, 0.0, 1.0, 0.0, 1.0)
    assert lib.rsfde_setup(C.byref(h), C.byref(bad), 1.5, 1.5, 1, 1, fake, 1e-6, .1, 20, None) == -1
    flip = rsfde_grid(15, 15, 1.0, 0.0, 0.0, 1.0)
    assert lib.rsfde_setup(C.byref(h), C.byref(flip), 1.5, 1.5, 1, 1, fake, 1e-6, .1, 20, None) == -1
    assert lib.rsfde_setup(C.byref(h), C.byref(g), 1.5, 1.5, 1, 1, None, 1e-6, .1, 20, None) == -1
    assert lib.rsfde_setup(C.byref(h), C.byref(g), 1.5, 1.5, 1, 1, fake, 1e-6, .1, 65, None) == -1
    big = rsfde_grid(8192, 15, 0.0, 1.0, 0.0, 1.0)
    assert lib.rsfde_setup(C.byref(h), C.byref(big), 1.5, 1.5, 1, 1, fake, 1e-6, .1, 20, None) == -7
    # the allocation-free product validates on the host, before any device call
    lib.rsfde_matvec_noalloc.argtypes = [C.POINTER(rsfde_grid), C.c_double, C.c_double, C.c_double,
                                         C.c_double, P, C.c_double, C.c_double, P, P, P]
    mv = lib.rsfde_matvec_noalloc
    assert mv(None, 1.5, 1.5, 1, 1, fake, 1e-6, .1, fake, P(0x2000), None) == -1
    assert mv(C.byref(g), 1.5, 1.5, 1, 1, None, 1e-6, .1, fake, P(0x2000), None) == -1
    assert mv(C.byref(g), 1.5, 1.5, 1, 1, fake, 1e-6, .1, fake, fake, None) == -1   # x == y
    assert mv(C.byref(g), 2.5, 1.5, 1, 1, fake, 1e-6, .1, fake, P(0x2000), None) == -1
    assert mv(C.byref(g), 1.5, 1.5, 1, 1, fake, 0.0, .1, fake, P(0x2000), None) == -1
    assert mv(C.byref(bad), 1.5, 1.5, 1, 1, fake, 1e-6, .1, fake, P(0x2000), None) == -1
    over = rsfde_grid(2048, 15, 0.0, 1.0, 0.0, 1.0)
    assert mv(C.byref(over), 1.5, 1.5, 1, 1, fake, 1e-6, .1, fake, P(0x2000), None) == -7
    # batched solves: host validation before any device call
    DP = C.POINTER(C.c_double)
    lib.rsfde_batch_setup.argtypes = [C.POINTER(P), C.POINTER(rsfde_grid), C.c_double, C.c_double,
                                      C.c_int32, DP, DP, P, C.c_double, C.c_double, C.c_int32, P]
    ks = (C.c_double * 40)(*([1.0] * 40))
    kneg = (C.c_double * 2)(1.0, -1.0)
    bs = lib.rsfde_batch_setup
    assert bs(None, C.byref(g), 1.5, 1.5, 2, ks, ks, fake, 1e-6, .1, 20, None) == -1
    assert bs(C.byref(h), C.byref(g), 1.5, 1.5, 0, ks, ks, fake, 1e-6, .1, 20, None) == -1
    assert bs(C.byref(h), C.byref(g), 1.5, 1.5, 33, ks, ks, fake, 1e-6, .1, 20, None) == -7
    assert bs(C.byref(h), C.byref(g), 1.5, 1.5, 2, ks, kneg, fake, 1e-6, .1, 20, None) == -1
    assert bs(C.byref(h), C.byref(g), 1.5, 1.5, 2, None, ks, fake, 1e-6, .1, 20, None) == -1
    g30 = rsfde_grid(30, 15, 0.0, 1.0, 0.0, 1.0)  # n1 + 1 not a power of two
    assert bs(C.byref(h), C.byref(g30), 1.5, 1.5, 2, ks, ks, fake, 1e-6, .1, 20, None) == -7
    assert h.value is None
    for fn, args in (("rsfde_batch_matvec", (None, fake, fake, None)),
                     ("rsfde_batch_precond_apply", (None, fake, fake, 0, None))):
        getattr(lib, fn).argtypes = [P] * 3 + ([C.c_int32] if "precond" in fn else []) + [P]
        assert getattr(lib, fn)(*args) == -1
    # calls on a NULL plan
    lib.rsfde_matvec.argtypes = [P, P, P, P]
    assert lib.rsfde_matvec(None, fake, fake, None) == -1
    lib.rsfde_set_coeffs.argtypes = [P, C.c_double, C.c_double]
    assert lib.rsfde_set_coeffs(None, 1.0, 1.0) == -1
    lib.rsfde_precond_apply.argtypes = [P, P, P, C.c_int32, P]
    assert lib.rsfde_precond_apply(None, fake, fake, 0, None) == -1
    st = rsfde_stats()
    o = rsfde_solver_opts(20, 100, 1e-8, 0, 0)
    lib.rsfde_step.argtypes = [P, P, P, C.c_int32, C.POINTER(rsfde_solver_opts), P,
                               C.POINTER(rsfde_stats), P]
    assert lib.rsfde_step(None, fake, None, 1, C.byref(o), fake, C.byref(st), None) == -1
    assert st.status == -1
    lib.rsfde_destroy.argtypes = [P]
    assert lib.rsfde_destroy(None) == 0


def test_fft_engine_selftest():
    from paper_2102_11576_amd.build import build_selftest
    exe = build_selftest()
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout


def test_new_entry_points_validate_on_the_host(lib):
    """rsfde_step_src and rsfde_march_ensemble reject bad arguments before any
    device work (no GPU needed): NULL plans, empty ensembles, NULL arrays."""
    from paper_2102_11576_amd._lib import rsfde_solver_opts, rsfde_stats
    P = C.c_void_p
    fake = C.c_void_p(0x1000)
    st = rsfde_stats()
    o = rsfde_solver_opts(20, 100, 1e-8, 0, 0, 0, 0, 0)
    lib.rsfde_step_src.argtypes = [P, P, P, C.c_int32, P, C.c_double,
                                   C.POINTER(rsfde_solver_opts), P, C.POINTER(rsfde_stats), P]
    assert lib.rsfde_step_src(None, fake, None, 4, fake, 1.0, C.byref(o), fake, C.byref(st),
                              None) == -1
    assert st.status == -1
    PP = C.POINTER(C.c_void_p)
    lib.rsfde_march_ensemble.argtypes = [C.c_int32, PP, PP, C.c_int32, C.c_int32,
                                         C.POINTER(rsfde_solver_opts), PP, PP,
                                         C.POINTER(rsfde_stats), PP]
    arr = (C.c_void_p * 2)(0x1000, 0x2000)
    assert lib.rsfde_march_ensemble(0, arr, arr, 1, 0, C.byref(o), arr, arr, None, None) == -1
    assert lib.rsfde_march_ensemble(1, None, arr, 1, 0, C.byref(o), arr, arr, None, None) == -1
    assert lib.rsfde_march_ensemble(1, arr, arr, -1, 0, C.byref(o), arr, arr, None, None) == -1
    assert lib.rsfde_march_ensemble(1, arr, arr, 1, 9, C.byref(o), arr, arr, None, None) == -1
    nul = (C.c_void_p * 2)(None, None)
    assert lib.rsfde_march_ensemble(1, nul, arr, 1, 0, C.byref(o), arr, arr, None, None) == -1


def test_setup3_host_validation_fails_fast(lib):
    from paper_2102_11576_amd._lib import rsfde_grid3
    P = C.c_void_p
    lib.rsfde_setup3.argtypes = [C.POINTER(P), C.POINTER(rsfde_grid3), C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_double, P, C.c_double,
                                 C.c_double, C.c_int32, P]
    h = P()
    fake = P(0x1000)  # never dereferenced: validation rejects first
    box = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    g = rsfde_grid3(15, 7, 31, *box)
    args = (1.5, 1.6, 1.7, 1.0, 1.0, 1.0)

    def call(grid=C.byref(g), a=args, mask=fake, eta=1e-6, dt=0.1, mr=20, out=C.byref(h)):
        return lib.rsfde_setup3(out, grid, *a, mask, eta, dt, mr, None)

    assert call(out=None) == -1
    assert call(grid=None) == -1
    assert call(mask=None) == -1
    assert call(eta=0.0) == -1
    assert call(dt=float("inf")) == -1
    assert call(mr=65) == -1
    for a in ((1.5, 1.6, 2.0, 1, 1, 1), (1.0, 1.6, 1.7, 1, 1, 1), (1.5, 1.6, 1.7, 1, 1, -1.0),
              (1.5, 1.6, 1.7, 1, float("nan"), 1)):
        assert call(a=a) == -1, a
    assert call(grid=C.byref(rsfde_grid3(15, 7, 0, *box))) == -1
    assert call(grid=C.byref(rsfde_grid3(15, 7, 31, 0.0, 1.0, 0.0, 1.0, 1.0, 1.0))) == -1
    # at most 4095 points per axis
    assert call(grid=C.byref(rsfde_grid3(8191, 7, 7, *box))) == -7
    assert h.value is None
    lib.rsfde_set_coeffs3.argtypes = [P, C.c_double, C.c_double, C.c_double]
    assert lib.rsfde_set_coeffs3(None, 1.0, 1.0, 1.0) == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and a
    message saying so (before touching any device)."""
    import json
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2, r.stderr[-2000:]
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]

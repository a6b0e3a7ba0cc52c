"""ctypes binding of librsfde.so (include/rsfde.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions keep the C names and take torch tensors (FP64 / uint8,
contiguous, on the GPU) or raw device pointers.  Importing this module fails
loudly if the library has not been built; there is no CPU fallback.
RSFDE_LIBRARY names another build of the same library to load instead (the
build whose host code carries the address and undefined-behaviour sanitizers).
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RSFDE_LIBRARY") or os.path.join(_HERE, "librsfde.so")

RSFDE_OK = 0
RSFDE_EINVAL = -1
RSFDE_ENOMEM = -2
RSFDE_EHIP = -3
RSFDE_ENOTCONV = -4
RSFDE_EBREAKDOWN = -5
RSFDE_ENONFINITE = -6
RSFDE_EUNSUPPORTED = -7

RSFDE_FP64, RSFDE_FP32, RSFDE_BF16 = 0, 1, 2
RSFDE_PRECOND_TAU, RSFDE_PRECOND_NONE = 0, 1
RSFDE_F_NONE, RSFDE_F_LOGISTIC, RSFDE_F_SIN, RSFDE_F_CUBIC, RSFDE_F_DECAY = 0, 1, 2, 3, 4
RSFDE_RIGHT, RSFDE_LEFT = 0, 1
RSFDE_ZSTORE_FP64, RSFDE_ZSTORE_FP32 = 0, 1

PRECISIONS = {"fp64": RSFDE_FP64, "fp32": RSFDE_FP32, "bf16": RSFDE_BF16}


class rsfde_grid(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32),
                ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("y_lo", C.c_double), ("y_hi", C.c_double)]


class rsfde_grid3(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32),
                ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("y_lo", C.c_double), ("y_hi", C.c_double),
                ("z_lo", C.c_double), ("z_hi", C.c_double)]


class rsfde_solver_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iters", C.c_int32), ("tol", C.c_double),
                ("precision", C.c_int32), ("precond", C.c_int32), ("reorth", C.c_int32),
                ("side", C.c_int32), ("sstep", C.c_int32), ("zstore", C.c_int32)]


class rsfde_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("relres", C.c_double), ("bnorm", C.c_double)]


class rsfde_kernel_profile(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("bytes", C.c_double)]


class RsfdeError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the HIP library is required; there is no fallback)")
    # torch first: the library then binds to the HIP runtime that torch has
    # loaded, and both see one device context.  Loaded before torch, it pulls
    # in the system HIP runtime as a second copy in the process, which finds
    # no device once torch's copy holds it.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.rsfde_setup.argtypes = [C.POINTER(P), C.POINTER(rsfde_grid), C.c_double, C.c_double,
                                C.c_double, C.c_double, P, C.c_double, C.c_double, C.c_int32, P]
    lib.rsfde_setup3.argtypes = [C.POINTER(P), C.POINTER(rsfde_grid3), C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_double, P, C.c_double,
                                 C.c_double, C.c_int32, P]
    lib.rsfde_set_coeffs.argtypes = [P, C.c_double, C.c_double]
    lib.rsfde_set_coeffs3.argtypes = [P, C.c_double, C.c_double, C.c_double]
    lib.rsfde_matvec.argtypes = [P, P, P, P]
    lib.rsfde_matvec_noalloc.argtypes = [C.POINTER(rsfde_grid), C.c_double, C.c_double, C.c_double,
                                         C.c_double, P, C.c_double, C.c_double, P, P, P]
    lib.rsfde_precond_apply.argtypes = [P, P, P, C.c_int32, P]
    lib.rsfde_step.argtypes = [P, P, P, C.c_int32, C.POINTER(rsfde_solver_opts), P,
                               C.POINTER(rsfde_stats), P]
    lib.rsfde_step_src.argtypes = [P, P, P, C.c_int32, P, C.c_double,
                                   C.POINTER(rsfde_solver_opts), P, C.POINTER(rsfde_stats), P]
    lib.rsfde_solve.argtypes = [P, P, P, C.POINTER(rsfde_solver_opts), C.POINTER(rsfde_stats), P]
    lib.rsfde_adjoint_step.argtypes = [P, P, P, P, C.c_int32, C.POINTER(rsfde_solver_opts), P, P,
                                       P, C.POINTER(rsfde_stats), P]
    PP = C.POINTER(C.c_void_p)
    lib.rsfde_march_ensemble.argtypes = [C.c_int32, PP, PP, C.c_int32, C.c_int32,
                                         C.POINTER(rsfde_solver_opts), PP, PP,
                                         C.POINTER(rsfde_stats), PP]
    DP = C.POINTER(C.c_double)
    lib.rsfde_batch_setup.argtypes = [C.POINTER(P), C.POINTER(rsfde_grid), C.c_double, C.c_double,
                                      C.c_int32, DP, DP, P, C.c_double, C.c_double, C.c_int32, P]
    lib.rsfde_batch_set_coeffs.argtypes = [P, DP, DP]
    lib.rsfde_batch_matvec.argtypes = [P, P, P, P]
    lib.rsfde_batch_precond_apply.argtypes = [P, P, P, C.c_int32, P]
    lib.rsfde_batch_step.argtypes = [P, P, P, C.c_int32, C.POINTER(rsfde_solver_opts), P,
                                     C.POINTER(rsfde_stats), P]
    lib.rsfde_batch_destroy.argtypes = [P]
    lib.rsfde_profile.argtypes = [P, C.c_int32]
    lib.rsfde_profile_read.argtypes = [P, C.POINTER(rsfde_kernel_profile), C.c_int32,
                                       C.POINTER(C.c_int32)]
    lib.rsfde_destroy.argtypes = [P]
    lib.rsfde_strerror.argtypes = [C.c_int]
    lib.rsfde_strerror.restype = C.c_char_p
    for f in ("rsfde_setup", "rsfde_setup3", "rsfde_set_coeffs", "rsfde_set_coeffs3", "rsfde_matvec",
              "rsfde_matvec_noalloc", "rsfde_precond_apply",
              "rsfde_step", "rsfde_step_src", "rsfde_solve", "rsfde_march_ensemble", "rsfde_adjoint_step", "rsfde_destroy",
              "rsfde_profile", "rsfde_profile_read", "rsfde_batch_setup", "rsfde_batch_set_coeffs",
              "rsfde_batch_matvec", "rsfde_batch_precond_apply", "rsfde_batch_step",
              "rsfde_batch_destroy"):
        getattr(lib, f).restype = C.c_int
    return lib


_lib = _load()
lib = _lib


def strerror(code: int) -> str:
    return _lib.rsfde_strerror(int(code)).decode()


def _ptr(x):
    """Device pointer of a tensor (or an int / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check_vec(t, N, name, dtype=None):
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != N:
        raise ValueError(f"{name}: expected a contiguous {dtype} GPU tensor with {N} elements, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def _raise(rc, where):
    if rc != RSFDE_OK:
        raise RsfdeError(rc, where)


DEFAULT_SSTEP = 10


def make_opts(restart=30, max_iters=10000, tol=1e-8, precision="fp64", precond="tau", reorth=0,
              side="right", sstep=None, zstore="fp64"):
    """reorth: 0 or 1 = two Gram-Schmidt passes (CGS2), -1 = one (one-vector
    form only).  side: "right" (flexible GMRES, true-residual stop) or "left"
    (the stopping rule of the paper's experiments).  sstep: 0/1 one Arnoldi
    vector per step, s >= 2 the s-step block form; None (default) picks the
    s-step form with s = 10 where it is supported (right side, sine-transform
    preconditioner in FP64 or FP32; the library itself takes the one-vector
    form on grids below 4096 unknowns) and the one-vector form elsewhere.
    zstore: "fp64" or "fp32", the storage of the flexible GMRES's preconditioned
    basis (FP32: rounded when stored; the product uses the stored vectors)."""
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    pc = {"tau": RSFDE_PRECOND_TAU, "none": RSFDE_PRECOND_NONE}[precond] \
        if isinstance(precond, str) else int(precond)
    sd = {"right": RSFDE_RIGHT, "left": RSFDE_LEFT}[side] if isinstance(side, str) else int(side)
    if sstep is None:
        ok = sd == RSFDE_RIGHT and pc == RSFDE_PRECOND_TAU and p in (RSFDE_FP64, RSFDE_FP32)
        sstep = DEFAULT_SSTEP if ok and int(restart) + 1 + DEFAULT_SSTEP <= 80 else 0
    zs = {"fp64": RSFDE_ZSTORE_FP64, "fp32": RSFDE_ZSTORE_FP32}[zstore] \
        if isinstance(zstore, str) else int(zstore)
    return rsfde_solver_opts(int(restart), int(max_iters), float(tol), p, pc, int(reorth), sd,
                             int(sstep), zs)


def rsfde_setup(n1, n2, box, alpha1, alpha2, kx, ky, mask, eta, dt, max_restart=30, stream=None):
    import torch
    _check_vec(mask, n1 * n2, "mask", torch.uint8)
    g = rsfde_grid(int(n1), int(n2), float(box[0]), float(box[1]), float(box[2]), float(box[3]))
    h = C.c_void_p()
    rc = _lib.rsfde_setup(C.byref(h), C.byref(g), float(alpha1), float(alpha2), float(kx),
                          float(ky), _ptr(mask), float(eta), float(dt), int(max_restart),
                          _stream(stream))
    _raise(rc, "rsfde_setup")
    return h


def rsfde_setup3(n, box, alphas, ks, mask, eta, dt, max_restart=30, stream=None):
    """n = (n1, n2, n3), box = (x_lo, x_hi, y_lo, y_hi, z_lo, z_hi), alphas and ks
    per axis; mask is a uint8 GPU tensor of n1*n2*n3 entries ([n3][n2][n1])."""
    import torch
    n1, n2, n3 = (int(v) for v in n)
    _check_vec(mask, n1 * n2 * n3, "mask", torch.uint8)
    g = rsfde_grid3(n1, n2, n3, *(float(v) for v in box))
    h = C.c_void_p()
    rc = _lib.rsfde_setup3(C.byref(h), C.byref(g), *(float(a) for a in alphas),
                           *(float(k) for k in ks), _ptr(mask), float(eta), float(dt),
                           int(max_restart), _stream(stream))
    _raise(rc, "rsfde_setup3")
    return h


def rsfde_set_coeffs(plan, kx, ky):
    _raise(_lib.rsfde_set_coeffs(plan, float(kx), float(ky)), "rsfde_set_coeffs")


def rsfde_set_coeffs3(plan, kx, ky, kz):
    _raise(_lib.rsfde_set_coeffs3(plan, float(kx), float(ky), float(kz)), "rsfde_set_coeffs3")


def rsfde_matvec(plan, x, y, stream=None):
    _raise(_lib.rsfde_matvec(plan, _ptr(x), _ptr(y), _stream(stream)), "rsfde_matvec")


def rsfde_matvec_noalloc(n1, n2, box, alpha1, alpha2, kx, ky, mask, eta, dt, x, y, stream=None):
    """y = M x without a plan and without any allocation (library-owned scratch
    array; n1, n2 <= 2047)."""
    g = rsfde_grid(int(n1), int(n2), float(box[0]), float(box[1]), float(box[2]), float(box[3]))
    _raise(_lib.rsfde_matvec_noalloc(C.byref(g), float(alpha1), float(alpha2), float(kx), float(ky),
                                     _ptr(mask), float(eta), float(dt), _ptr(x), _ptr(y),
                                     _stream(stream)), "rsfde_matvec_noalloc")


def rsfde_precond_apply(plan, r, z, precision=RSFDE_FP64, stream=None):
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _raise(_lib.rsfde_precond_apply(plan, _ptr(r), _ptr(z), p, _stream(stream)),
           "rsfde_precond_apply")


def rsfde_step(plan, u_prev, u_prev2, f_kind, opts, u_next, stream=None, check=True):
    st = rsfde_stats()
    rc = _lib.rsfde_step(plan, _ptr(u_prev), _ptr(u_prev2), int(f_kind), C.byref(opts),
                         _ptr(u_next), C.byref(st), _stream(stream))
    if check:
        _raise(rc, "rsfde_step")
    return st


def rsfde_step_src(plan, u_prev, u_prev2, f_kind, src, src_scale, opts, u_next, stream=None,
                   check=True):
    st = rsfde_stats()
    rc = _lib.rsfde_step_src(plan, _ptr(u_prev), _ptr(u_prev2), int(f_kind), _ptr(src),
                             float(src_scale), C.byref(opts), _ptr(u_next), C.byref(st),
                             _stream(stream))
    if check:
        _raise(rc, "rsfde_step_src")
    return st


def rsfde_solve(plan, b, x, opts, stream=None, check=True):
    st = rsfde_stats()
    rc = _lib.rsfde_solve(plan, _ptr(b), _ptr(x), C.byref(opts), C.byref(st), _stream(stream))
    if check:
        _raise(rc, "rsfde_solve")
    return st


def rsfde_adjoint_step(plan, u_prev, u_cur, lam_cur, f_kind, opts, lam_prev, mu_guess, dk,
                       stream=None, check=True):
    st = rsfde_stats()
    rc = _lib.rsfde_adjoint_step(plan, _ptr(u_prev), _ptr(u_cur), _ptr(lam_cur), int(f_kind),
                                 C.byref(opts), _ptr(lam_prev), _ptr(mu_guess), _ptr(dk),
                                 C.byref(st), _stream(stream))
    if check:
        _raise(rc, "rsfde_adjoint_step")
    return st


def rsfde_march_ensemble(plans, u0s, m, f_kind, opts, u_outs, works, streams=None, check=True):
    """plans: list of plan handles; u0s, u_outs: tensors (one per plan); works:
    2 tensors per plan; streams: None or one torch stream (or raw handle) per plan."""
    n = len(plans)
    arr = lambda xs: (C.c_void_p * len(xs))(*[_ptr(x) if not isinstance(x, C.c_void_p) else x.value  # noqa: E731
                                              for x in xs])
    hp = (C.c_void_p * n)(*[p.value if isinstance(p, C.c_void_p) else p for p in plans])
    st = (rsfde_stats * n)()
    sp = None if streams is None else (C.c_void_p * n)(*[_stream(s) for s in streams])
    rc = _lib.rsfde_march_ensemble(n, hp, arr(u0s), int(m), int(f_kind), C.byref(opts),
                                   arr(u_outs), arr(works), st, sp)
    if check:
        _raise(rc, "rsfde_march_ensemble")
    return [st[i] for i in range(n)]


def _dvec(vals):
    vals = [float(v) for v in vals]
    return (C.c_double * len(vals))(*vals)


def rsfde_batch_setup(n1, n2, box, alpha1, alpha2, kxs, kys, mask, eta, dt, max_restart=30,
                      stream=None):
    import torch
    if len(kxs) != len(kys):
        raise ValueError("one kx and one ky per member")
    _check_vec(mask, n1 * n2, "mask", torch.uint8)
    g = rsfde_grid(int(n1), int(n2), float(box[0]), float(box[1]), float(box[2]), float(box[3]))
    h = C.c_void_p()
    rc = _lib.rsfde_batch_setup(C.byref(h), C.byref(g), float(alpha1), float(alpha2), len(kxs),
                                _dvec(kxs), _dvec(kys), _ptr(mask), float(eta), float(dt),
                                int(max_restart), _stream(stream))
    _raise(rc, "rsfde_batch_setup")
    return h


def rsfde_batch_set_coeffs(batch, kxs, kys):
    _raise(_lib.rsfde_batch_set_coeffs(batch, _dvec(kxs), _dvec(kys)), "rsfde_batch_set_coeffs")


def rsfde_batch_matvec(batch, x, y, stream=None):
    _raise(_lib.rsfde_batch_matvec(batch, _ptr(x), _ptr(y), _stream(stream)), "rsfde_batch_matvec")


def rsfde_batch_precond_apply(batch, r, z, precision=RSFDE_FP64, stream=None):
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _raise(_lib.rsfde_batch_precond_apply(batch, _ptr(r), _ptr(z), p, _stream(stream)),
           "rsfde_batch_precond_apply")


def rsfde_batch_step(batch, count, u_prev, u_prev2, f_kind, opts, u_next, stream=None,
                     check=True):
    st = (rsfde_stats * count)()
    rc = _lib.rsfde_batch_step(batch, _ptr(u_prev), _ptr(u_prev2), int(f_kind), C.byref(opts),
                               _ptr(u_next), st, _stream(stream))
    if check:
        _raise(rc, "rsfde_batch_step")
    return [st[i] for i in range(count)]


def rsfde_batch_destroy(batch):
    _raise(_lib.rsfde_batch_destroy(batch), "rsfde_batch_destroy")


def rsfde_destroy(plan):
    _raise(_lib.rsfde_destroy(plan), "rsfde_destroy")


def rsfde_profile(plan, enable):
    _raise(_lib.rsfde_profile(plan, 1 if enable else 0), "rsfde_profile")


def rsfde_profile_read(plan):
    """{family: (launches, total_ms, algorithmic_bytes)} since the last read."""
    buf = (rsfde_kernel_profile * 32)()
    n = C.c_int32(0)
    _raise(_lib.rsfde_profile_read(plan, buf, 32, C.byref(n)), "rsfde_profile_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms), float(buf[i].bytes))
            for i in range(n.value)}

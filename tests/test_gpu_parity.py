"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances
----------
matvec      : |w_gpu - w_ref|_inf <= 1e-13 * ||M||_inf ||z||_inf   (FFT rounding is
              ~ eps log2(L) times that norm product; 1e-13 leaves ~40x headroom)
precond FP64: |z_gpu - z_ref|_inf <= 1e-12 * ||z_ref||_inf          (orthogonal transforms)
precond FP32: |z_gpu - z_ref|_inf <= 2e-5  * ||z_ref||_inf          (FP32 internals)
step (FP64) : ||u_gpu - u_lu||_inf <= 1e-10 ||u_lu||_inf            (the parity bound of the step)
"""

import numpy as np
import pytest
import torch

import oracle as O
from workloads.configs import make_config, domain_mask, _ellipse

pytestmark = pytest.mark.gpu

rsfde = pytest.importorskip("paper_2102_11576_amd")
from paper_2102_11576_amd import RsfdePlan, make_opts  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).reshape(-1)


def _plan(p, max_restart=30):
    return RsfdePlan(p.n1, p.n2, p.box, p.alpha1, p.alpha2, p.kx, p.ky, torch.as_tensor(p.mask),
                     p.eta, p.dt, max_restart)


def _problem(n1, n2, seed=0, name="c3"):
    w = make_config(name, n=max(n1, n2))
    box = (0.0, 1.0 * n1 / max(n1, n2) + 0.3, 0.0, 1.0)
    mask = domain_mask(n1, n2, box, _ellipse(box[1] / 2, 0.5, 0.4 * box[1], 0.35, 20.0))
    return O.Problem(n1, n2, box, w.alpha1 - 0.1 * (seed % 3), w.alpha2, 0.9, 1.3, w.eta,
                     w.T / w.m, mask)


def _norm_M_inf(p):
    tx = np.abs(p.cx * O.toeplitz_first_column(p.alpha1, p.n1))
    ty = np.abs(p.cy * O.toeplitz_first_column(p.alpha2, p.n2))
    return 1.0 + p.d + 2 * tx.sum() + 2 * ty.sum()


SHAPES = [(1, 1), (2, 3), (3, 3), (7, 5), (5, 7), (15, 15), (31, 17), (63, 63), (64, 64),
          (100, 37), (127, 127), (255, 255)]


@pytest.mark.parametrize("n1,n2", SHAPES)
def test_matvec_parity(n1, n2):
    p = _problem(n1, n2, seed=n1 + n2)
    rng = np.random.default_rng(n1 * 1000 + n2)
    Z = rng.standard_normal((n2, n1))
    ref = O.matvec(p, Z)
    with _plan(p) as pl:
        out = pl.matvec(_t(Z)).cpu().numpy().reshape(n2, n1)
    err = np.abs(out - ref).max()
    assert err <= 1e-13 * _norm_M_inf(p) * np.abs(Z).max(), err


# From n + 1 = 256 on, a direction's sine transforms take the symmetric form
# (half the FFT work); mixed shapes pair it with the plain form in the other
# direction, odd n2 leaves a half-empty last row pair.
PC_SHAPES = [(1, 1), (3, 3), (1, 7), (7, 3), (15, 15), (31, 63), (63, 63), (127, 127),
             (255, 255), (511, 255), (255, 63), (63, 255), (1023, 15), (15, 1023)]


@pytest.mark.parametrize("n1,n2", PC_SHAPES)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_precond_parity(n1, n2, precision, tol):
    p = _problem(n1, n2, seed=n1)
    rng = np.random.default_rng(7 + n1 + n2)
    V = rng.standard_normal((n2, n1))
    ref = O.precond_apply(p, V)
    with _plan(p) as pl:
        out = pl.precond(_t(V), precision=precision).cpu().numpy().reshape(n2, n1)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    assert err <= tol, err


# Rectangular grids with n1 + 1 and n2 + 1 powers of two: every Arnoldi step
# runs the preconditioner's last pass fused with the matvec row pass, with the
# strip-tiled intermediates over n1 columns (partial strips included) and an
# odd number of rows (a half-empty last row pair).
RECT = [(3, 1), (1, 3), (7, 3), (3, 15), (15, 63), (63, 7), (127, 31), (255, 15), (15, 255)]


@pytest.mark.parametrize("n1,n2", RECT)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_rectangular_matches_dense(n1, n2, precision):
    p = _problem(n1, n2, seed=n1 + 3 * n2)
    b = np.random.default_rng(n1 * 7 + n2).standard_normal(n1 * n2)
    x_ref = np.linalg.solve(O.dense_M(p), b)
    with _plan(p) as pl:
        x = torch.zeros(n1 * n2, dtype=torch.float64, device=DEV)
        x, st = pl.solve(_t(b), x, make_opts(30, 10000, 1e-12, precision=precision))
        x = x.cpu().numpy()
    r = b - O.matvec(p, x.reshape(n2, n1)).ravel()
    assert np.linalg.norm(r) <= 1.05e-12 * np.linalg.norm(b), (np.linalg.norm(r), st)
    assert np.abs(x - x_ref).max() <= 1e-10 * np.abs(x_ref).max(), st


@pytest.mark.parametrize("n1,n2", [(255, 63), (63, 511)])
def test_sstep_solve_rectangular_true_residual(n1, n2):
    """The s-step form (N >= 4096) on rectangular grids: the true residual of
    the GPU solution, measured by the oracle's operator, meets the tolerance."""
    p = _problem(n1, n2, seed=5)
    b = np.random.default_rng(n1 + n2).standard_normal(n1 * n2)
    tol = 1e-10
    with _plan(p) as pl:
        x = torch.zeros(n1 * n2, dtype=torch.float64, device=DEV)
        x, st = pl.solve(_t(b), x, make_opts(30, 10000, tol, sstep=8))
        x = x.cpu().numpy()
    r = b - O.matvec_fast(p, x.reshape(n2, n1)).ravel()
    assert np.linalg.norm(r) <= 1.05 * tol * np.linalg.norm(b), (np.linalg.norm(r), st)
    assert st.iters > 0


def test_step_matches_lu_c1():
    """Config c1 as specified (63^2, 16 steps, GMRES(20), tol 1e-10) vs dense LU."""
    w = make_config("c1")
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w) as pl:
        u, iters, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(w.restart, 10000, w.tol))
        u = u.cpu().numpy().reshape(w.n2, w.n1)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    assert err <= 1e-10, err
    assert all(i > 0 for i in iters)


@pytest.mark.parametrize("name,n,m", [("c2", 31, 3), ("c3", 31, 3), ("c4", 15, 3), ("c5", 31, 2)])
def test_step_matches_lu_small(name, n, m):
    w = make_config(name, n=n, m=m)
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w) as pl:
        u, _, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(w.restart, 10000, 1e-12))
        u = u.cpu().numpy().reshape(w.n2, w.n1)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    assert err <= 1e-10, err


@pytest.mark.parametrize("name,n", [("c1", 31), ("c3", 31), ("c2", 63)])
def test_iteration_counts_match_oracle_gmres(name, n):
    """Right-preconditioned GMRES: the GPU's inner iterations per step are within
    +-2 of the oracle's MGS GMRES on the same problem and stopping rule."""
    w = make_config(name, n=n, m=3)
    p = O.problem_from_workload(w)
    _, it_ref = O.march_gmres(p, w.u0, w.m, w.f_kind, w.restart, w.tol)
    with RsfdePlan.from_workload(w) as pl:
        _, it_gpu, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(w.restart, 10000, w.tol))
    assert all(abs(a - b) <= 2 for a, b in zip(it_gpu, it_ref)), (it_gpu, it_ref)


def test_unpreconditioned_and_nonpow2_grid():
    """n+1 not a power of two: plain GMRES and the chirp-form preconditioner both
    match LU."""
    w = make_config("c4", n=20, m=2)
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w) as pl:
        for pc in ("none", "tau"):
            u, _, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(30, 100000, 1e-12, precond=pc))
            u = u.cpu().numpy().reshape(w.n2, w.n1)
            assert np.abs(u - ref).max() / np.abs(ref).max() <= 1e-10, pc


def test_error_paths():
    w = make_config("c1", n=15, m=1)
    with RsfdePlan.from_workload(w) as pl:
        u0 = _t(w.u0)
        # iteration cap
        _, st = pl.step(u0, None, w.f_kind, make_opts(20, 1, 1e-300), check=False)
        assert st.status == rsfde._lib.RSFDE_ENOTCONV and st.iters == 1
        # non-finite input
        bad = u0.clone()
        bad[5] = float("nan")
        _, st = pl.step(bad, None, w.f_kind, make_opts(20, 100, 1e-8), check=False)
        assert st.status == rsfde._lib.RSFDE_ENONFINITE
        # zero right-hand side -> zero solution
        z = torch.zeros_like(u0)
        out, st = pl.step(z, None, w.f_kind, make_opts(20, 100, 1e-8))
        assert st.status == 0 and float(out.abs().max()) == 0.0
        # invalid options
        with pytest.raises(rsfde.RsfdeError):
            pl.step(u0, None, w.f_kind, make_opts(0, 100, 1e-8))
        with pytest.raises(rsfde.RsfdeError):
            pl.step(u0, None, 9, make_opts(20, 100, 1e-8))


def test_all_inside_and_all_outside_masks():
    for val in (0, 1):
        w = make_config("c1", n=15, m=2)
        w.mask = np.full_like(w.mask, val)
        w.u0 = np.random.default_rng(val).random(w.u0.shape)
        p = O.problem_from_workload(w)
        ref = O.march_lu(p, w.u0, w.m, w.f_kind)
        with RsfdePlan.from_workload(w) as pl:
            u, _, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(20, 1000, 1e-12))
        err = np.abs(u.cpu().numpy().reshape(15, 15) - ref).max() / np.abs(ref).max()
        assert err <= 1e-10, (val, err)


@pytest.mark.parametrize("restart", [1, 5, 33, 40, 64])
def test_long_and_short_restarts(restart):
    """Restart lengths beyond one 32-vector chunk (split multi-dot / axpy / update)
    and degenerate GMRES(1) agree with LU."""
    w = make_config("c3", n=31, m=2)
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w, max_restart=restart) as pl:
        u, iters, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(restart, 100000, 1e-12,
                                                                   precond="none"))
        u = u.cpu().numpy().reshape(w.n2, w.n1)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    assert err <= 1e-10, (restart, err, iters)


BF16_SHAPES = [(1, 1), (7, 3), (20, 33), (63, 63), (100, 130), (255, 255), (300, 129)]


@pytest.mark.parametrize("n1,n2", BF16_SHAPES)
def test_precond_bf16_mfma_close_to_fp64(n1, n2):
    """BF16-operand / FP32-accumulate sine-matrix GEMMs (any n, including sizes
    that are not 2^k - 1) against the FP64 oracle.  Each of the four products
    rounds its operands to BF16 (relative 2^-9), so the apply agrees to ~1e-2:
    the test bound is 4e-2 of ||z||_inf."""
    p = _problem(n1, n2, seed=3)
    rng = np.random.default_rng(17 + n1 * n2)
    V = rng.standard_normal((n2, n1))
    ref = O.precond_apply(p, V)
    with _plan(p) as pl:
        out = pl.precond(_t(V), precision="bf16").cpu().numpy().reshape(n2, n1)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    assert err <= 4e-2, err


@pytest.mark.parametrize("name,n,m", [("c3", 31, 2), ("c1", 20, 2), ("c5", 33, 2)])
def test_step_bf16_preconditioner_matches_lu(name, n, m):
    """Flexible GMRES with the BF16 preconditioner reaches the FP64 solution:
    the outer residual, Arnoldi and update stay FP64."""
    w = make_config(name, n=n, m=m)
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w) as pl:
        u, iters, _ = pl.march(_t(w.u0), w.m, w.f_kind,
                               make_opts(w.restart, 10000, 1e-12, precision="bf16"))
        u = u.cpu().numpy().reshape(w.n2, w.n1)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    assert err <= 1e-10, (err, iters)


@pytest.mark.parametrize("precision,reorth", [("fp64", 1), ("fp32", 1), ("bf16", -1), ("bf16", 1)])
def test_reorthogonalisation_option(precision, reorth):
    """One or two classical Gram-Schmidt passes, any preconditioner precision: the
    converged solution matches LU."""
    w = make_config("c3", n=31, m=2)
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w) as pl:
        u, iters, _ = pl.march(_t(w.u0), w.m, w.f_kind,
                               make_opts(w.restart, 10000, 1e-12, precision=precision,
                                         reorth=reorth))
        u = u.cpu().numpy().reshape(w.n2, w.n1)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    assert err <= 1e-10, (err, iters)


def test_package_imported_before_torch():
    """A script that imports the package before torch still finds the device:
    the package loads torch before the HIP library, so both use one HIP
    runtime (with the library loaded first, setup found no device)."""
    import subprocess
    import sys
    from pathlib import Path
    code = ("import paper_2102_11576_amd as m\n"
            "from workloads.configs import make_config\n"
            "w = make_config('c1')\n"
            "with m.RsfdePlan.from_workload(w) as pl:\n"
            "    print('setup ok')\n")
    root = Path(__file__).resolve().parents[1]
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0 and "setup ok" in r.stdout, r.stderr[-2000:]

"""s-step form of the right-preconditioned GMRES (opts.sstep = s >= 2) against
the dense LU oracle and against the one-vector form.

The s-step solve spans the same Krylov space and stops on the same estimates,
so on these well-conditioned blocks (s <= 8) the iteration count of every
step equals the one-vector count to within one with the FP64 preconditioner,
and the solutions meet the same bound as the one-vector solver (1e-10 against
LU at tol 1e-12).  With FP32 internals the preconditioner is a fixed linear
operator only up to FP32 rounding, which the s-step recurrence assumes, so
counts may differ by a few (bar: 3).
"""

import numpy as np
import pytest
import torch

import oracle as O
from workloads.configs import make_config

pytestmark = pytest.mark.gpu

rsfde = pytest.importorskip("paper_2102_11576_amd")
from paper_2102_11576_amd import RsfdePlan, make_opts  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).reshape(-1)


@pytest.fixture(scope="module")
def c4_71():
    w = make_config("c4", n=71, m=3)   # N = 5041: above the s-step size floor
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    return w, ref


@pytest.mark.parametrize("s", [2, 3, 5, 8])
def test_sstep_matches_lu(c4_71, s):
    w, ref = c4_71
    with RsfdePlan.from_workload(w) as pl:
        u, _, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(30, 100000, 1e-12, sstep=s))
        u = u.cpu().numpy().reshape(w.n2, w.n1)
    assert np.abs(u - ref).max() / np.abs(ref).max() <= 1e-10


@pytest.mark.parametrize("s,restart,reach", [(8, 60, 56), (16, 30, 32), (16, 48, 32)])
def test_sstep_large_coefficient_tables_match_lu(s, restart, reach):
    """Block updates whose coefficient table (nq*s + s*s doubles) outgrows the
    kernel-argument limit (448) go through the staged copy: the first such
    block starts at m = 48 for s = 8 and at m = 16 for s = 16, so a cycle
    longer than `reach` iterations updates one.  Earlier blocks pass theirs as
    arguments, so both paths run.  The c3 shape at 71^2 needs 63-88
    iterations per step at tol 1e-12 (oracle GMRES)."""
    w = make_config("c3", n=71, m=3)
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w, max_restart=64) as pl:
        u, its, _ = pl.march(_t(w.u0), w.m, w.f_kind,
                             make_opts(restart, 100000, 1e-12, sstep=s))
        u = u.cpu().numpy().reshape(w.n2, w.n1)
    assert min(its) > reach, its
    assert np.abs(u - ref).max() / np.abs(ref).max() <= 1e-10


@pytest.mark.parametrize("s,restart,precision", [(5, 30, "fp64"), (3, 7, "fp64"), (4, 30, "fp32"),
                                                 (5, 12, "fp64")])
def test_sstep_iterations_match_one_vector_form(s, restart, precision):
    w = make_config("c3", n=127, m=3)
    with RsfdePlan.from_workload(w) as pl:
        _, it1, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(restart, 100000, w.tol, precision, sstep=0))
        u, its, _ = pl.march(_t(w.u0), w.m, w.f_kind,
                             make_opts(restart, 100000, w.tol, precision, sstep=s))
    bar = 1 if precision == "fp64" else 3
    assert all(abs(a - b) <= bar for a, b in zip(it1, its)), (it1, its)


def test_sstep_options_rejected_where_unsupported():
    w = make_config("c4", n=71, m=1)
    with RsfdePlan.from_workload(w) as pl:
        for kw in (dict(side="left"), dict(precond="none")):
            with pytest.raises(rsfde.RsfdeError) as ei:
                pl.step(_t(w.u0), None, w.f_kind, make_opts(30, 100, 1e-8, sstep=5, **kw))
            assert ei.value.code == rsfde._lib.RSFDE_EUNSUPPORTED
        with pytest.raises(rsfde.RsfdeError) as ei:
            pl.step(_t(w.u0), None, w.f_kind, make_opts(30, 100, 1e-8, sstep=17))
        assert ei.value.code == rsfde._lib.RSFDE_EINVAL


@pytest.mark.parametrize("s,precision", [(5, "fp64"), (8, "fp64"), (10, "fp64"), (8, "fp32")])
def test_sstep_full_size_2047_true_residual(s, precision):
    """Two steps at 2047^2 (the benchmark workload; at this stiffness blocks are
    truncated and cycles restarted where the s-step directions become
    numerically dependent): the oracle recomputes b and the true residual of
    the GPU's second-step solution."""
    w = make_config("c3")
    p = O.problem_from_workload(w)
    opts = make_opts(w.restart, 100000, w.tol, precision, sstep=s)
    with RsfdePlan.from_workload(w) as pl:
        u0 = _t(w.u0)
        u1, _ = pl.step(u0, None, w.f_kind, opts)
        u2, st = pl.step(u1, u0, w.f_kind, opts)
        a1 = u1.cpu().numpy().reshape(w.n2, w.n1)
        a2 = u2.cpu().numpy().reshape(w.n2, w.n1)
    b = O.rhs(p, a1, w.f_kind)
    r = b - O.matvec_fast(p, a2)
    assert np.linalg.norm(r) <= (w.tol + 1e-12) * np.linalg.norm(b)
    assert st.relres <= w.tol
    assert 40 < st.iters < 300


def test_sstep_iteration_cap_and_nonfinite_input():
    w = make_config("c4", n=71, m=1)
    with RsfdePlan.from_workload(w) as pl:
        u0 = _t(w.u0)
        _, st = pl.step(u0, None, w.f_kind, make_opts(30, 5, 1e-14, sstep=4), check=False)
        assert st.status == rsfde._lib.RSFDE_ENOTCONV and st.iters == 5
        bad = u0.clone()
        bad[17] = float("nan")
        _, st = pl.step(bad, None, w.f_kind, make_opts(30, 100, 1e-8, sstep=4), check=False)
        assert st.status == rsfde._lib.RSFDE_ENONFINITE


@pytest.mark.parametrize("s,precision", [(0, "fp64"), (8, "fp64"), (0, "fp32"), (8, "fp32")])
def test_fp32_basis_storage_matches_dense_solve(s, precision):
    """The preconditioned basis kept in FP32 (zstore): each z_j is rounded when
    stored and M z_j is formed from the stored vector, so the flexible GMRES
    still stops on the FP64 true residual and meets the dense solution's bar.
    127 x 63 (n + 1 powers of two, the fused pass; 8001 unknowns, above the
    s-step floor), the c4 orders on an ellipse."""
    from workloads.configs import domain_mask, _ellipse
    w = make_config("c4", n=127)
    box = (0.0, 1.0, 0.0, 0.5)
    mask = domain_mask(127, 63, box, _ellipse(0.5, 0.25, 0.4, 0.2, 10.0))
    p = O.Problem(127, 63, box, w.alpha1, w.alpha2, 1.1, 0.8, w.eta, 1.0 / 32, mask)
    b = np.random.default_rng(s + 3).standard_normal(p.n1 * p.n2)
    x_ref = np.linalg.solve(O.dense_M(p), b)
    with RsfdePlan(p.n1, p.n2, p.box, p.alpha1, p.alpha2, p.kx, p.ky, torch.as_tensor(p.mask),
                   p.eta, p.dt) as pl:
        x = torch.zeros(p.n1 * p.n2, dtype=torch.float64, device=DEV)
        x, st = pl.solve(_t(b), x, make_opts(30, 100000, 1e-12, precision, sstep=s, zstore="fp32"))
        x = x.cpu().numpy()
    r = b - O.matvec(p, x.reshape(p.n2, p.n1)).ravel()
    assert np.linalg.norm(r) <= 1.05e-12 * np.linalg.norm(b), st
    assert np.abs(x - x_ref).max() <= 1e-10 * np.abs(x_ref).max(), st


@pytest.mark.parametrize("s", [0, 10])
def test_fp32_basis_storage_full_size_2047(s):
    """Two steps at 2047^2 with the basis in FP32: the oracle recomputes the
    second step's true residual."""
    w = make_config("c3")
    p = O.problem_from_workload(w)
    opts = make_opts(w.restart, 100000, w.tol, sstep=s, zstore="fp32")
    with RsfdePlan.from_workload(w) as pl:
        u0 = _t(w.u0)
        u1, _ = pl.step(u0, None, w.f_kind, opts)
        u2, st = pl.step(u1, u0, w.f_kind, opts)
        a1 = u1.cpu().numpy().reshape(w.n2, w.n1)
        a2 = u2.cpu().numpy().reshape(w.n2, w.n1)
    b = O.rhs(p, a1, w.f_kind)
    r = b - O.matvec_fast(p, a2)
    assert np.linalg.norm(r) <= (w.tol + 1e-12) * np.linalg.norm(b)
    assert st.relres <= w.tol


def test_fp32_basis_storage_rejected_where_unsupported():
    w = make_config("c4", n=71, m=1)
    with RsfdePlan.from_workload(w) as pl:
        for kw in (dict(side="left"), dict(precond="none"), dict(precision="bf16")):
            with pytest.raises(rsfde.RsfdeError) as ei:
                pl.step(_t(w.u0), None, w.f_kind, make_opts(30, 100, 1e-8, zstore="fp32", **kw))
            assert ei.value.code == rsfde._lib.RSFDE_EUNSUPPORTED
    w2 = make_config("c4", n=70, m=1)   # n + 1 not a power of two: no fused pass
    with RsfdePlan.from_workload(w2) as pl:
        with pytest.raises(rsfde.RsfdeError) as ei:
            pl.step(_t(w2.u0), None, w2.f_kind, make_opts(30, 100, 1e-8, zstore="fp32"))
        assert ei.value.code == rsfde._lib.RSFDE_EUNSUPPORTED

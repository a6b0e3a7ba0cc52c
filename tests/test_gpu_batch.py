"""Batched independent solves (rsfde_batch_*): every member against the oracle.

* operators: each member's M z and P_hat^{-1} v (its own kx, ky) against the
  oracle's forms for that member, with the bars of the single-plan tests
  (matvec 1e-13 ||M||_inf ||z||_inf; preconditioner element-wise per region);
* steps: each member's march against the dense-LU march of its own problem
  (31^2, tol 1e-12: 1e-10 relative), and at 511^2 (the differentiation
  workload's grid) each member's true residual recomputed by the oracle
  (<= (tol + 1e-12) ||b||);
* the batch takes the same decisions as the single plan's one-vector form:
  per-step iteration counts equal member by member;
* members that stop at different steps, a zero right-hand side and a
  non-finite input in one member leave the others' results intact.
"""

import numpy as np
import pytest
import torch

import oracle as O
from workloads.configs import make_config, fd_direction
from bars import assert_precond

pytestmark = pytest.mark.gpu

rsfde = pytest.importorskip("paper_2102_11576_amd")
from paper_2102_11576_amd import RsfdeBatch, RsfdePlan, make_opts  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).reshape(-1)


def _norm_M_inf(p):
    tx = np.abs(p.cx * O.toeplitz_first_column(p.alpha1, p.n1))
    ty = np.abs(p.cy * O.toeplitz_first_column(p.alpha2, p.n2))
    return 1.0 + p.d + 2 * tx.sum() + 2 * ty.sum()


def _members(w, B, seed=0):
    """Per-member (kx, ky, u0) of a workload: coefficients spread around the
    workload's, initial fields perturbed along seeded directions."""
    kxs = [w.kx * (0.6 + 0.15 * i) for i in range(B)]
    kys = [w.ky * (1.3 - 0.1 * i) for i in range(B)]
    u0s = []
    for i in range(B):
        du, _, _ = fd_direction(w.u0.shape, seed + i)
        u0s.append(w.u0 + 0.05 * np.sqrt(w.N) * du * w.mask)
    return kxs, kys, u0s


@pytest.mark.parametrize("name,n1,n2,B", [("c1", 63, 63, 3), ("c3", 127, 31, 4), ("c4", 255, 255, 2)])
def test_batched_operators_match_oracle(name, n1, n2, B):
    w = make_config(name, n=max(n1, n2))
    w.n1, w.n2 = n1, n2
    from workloads.configs import domain_mask, _ellipse
    w.mask = domain_mask(n1, n2, w.box, _ellipse(0.5, 0.5, 0.4, 0.3, 15.0))
    kxs = [w.kx * (0.6 + 0.15 * i) for i in range(B)]
    kys = [w.ky * (1.3 - 0.1 * i) for i in range(B)]
    rng = np.random.default_rng(n1 + B)
    Z = [rng.standard_normal((n2, n1)) for _ in range(B)]
    with RsfdeBatch(n1, n2, w.box, w.alpha1, w.alpha2, kxs, kys, torch.as_tensor(w.mask), w.eta,
                    w.T / w.m) as bt:
        x = _t(np.stack(Z))
        y = bt.matvec(x).cpu().numpy().reshape(B, n2, n1)
        z64 = bt.precond(x, precision="fp64").cpu().numpy().reshape(B, n2, n1)
        z32 = bt.precond(x, precision="fp32").cpu().numpy().reshape(B, n2, n1)
    for i in range(B):
        p = O.Problem(n1, n2, w.box, w.alpha1, w.alpha2, kxs[i], kys[i], w.eta, w.T / w.m, w.mask)
        ref = O.matvec(p, Z[i])
        assert np.abs(y[i] - ref).max() <= 1e-13 * _norm_M_inf(p) * np.abs(Z[i]).max(), i
        zref = O.precond_apply(p, Z[i])
        assert_precond(z64[i], zref, p, "fp64", f"member {i} fp64")
        assert_precond(z32[i], zref, p, "fp32", f"member {i} fp32")


def test_batched_march_matches_lu_per_member():
    w = make_config("c4", n=31, m=4)
    B = 5
    kxs, kys, u0s = _members(w, B)
    opts = make_opts(w.restart, 100000, 1e-12, sstep=0)
    with RsfdeBatch.from_workload(w, kxs, kys) as bt:
        u, iters = bt.march(_t(np.stack(u0s)), w.m, w.f_kind, opts)
        u = u.cpu().numpy().reshape(B, w.n2, w.n1)
    for i in range(B):
        p = O.problem_from_workload(w, kxs[i], kys[i])
        ref = O.march_lu(p, u0s[i], w.m, w.f_kind)
        assert np.abs(u[i] - ref).max() <= 1e-10 * np.abs(ref).max(), (i, iters)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_steps_equal_single_plan_steps(precision):
    """Same kernels, same order of operations: each member's iteration count
    per step equals the single plan's (one-vector form, two Gram-Schmidt
    passes), and the solutions agree to rounding."""
    w = make_config("c3", n=63, m=3)
    B = 4
    kxs, kys, u0s = _members(w, B, seed=7)
    opts = make_opts(w.restart, 100000, w.tol, precision, sstep=0)
    with RsfdeBatch.from_workload(w, kxs, kys) as bt:
        ub, itb = bt.march(_t(np.stack(u0s)), w.m, w.f_kind, opts)
        ub = ub.cpu().numpy().reshape(B, w.n2, w.n1)
    for i in range(B):
        with RsfdePlan.from_workload(w, kx=kxs[i], ky=kys[i]) as pl:
            us, its, _ = pl.march(_t(u0s[i]), w.m, w.f_kind, opts)
            us = us.cpu().numpy().reshape(w.n2, w.n1)
        assert [row[i] for row in itb] == its, (i, itb, its)
        assert np.abs(ub[i] - us).max() <= 1e-12 * np.abs(us).max(), i


def test_batched_full_grid_true_residuals():
    """The 511^2 differentiation-workload grid, 4 members: the oracle recomputes
    each member's b and its true residual b - M u."""
    w = make_config("c4")
    B = 4
    kxs, kys, u0s = _members(w, B, seed=3)
    opts = make_opts(w.restart, 100000, w.tol, sstep=0)
    with RsfdeBatch.from_workload(w, kxs, kys) as bt:
        u1, sts = bt.step(_t(np.stack(u0s)), None, w.f_kind, opts)
        u1 = u1.cpu().numpy().reshape(B, w.n2, w.n1)
    for i in range(B):
        p = O.problem_from_workload(w, kxs[i], kys[i])
        b = O.rhs(p, u0s[i], w.f_kind)
        r = b - O.matvec_fast(p, u1[i])
        assert np.linalg.norm(r) <= (w.tol + 1e-12) * np.linalg.norm(b), (i, sts[i])
        assert sts[i].status == 0 and sts[i].iters > 0


def test_batched_member_statuses():
    """Members that stop at different steps (different stiffness), one with a
    zero right-hand side and one with a non-finite value: each gets its own
    status, and the converged members match their LU solutions."""
    w = make_config("c1", n=31, m=1)
    B = 4
    kxs = [0.01, 1.0, 3.0, 1.0]
    kys = [0.01, 1.0, 3.0, 1.0]
    u0s = [w.u0, w.u0, np.zeros_like(w.u0), w.u0.copy()]
    u0s[3][5, 7] = np.nan
    opts = make_opts(w.restart, 100000, 1e-12, sstep=0)
    with RsfdeBatch.from_workload(w, kxs, kys) as bt:
        u1, sts = bt.step(_t(np.stack(u0s)), None, w.f_kind, opts, check=False)
        u1 = u1.cpu().numpy().reshape(B, w.n2, w.n1)
    assert sts[0].iters < sts[1].iters
    assert sts[2].status == 0 and sts[2].iters == 0 and np.abs(u1[2]).max() == 0.0
    assert sts[3].status == rsfde._lib.RSFDE_ENONFINITE
    for i in (0, 1):
        p = O.problem_from_workload(w, kxs[i], kys[i])
        ref = O.march_lu(p, u0s[i], 1, w.f_kind)
        assert sts[i].status == 0
        assert np.abs(u1[i] - ref).max() <= 1e-10 * np.abs(ref).max(), i


def test_batch_options_and_shapes_rejected():
    w = make_config("c4", n=31, m=1)
    with pytest.raises(rsfde.RsfdeError) as ei:   # n + 1 not a power of two
        RsfdeBatch(30, 30, w.box, w.alpha1, w.alpha2, [1.0], [1.0],
                   torch.ones(900, dtype=torch.uint8), w.eta, 0.1)
    assert ei.value.code == rsfde._lib.RSFDE_EUNSUPPORTED
    with RsfdeBatch.from_workload(w, [1.0, 2.0], [1.0, 1.0]) as bt:
        u = _t(np.stack([w.u0, w.u0]))
        for kw in (dict(side="left"), dict(precision="bf16"), dict(precond="none")):
            with pytest.raises(rsfde.RsfdeError) as ei:
                bt.step(u, None, w.f_kind, make_opts(30, 100, 1e-8, sstep=0, **kw))
            assert ei.value.code == rsfde._lib.RSFDE_EUNSUPPORTED

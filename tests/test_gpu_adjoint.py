"""GPU parity of the adjoint (differentiation) path.

* gradients of L = ||u(T) - u_tgt||^2 w.r.t. (u0, kx, ky) from RsfdeMarch
  (HIP forward + adjoint GMRES, sqrt(m) checkpointing) against the oracle's
  dense-LU adjoint: relative error <= 1e-8 (solves at tol 1e-12 or below),
  in the one-vector GMRES form (grids below 4096 unknowns always take it) and
  in the s-step form (71^2 = 5041 unknowns, s = 8 and 10, forward and adjoint
  solves both in blocks);
* the 511^2 differentiation workload (disk r=0.4, alpha=(1.3,1.6), 32 steps,
  u_tgt from kx=1.2, ky=0.8): central finite differences, h = 1e-6, on 16
  seeded directions, relative agreement <= 1e-5 (FD noise ~ tol/h = 1e-6),
  in both GMRES forms (the s-step form with s = 10 is the one the benchmark
  times).
"""

import numpy as np
import pytest
import torch

import oracle as O
from workloads.configs import make_config, fd_direction

pytestmark = pytest.mark.gpu

rsfde = pytest.importorskip("paper_2102_11576_amd")
from paper_2102_11576_amd import RsfdePlan, make_opts  # noqa: E402
from paper_2102_11576_amd.autograd import RsfdeMarch  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).reshape(-1)


@pytest.mark.parametrize("name,n,m,every", [("c4", 15, 4, 0), ("c3", 15, 5, 2), ("c5", 15, 3, 1),
                                            ("c1", 31, 6, 0)])
def test_adjoint_matches_oracle(name, n, m, every):
    w = make_config(name, n=n, m=m)
    w.u0 = w.u0 + 0.3 * w.mask
    rng = np.random.default_rng(5)
    u_tgt = 0.1 * rng.standard_normal(w.u0.shape)
    kx, ky = 0.9, 1.2
    L_ref, g0_ref, gkx_ref, gky_ref = O.loss_and_grads_lu(w, u_tgt, kx, ky)
    opts = make_opts(w.restart, 100000, 1e-13)
    with RsfdePlan.from_workload(w, kx=kx, ky=ky) as pl:
        u0 = _t(w.u0).requires_grad_(True)
        tkx = torch.tensor(kx, dtype=torch.float64, device=DEV, requires_grad=True)
        tky = torch.tensor(ky, dtype=torch.float64, device=DEV, requires_grad=True)
        uT = RsfdeMarch.apply(u0, tkx, tky, pl, w.m, w.f_kind, opts, every)
        L = ((uT - _t(u_tgt)) ** 2).sum()
        L.backward()
    assert float(L.detach()) == pytest.approx(L_ref, rel=1e-10)
    g0 = u0.grad.cpu().numpy().reshape(w.n2, w.n1)
    assert np.abs(g0 - g0_ref).max() <= 1e-8 * np.abs(g0_ref).max()
    assert float(tkx.grad) == pytest.approx(gkx_ref, rel=1e-8)
    assert float(tky.grad) == pytest.approx(gky_ref, rel=1e-8)


@pytest.mark.parametrize("sstep", [8, 10])
def test_sstep_adjoint_matches_oracle(sstep):
    """Forward and adjoint solves in s-step blocks (71^2: above the 4096-unknown
    floor of the block form), checkpoint segments of 2 steps, against the
    oracle's dense-LU adjoint of the same march."""
    w = make_config("c4", n=71, m=4)
    w.u0 = w.u0 + 0.3 * w.mask
    assert w.N >= 4096
    rng = np.random.default_rng(11)
    u_tgt = 0.1 * rng.standard_normal(w.u0.shape)
    kx, ky = 1.1, 0.8
    L_ref, g0_ref, gkx_ref, gky_ref = O.loss_and_grads_lu(w, u_tgt, kx, ky)
    opts = make_opts(w.restart, 100000, 1e-12, sstep=sstep)
    with RsfdePlan.from_workload(w, kx=kx, ky=ky) as pl:
        u0 = _t(w.u0).requires_grad_(True)
        tkx = torch.tensor(kx, dtype=torch.float64, device=DEV, requires_grad=True)
        tky = torch.tensor(ky, dtype=torch.float64, device=DEV, requires_grad=True)
        uT = RsfdeMarch.apply(u0, tkx, tky, pl, w.m, w.f_kind, opts, 2)
        L = ((uT - _t(u_tgt)) ** 2).sum()
        L.backward()
    assert float(L.detach()) == pytest.approx(L_ref, rel=1e-10)
    g0 = u0.grad.cpu().numpy().reshape(w.n2, w.n1)
    assert np.abs(g0 - g0_ref).max() <= 1e-8 * np.abs(g0_ref).max()
    assert float(tkx.grad) == pytest.approx(gkx_ref, rel=1e-8)
    assert float(tky.grad) == pytest.approx(gky_ref, rel=1e-8)


def test_adjoint_dot_product_identity():
    """<M^{-1} a, c> = <a, M^{-1} c> through rsfde_solve (M symmetric)."""
    w = make_config("c4", n=63, m=4)
    rng = np.random.default_rng(0)
    a, c = _t(rng.standard_normal(w.N)), _t(rng.standard_normal(w.N))
    opts = make_opts(30, 100000, 1e-13)
    with RsfdePlan.from_workload(w) as pl:
        xa, _ = pl.solve(a, torch.zeros_like(a), opts)
        xc, _ = pl.solve(c, torch.zeros_like(c), opts)
    l, r = float(torch.dot(xa, c)), float(torch.dot(a, xc))
    assert l == pytest.approx(r, rel=1e-10)


@pytest.mark.parametrize("sstep", [0, 10])
def test_fd_check_differentiation_workload(sstep):
    w = make_config("c4")                      # 511^2, 32 steps
    opts = make_opts(w.restart, 100000, 1e-12, sstep=sstep)
    kx0, ky0 = w.kx, w.ky
    with RsfdePlan.from_workload(w) as pl:
        u0 = _t(w.u0)
        # target from the same u0 marched at the target coefficients
        pl.set_coeffs(*w.extra["target_k"])
        u_tgt, _, _ = pl.march(u0, w.m, w.f_kind, opts)
        u_tgt = u_tgt.clone()

        def loss(uu0, kx, ky):
            pl.set_coeffs(kx, ky)
            uT, _, _ = pl.march(uu0, w.m, w.f_kind, opts)
            return float(((uT - u_tgt) ** 2).sum())

        x0 = u0.clone().requires_grad_(True)
        tkx = torch.tensor(kx0, dtype=torch.float64, device=DEV, requires_grad=True)
        tky = torch.tensor(ky0, dtype=torch.float64, device=DEV, requires_grad=True)
        uT = RsfdeMarch.apply(x0, tkx, tky, pl, w.m, w.f_kind, opts)
        ((uT - u_tgt) ** 2).sum().backward()
        g0, gkx, gky = x0.grad, float(tkx.grad), float(tky.grad)
        h = w.extra["fd_h"]
        worst = 0.0
        for i in range(w.extra["fd_dirs"]):
            du, dkx, dky = fd_direction(w.u0.shape, i)
            dut = _t(du)
            Lp = loss(u0 + h * dut, kx0 + h * dkx, ky0 + h * dky)
            Lm = loss(u0 - h * dut, kx0 - h * dkx, ky0 - h * dky)
            fd = (Lp - Lm) / (2 * h)
            an = float(torch.dot(g0, dut)) + gkx * dkx + gky * dky
            worst = max(worst, abs(fd - an) / max(abs(an), 1e-300))
    assert worst <= 1e-5, worst


def test_c5_adjoint_on_two_steps():
    """The 4095^2 hexagon configuration's backward pass (FP32 preconditioner
    in forward and adjoint solves, f = u - u^3, L = ||u(T)||^2) on its first
    two steps: the gradient against central differences on one seeded
    direction.  tol 1e-10 (the true residual's FP64 rounding floor at this
    stiffness is near 5e-11) and h = 1e-4: FD noise ~ 2 tol / h = 2e-6
    relative; bar 1e-4."""
    w = make_config("c5", m=2)
    opts = make_opts(w.restart, 100000, 1e-10, "fp32", sstep=0)
    with RsfdePlan.from_workload(w) as pl:
        u0 = _t(w.u0)
        x0 = u0.clone().requires_grad_(True)
        tkx = torch.tensor(w.kx, dtype=torch.float64, device=DEV, requires_grad=True)
        tky = torch.tensor(w.ky, dtype=torch.float64, device=DEV, requires_grad=True)
        uT = RsfdeMarch.apply(x0, tkx, tky, pl, w.m, w.f_kind, opts)
        (uT * uT).sum().backward()
        g0, gkx, gky = x0.grad, float(tkx.grad), float(tky.grad)

        def loss(uu0, kx, ky):
            pl.set_coeffs(kx, ky)
            u, _, _ = pl.march(uu0, w.m, w.f_kind, opts)
            return float((u * u).sum())

        du, dkx, dky = fd_direction(w.u0.shape, 0)
        dut = _t(du)
        h = 1e-4
        fd = (loss(u0 + h * dut, w.kx + h * dkx, w.ky + h * dky)
              - loss(u0 - h * dut, w.kx - h * dkx, w.ky - h * dky)) / (2 * h)
    an = float(torch.dot(g0, dut)) + gkx * dkx + gky * dky
    assert abs(fd - an) <= 1e-4 * abs(an), (fd, an)

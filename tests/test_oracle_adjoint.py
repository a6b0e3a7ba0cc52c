"""Pins of the oracle's adjoint march (O3) against central finite differences."""

import numpy as np
import pytest

import oracle as O
from workloads.configs import make_config


def test_M_symmetric_dot_product_identity():
    w = make_config("c4", n=8, m=2)
    p = O.problem_from_workload(w)
    rng = np.random.default_rng(0)
    a = rng.standard_normal((p.n2, p.n1))
    c = rng.standard_normal((p.n2, p.n1))
    assert np.sum(O.matvec(p, a) * c) == pytest.approx(np.sum(a * O.matvec(p, c)), rel=1e-13)


@pytest.mark.parametrize("name", ["c4", "c3", "c5"])
def test_adjoint_gradients_match_central_fd(name):
    w = make_config(name, n=7, m=4)
    w.u0 = w.u0 + 0.3 * w.mask  # make f'(u) non-trivial everywhere inside
    rng = np.random.default_rng(7)
    u_tgt = rng.standard_normal(w.u0.shape) * 0.1
    kx, ky = 0.9, 1.1
    L, g0, gkx, gky = O.loss_and_grads_lu(w, u_tgt, kx, ky)
    h = 1e-6
    du = rng.standard_normal(w.u0.shape)
    for (dkx, dky, dd) in ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (0.3, -0.7, 1.0)):
        Lp = O.loss_and_grads_lu(w, u_tgt, kx + h * dkx, ky + h * dky, w.u0 + h * dd * du)[0]
        Lm = O.loss_and_grads_lu(w, u_tgt, kx - h * dkx, ky - h * dky, w.u0 - h * dd * du)[0]
        fd = (Lp - Lm) / (2 * h)
        an = gkx * dkx + gky * dky + dd * np.sum(g0 * du)
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9)

"""Pins of the oracle's coefficients and matrix structure (Section 2, Lemma 2.1,
Corollary 2.1, Lemma 2.3) against closed forms and brute force."""

import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.special import binom

import oracle as O
from workloads.configs import make_config


@given(alpha=st.floats(1.01, 1.99), n=st.integers(1, 60))
@settings(max_examples=60, deadline=None)
def test_gl_weights_binomial_closed_form(alpha, n):
    # g_l = (-1)^l C(alpha, l): the generating function (1 - z)^alpha.
    g = O.gl_weights(alpha, n)
    ref = np.array([(-1) ** l * binom(alpha, l) for l in range(n + 1)])
    assert np.allclose(g, ref, rtol=1e-13, atol=1e-16)
    # partial sums sum_{l<=k} g_l = (-1)^k C(alpha-1, k)
    ps = np.cumsum(g)
    ref_ps = np.array([(-1) ** k * binom(alpha - 1.0, k) for k in range(n + 1)])
    assert np.allclose(ps, ref_ps, rtol=1e-12, atol=1e-15)


@given(alpha=st.floats(1.01, 1.99), n=st.integers(3, 80))
@settings(max_examples=60, deadline=None)
def test_lemma_2_1_properties(alpha, n):
    g = O.gl_weights(alpha, n)
    assert g[0] == 1.0
    assert g[1] == pytest.approx(-alpha, abs=1e-15)
    assert np.all(g[2:] > 0)
    assert np.all(np.diff(g[2:]) < 0)          # g_2 > g_3 > ... > 0
    assert np.all(np.cumsum(g)[1:] < 0)        # sum_{l=0}^{k} g_l < 0, k >= 1


def test_gl_sum_tends_to_zero():
    g = O.gl_weights(1.5, 200000)
    assert abs(g.sum()) < 1e-3  # partial sums ~ k^{-alpha+1}/Gamma(2-alpha) -> 0


def test_riesz_constant():
    for a in (1.1, 1.5, 1.9):
        assert O.riesz_c(a) > 0
        assert O.riesz_c(a) == pytest.approx(-0.5 / math.cos(a * math.pi / 2), rel=1e-15)
    # alpha -> 2 gives c = 1/2 (the Laplacian limit: -1/(2 cos pi))
    assert O.riesz_c(2.0 - 1e-12) == pytest.approx(0.5, rel=1e-9)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.9])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 16])
def test_G_equals_scheme_sums(alpha, n):
    """The Toeplitz matrix (G) equals the literal sums of (difference_scheme)."""
    assert np.allclose(O.G_dense(alpha, n), O.scheme_rows_bruteforce(alpha, n), rtol=0, atol=1e-14)


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.95])
def test_G_negative_definite_and_A(alpha):
    G = O.G_dense(alpha, 25)
    assert np.allclose(G, G.T)
    assert np.linalg.eigvalsh(G).max() < 0
    w = make_config("c1", n=7)
    p = O.problem_from_workload(w)
    A = O.dense_A(p)
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).max() < 0   # Corollary 2.1


def _scheme_apply_2d(p, U):
    """Left-hand side of (difference_scheme) evaluated point by point."""
    n1, n2 = p.n1, p.n2
    g1 = O.gl_weights(p.alpha1, n1 + 3)
    g2 = O.gl_weights(p.alpha2, n2 + 3)
    Z = np.zeros((n2 + 2, n1 + 2))   # with the zero boundary values (B2)
    Z[1:-1, 1:-1] = U
    out = np.zeros_like(U)
    for j in range(1, n2 + 1):
        for i in range(1, n1 + 1):
            sx = sum(g1[l] * Z[j, i - l + 1] for l in range(0, i + 2)) + \
                 sum(g1[l] * Z[j, i + l - 1] for l in range(0, n1 - i + 3))
            sy = sum(g2[l] * Z[j - l + 1, i] for l in range(0, j + 2)) + \
                 sum(g2[l] * Z[j + l - 1, i] for l in range(0, n2 - j + 3))
            dij = p.d * (1 - p.mask[j - 1, i - 1])
            out[j - 1, i - 1] = Z[j, i] - p.cx * sx - p.cy * sy + dij * Z[j, i]
    return out


def test_dense_M_and_matvec_equal_pointwise_scheme():
    """Both the Kronecker form (toeplitz_A) and the O2 matvec equal the scheme
    evaluated point by point, on a rectangular grid with alpha1 != alpha2."""
    from workloads.configs import domain_mask, _ellipse
    n1, n2 = 7, 5
    box = (0.0, 1.3, 0.0, 0.7)
    mask = domain_mask(n1, n2, box, _ellipse(0.65, 0.35, 0.6, 0.3))
    assert 0 < mask.sum() < n1 * n2
    p = O.Problem(n1, n2, box, 1.3, 1.8, 0.7, 1.9, 1e-3, 0.05, mask)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((n2, n1))
    ref = _scheme_apply_2d(p, U)
    assert np.allclose((O.dense_M(p) @ U.ravel()).reshape(n2, n1), ref, rtol=1e-13, atol=1e-12)
    assert np.allclose(O.matvec(p, U), ref, rtol=1e-13, atol=1e-12)


def test_cx_cy_values():
    w = make_config("c1", n=63)
    p = O.problem_from_workload(w)
    h = 1.0 / 64
    assert p.cx == pytest.approx((1 / 16) * 1.0 * O.riesz_c(1.5) / h ** 1.5, rel=1e-15)
    assert p.cy == pytest.approx((1 / 16) * 1.0 * O.riesz_c(1.7) / h ** 1.7, rel=1e-15)
    assert p.cx == pytest.approx(22.6, rel=2e-3)
    assert p.cy == pytest.approx(41.3, rel=2e-3)


def test_lemma_2_3_M_spd_and_dominance():
    w = make_config("c1", n=9)
    p = O.problem_from_workload(w)
    M = O.dense_M(p)
    assert np.allclose(M, M.T)
    assert np.linalg.eigvalsh(M).min() >= 1.0 - 1e-12
    off = np.abs(M).sum(axis=1) - np.abs(np.diag(M))
    assert np.all(off <= np.diag(M) - 1.0 + 1e-9)

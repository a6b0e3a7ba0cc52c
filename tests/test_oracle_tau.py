"""Pins of the tau matrix, the sine transform and the preconditioner (Section 4)."""

import numpy as np
import pytest
import scipy.fft
from hypothesis import given, settings, strategies as st

import oracle as O
from workloads.configs import make_config


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 15, 31])
def test_S_is_symmetric_orthogonal_involution(n):
    S = O.dst1_matrix(n)
    assert np.allclose(S, S.T)
    assert np.allclose(S @ S, np.eye(n), atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 5, 16, 63])
def test_S_matches_library_dst1(n):
    rng = np.random.default_rng(n)
    v = rng.standard_normal(n)
    ref = scipy.fft.dst(v, type=1, norm="ortho")
    assert np.allclose(O.dst1_matrix(n) @ v, ref, rtol=0, atol=1e-14)


@given(n=st.integers(1, 24), seed=st.integers(0, 2 ** 31 - 1))
@settings(max_examples=50, deadline=None)
def test_tau_is_diagonalised_by_S_with_closed_form_eigenvalues(n, seed):
    """tau(T) = T - H (Hankel correction) is S Lambda S, Lambda from the first column."""
    t = np.random.default_rng(seed).standard_normal(n)
    S = O.dst1_matrix(n)
    D = S @ O.tau_matrix(t) @ S
    assert np.allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-12 * max(1.0, np.abs(t).sum()))
    assert np.allclose(np.diag(D), O.tau_eigenvalues(t), atol=1e-12 * max(1.0, np.abs(t).sum()))


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
def test_lemma_4_1_tau_of_G_negative_definite(alpha):
    for n in (3, 10, 31, 64):
        lam = O.tau_eigenvalues(O.toeplitz_first_column(alpha, n))
        assert np.all(lam < 0)


def _small_problem(name="c1", n=7):
    return O.problem_from_workload(make_config(name, n=n))


@pytest.mark.parametrize("name,n", [("c1", 5), ("c3", 7), ("c5", 6)])
def test_precond_apply_equals_dense_formula(name, n):
    p = _small_problem(name, n)
    rng = np.random.default_rng(3)
    V = rng.standard_normal((p.n2, p.n1))
    z_dense = (O.precond_dense(p) @ V.ravel()).reshape(p.n2, p.n1)
    z = O.precond_apply(p, V)
    assert np.allclose(z, z_dense, rtol=1e-12, atol=1e-13 * np.abs(z_dense).max())


def test_precond_is_P_inverse_when_no_penalty_region():
    """With no penalty points P_hat^{-1} = P^{-1} = (I - tau_1(A))^{-1} exactly."""
    p = _small_problem("c1", 6)
    p.mask = np.ones_like(p.mask)
    rng = np.random.default_rng(1)
    V = rng.standard_normal((p.n2, p.n1))
    z = O.precond_apply(p, V)
    assert np.allclose((O.P_dense(p) @ z.ravel()).reshape(V.shape), V, atol=1e-10)


def test_lemma_4_3_denominators_positive():
    for name in ("c1", "c3", "c5"):
        p = _small_problem(name, 15)
        lx, ly = O.tau_eigs_xy(p)
        assert (1.0 - lx[None, :] - ly[:, None]).min() > 1.0


@pytest.mark.parametrize("name", ["c1", "c4"])
def test_lemma_4_4_and_4_5_spectra(name):
    """spec(tau_1(A)^{-1} A) and spec(P^{-1} M) lie in (1/2, 3/2)."""
    p = _small_problem(name, 9)
    A = O.dense_A(p)
    tx = p.cx * O.toeplitz_first_column(p.alpha1, p.n1)
    ty = p.cy * O.toeplitz_first_column(p.alpha2, p.n2)
    tau1 = np.kron(np.eye(p.n2), O.tau_matrix(tx)) + np.kron(O.tau_matrix(ty), np.eye(p.n1))
    ev = np.linalg.eigvals(np.linalg.solve(tau1, A)).real
    assert ev.min() > 0.5 and ev.max() < 1.5
    ev2 = np.linalg.eigvals(np.linalg.solve(O.P_dense(p), O.dense_M(p))).real
    assert ev2.min() > 0.5 and ev2.max() < 1.5


@pytest.mark.parametrize("name,n", [("c1", 9), ("c3", 16), ("c2", 5)])
def test_fast_variants_equal_dense_forms(name, n):
    p = _small_problem(name, n)
    p.n2 = p.n1  # square
    rng = np.random.default_rng(11)
    V = rng.standard_normal((p.n2, p.n1))
    assert np.allclose(O.precond_apply_fft(p, V), O.precond_apply(p, V), rtol=1e-12, atol=1e-14)
    ref = O.matvec(p, V)
    assert np.allclose(O.matvec_fast(p, V), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    for (j, i) in ((0, 0), (n - 1, 0), (n // 2, n // 3), (n - 1, n - 1)):
        assert O.matvec_entry(p, V, j, i) == pytest.approx(ref[j, i], rel=1e-12, abs=1e-12 * np.abs(ref).max())

"""Pins of the 3-D oracle (the higher-dimensional extension the paper leaves to
future work).  Each check ties it to something other than itself:

* kz = 0 decouples the z-slices: every operator and the march must reduce,
  slice by slice, to the two-dimensional oracle (pinned by its own tests
  against the paper's tables, closed forms and LU);
* permuting the array axes together with the per-axis parameters permutes the
  result (catches an operator applied along the wrong axis, a swapped
  Kronecker order or a mixed-up per-axis constant);
* the axis-wise operators equal the Kronecker-dense matrices, the direct
  Toeplitz sums and the library (FFT) forms;
* the preconditioner equals the dense formula with explicit inverses of the
  tau matrices, and inverts I - tau_1(A) exactly on an all-inside domain;
* M is symmetric with spectrum >= 1 (the 3-D form of Lemma 2.3's argument);
* GMRES on the axis-wise operators reaches the LU solution;
* the adjoint gradients (u0, kx, ky, kz) equal central finite differences of
  the LU march, and with one z-slice its x and y gradients equal the
  two-dimensional oracle's adjoint.
"""

import numpy as np
import pytest

import oracle as O
from workloads.three_d import ellipsoid_mask, make_config3d


def _p3(shape=(5, 6, 7), kz=1.0, mask=None, seed=0):
    n1, n2, n3 = shape
    if mask is None:
        mask = ellipsoid_mask(n1, n2, n3)
    return O.Problem3(n1, n2, n3, (0.0, 1.0, -0.2, 0.9, 0.1, 1.3), 1.35, 1.6, 1.85,
                      1.0, 0.7, kz, 1e-3, 0.05, mask)


def _rand(shape, seed=1):
    return np.random.default_rng(seed).standard_normal(shape)


def _slice2d(p: O.Problem3, k: int) -> O.Problem:
    return O.Problem(p.n1, p.n2, p.box[:4], p.alpha1, p.alpha2, p.kx, p.ky, p.eta, p.dt, p.mask[k])


def test_kz0_operators_reduce_to_2d_slices():
    p = _p3((7, 5, 6), kz=0.0)
    V = _rand(p.shape)
    mv, pc = O.matvec3(p, V), O.precond3_apply(p, V)
    for k in range(p.n3):
        q = _slice2d(p, k)
        np.testing.assert_allclose(mv[k], O.matvec(q, V[k]), rtol=0, atol=1e-12 * np.abs(mv).max())
        np.testing.assert_allclose(pc[k], O.precond_apply(q, V[k]), rtol=0,
                                   atol=1e-12 * np.abs(pc).max())


def test_kz0_march_reduces_to_2d_slices():
    w = make_config3d(shape=(7, 6, 3), m=3, kz=0.0)
    p = O.problem3_from_workload(w)
    u3 = O.march3_lu(p, w.u0, w.m, w.f_kind)
    for k in range(p.n3):
        u2 = O.march_lu(_slice2d(p, k), w.u0[k], w.m, w.f_kind)
        np.testing.assert_allclose(u3[k], u2, rtol=0, atol=1e-12 * np.abs(u3).max())


@pytest.mark.parametrize("perm", [(2, 1, 0), (1, 2, 0), (0, 2, 1)])
def test_axis_permutation_equivariance(perm):
    """perm lists, for each new axis (x, y, z), the old axis it takes."""
    p = _p3((5, 6, 7), mask=(_rand((7, 6, 5), 3) > 0).astype(np.uint8))
    V = _rand(p.shape, 2)
    n = (p.n1, p.n2, p.n3)
    al = (p.alpha1, p.alpha2, p.alpha3)
    ks = (p.kx, p.ky, p.kz)
    box = [(p.box[2 * a], p.box[2 * a + 1]) for a in range(3)]
    # array axis of physical axis a is 2 - a
    ax_perm = tuple(2 - perm[2 - t] for t in range(3))
    q = O.Problem3(n[perm[0]], n[perm[1]], n[perm[2]],
                   box[perm[0]] + box[perm[1]] + box[perm[2]],
                   al[perm[0]], al[perm[1]], al[perm[2]], ks[perm[0]], ks[perm[1]], ks[perm[2]],
                   p.eta, p.dt, np.ascontiguousarray(p.mask.transpose(ax_perm)))
    Vq = np.ascontiguousarray(V.transpose(ax_perm))
    for f in (O.matvec3, O.precond3_apply):
        a = f(p, V).transpose(ax_perm)
        b = f(q, Vq)
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.abs(a).max())


def test_matvec3_forms_agree():
    p = _p3((5, 6, 7))
    V = _rand(p.shape, 4)
    ref = (O.dense_M3(p) @ V.ravel()).reshape(p.shape)
    mv = O.matvec3(p, V)
    np.testing.assert_allclose(mv, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(O.matvec3_fast(p, V), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    for (k, j, i) in [(0, 0, 0), (6, 5, 4), (3, 2, 1), (0, 5, 2), (6, 0, 4)]:
        assert abs(O.matvec3_entry(p, V, k, j, i) - ref[k, j, i]) <= 1e-12 * np.abs(ref).max()


def test_precond3_forms_agree_with_dense_formula():
    p = _p3((5, 6, 7))
    V = _rand(p.shape, 5)
    ref = (O.precond3_dense(p) @ V.ravel()).reshape(p.shape)
    np.testing.assert_allclose(O.precond3_apply(p, V), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(O.precond3_apply_fft(p, V), ref, rtol=0,
                               atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("inside", [1, 0])
def test_precond3_inverts_tau_system_on_uniform_masks(inside):
    """All inside: P_hat^{-1} = (I - tau_1(A))^{-1}; all outside: ((1+d)I - tau_1(A))^{-1}."""
    p = _p3((6, 5, 4), mask=np.full((4, 5, 6), inside, np.uint8))
    tx = p.cx * O.toeplitz_first_column(p.alpha1, p.n1)
    ty = p.cy * O.toeplitz_first_column(p.alpha2, p.n2)
    tz = p.cz * O.toeplitz_first_column(p.alpha3, p.n3)
    I1, I2, I3 = np.eye(p.n1), np.eye(p.n2), np.eye(p.n3)
    tau1 = (np.kron(I3, np.kron(I2, O.tau_matrix(tx))) + np.kron(I3, np.kron(O.tau_matrix(ty), I1))
            + np.kron(O.tau_matrix(tz), np.kron(I2, I1)))
    shift = 1.0 if inside else 1.0 + p.d
    V = _rand(p.shape, 6)
    z = O.precond3_apply(p, V).ravel()
    back = shift * z - tau1 @ z
    np.testing.assert_allclose(back, V.ravel(), rtol=0, atol=1e-12 * np.abs(V).max())


def test_M3_symmetric_with_spectrum_at_least_one():
    p = _p3((5, 4, 6))
    M = O.dense_M3(p)
    assert np.abs(M - M.T).max() <= 1e-14 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() >= 1.0 - 1e-12


@pytest.mark.parametrize("side", ["right", "left"])
def test_gmres3_matches_lu(side):
    w = make_config3d(shape=(7, 6, 5), m=3)
    p = O.problem3_from_workload(w)
    u_lu = O.march3_lu(p, w.u0, w.m, w.f_kind)
    u_g, iters = O.march3_gmres(p, w.u0, w.m, w.f_kind, 20, 1e-13, side=side)
    assert np.abs(u_g - u_lu).max() <= 1e-10 * np.abs(u_lu).max()
    assert all(i > 0 for i in iters)


def _loss3(p, u0, m, f_kind, tgt):
    u = O.march3_lu(p, u0, m, f_kind)
    return float(np.sum((u - tgt) ** 2))


@pytest.mark.parametrize("f_kind", [1, 3])
def test_adjoint3_matches_central_fd(f_kind):
    p = _p3((4, 5, 3))
    rng = np.random.default_rng(11)
    u0 = 0.3 * p.mask + 0.2 * rng.standard_normal(p.shape)
    tgt = 0.1 * rng.standard_normal(p.shape)
    m = 3
    L, g0, gx, gy, gz = O.loss_and_grads3_lu(p, u0, m, f_kind, tgt)
    assert L == pytest.approx(_loss3(p, u0, m, f_kind, tgt), rel=1e-14)
    h = 1e-6
    du = rng.standard_normal(p.shape)
    import dataclasses
    for d in ((1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (0.4, -0.6, 0.8, 1)):
        pp = dataclasses.replace(p, kx=p.kx + h * d[0], ky=p.ky + h * d[1], kz=p.kz + h * d[2])
        pm = dataclasses.replace(p, kx=p.kx - h * d[0], ky=p.ky - h * d[1], kz=p.kz - h * d[2])
        fd = (_loss3(pp, u0 + h * d[3] * du, m, f_kind, tgt)
              - _loss3(pm, u0 - h * d[3] * du, m, f_kind, tgt)) / (2 * h)
        an = gx * d[0] + gy * d[1] + gz * d[2] + d[3] * float(np.sum(g0 * du))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9), d


def test_adjoint3_one_slice_reduces_to_2d():
    # one z-slice with kz = 0 is the two-dimensional problem
    p = _p3((6, 5, 1), kz=0.0)
    rng = np.random.default_rng(5)
    u0 = 0.3 * p.mask + 0.2 * rng.standard_normal(p.shape)
    tgt = 0.1 * rng.standard_normal(p.shape)
    L, g0, gx, gy, _ = O.loss_and_grads3_lu(p, u0, 3, 1, tgt)
    q = _slice2d(p, 0)
    u, traj = O.march_lu(q, u0[0], 3, 1, keep_all=True)
    g0_2, gx_2, gy_2 = O.adjoint_lu(q, traj, 2.0 * (u - tgt[0]), 1)
    assert L == pytest.approx(float(np.sum((u - tgt[0]) ** 2)), rel=1e-12)
    assert np.allclose(g0[0], g0_2, rtol=1e-11, atol=1e-14)
    assert gx == pytest.approx(gx_2, rel=1e-11)
    assert gy == pytest.approx(gy_2, rel=1e-11)

"""Plain FP64 reference for the three-dimensional penalized Riesz problem.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The paper treats two dimensions and names higher dimensions as future work
(concluding section); it gives no 3-D method.  The reading used here carries
each two-dimensional construction over with one more Kronecker factor:

* Section 2's implicit step: M = I - A + D with
  A = I_{n3} (x) I_{n2} (x) A_x + I_{n3} (x) A_y (x) I_{n1} + A_z (x) I_{n2} (x) I_{n1},
  A_s = c_s G_{n_s}^(alpha_s), c_s = dt k_s c_alpha_s / h_s^alpha_s, and
  D = diag(dt/eta * phi) outside the domain; b = u^{k-1} + dt mask f(u^{k-1}).
* Section 4.1's preconditioner: tau_1(A) is the same Kronecker sum of the
  tau matrices, diagonalised by S_{n3} (x) S_{n2} (x) S_{n1} with eigenvalues
  lx_i + ly_j + lz_k (Lemma 4.2's factorisation with three factors), so
  P_hat^{-1} = (I - Phi)(I - tau_1(A))^{-1} + Phi((1 + dt/eta) I - tau_1(A))^{-1}
  is two 3-D sine transforms around a diagonal scaling.

Arrays are [n3][n2][n1] (x fastest).  The one-dimensional ingredients (GL
weights, Toeplitz columns, tau eigenvalues, S_n) are the two-dimensional
oracle's, which its own tests pin.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Tuple

import numpy as np
import scipy.linalg as sla

from .rsfde_oracle import (G_dense, dst1_matrix, f_eval, fprime_eval, gmres, riesz_c,
                           tau_eigenvalues, tau_matrix, toeplitz_first_column)

__all__ = [
    "Problem3", "problem3_from_workload", "A3_parts", "dense_A3", "dense_M3",
    "matvec3", "matvec3_fast", "matvec3_entry", "tau_eigs3", "precond3_apply",
    "precond3_apply_fft", "precond3_dense", "rhs3", "march3_lu", "march3_gmres",
    "march3_lu_traj", "adjoint3_lu", "loss_and_grads3_lu",
]


@dataclass
class Problem3:
    n1: int
    n2: int
    n3: int
    box: Tuple[float, float, float, float, float, float]
    alpha1: float
    alpha2: float
    alpha3: float
    kx: float
    ky: float
    kz: float
    eta: float
    dt: float
    mask: np.ndarray  # uint8 [n3][n2][n1]

    def _c(self, axis: int) -> float:
        n = (self.n1, self.n2, self.n3)[axis]
        lo, hi = self.box[2 * axis], self.box[2 * axis + 1]
        h = (hi - lo) / (n + 1)
        alpha = (self.alpha1, self.alpha2, self.alpha3)[axis]
        k = (self.kx, self.ky, self.kz)[axis]
        return self.dt * k * riesz_c(alpha) / h ** alpha

    @property
    def cx(self):
        return self._c(0)

    @property
    def cy(self):
        return self._c(1)

    @property
    def cz(self):
        return self._c(2)

    @property
    def d(self):
        return self.dt / self.eta

    @property
    def phi(self):
        return 1.0 - self.mask.astype(np.float64)

    @property
    def shape(self):
        return (self.n3, self.n2, self.n1)


def problem3_from_workload(w) -> Problem3:
    return Problem3(w.n1, w.n2, w.n3, w.box, w.alpha1, w.alpha2, w.alpha3, w.kx, w.ky, w.kz,
                    w.eta, w.T / w.m, w.mask)


def _cols(p: Problem3):
    return (p.cx * toeplitz_first_column(p.alpha1, p.n1),
            p.cy * toeplitz_first_column(p.alpha2, p.n2),
            p.cz * toeplitz_first_column(p.alpha3, p.n3))


def A3_parts(p: Problem3):
    """A_x, A_y, A_z = c_s G^(alpha_s) (Section 2, one factor per axis)."""
    return (p.cx * G_dense(p.alpha1, p.n1), p.cy * G_dense(p.alpha2, p.n2),
            p.cz * G_dense(p.alpha3, p.n3))


def dense_A3(p: Problem3) -> np.ndarray:
    """The Kronecker sum with x fastest (tiny grids only)."""
    Ax, Ay, Az = A3_parts(p)
    I1, I2, I3 = np.eye(p.n1), np.eye(p.n2), np.eye(p.n3)
    return (np.kron(I3, np.kron(I2, Ax)) + np.kron(I3, np.kron(Ay, I1))
            + np.kron(Az, np.kron(I2, I1)))


def dense_M3(p: Problem3) -> np.ndarray:
    N = p.n1 * p.n2 * p.n3
    return np.eye(N) - dense_A3(p) + np.diag(p.d * p.phi.ravel())


def _along(Amat: np.ndarray, V: np.ndarray, axis: int) -> np.ndarray:
    """Apply the matrix Amat to every line of V along array axis `axis`."""
    return np.moveaxis(np.tensordot(Amat, V, axes=([1], [axis])), 0, axis)


def matvec3(p: Problem3, V: np.ndarray, parts=None) -> np.ndarray:
    """M v on V[n3][n2][n1]: V - A_x along x - A_y along y - A_z along z + d phi V."""
    Ax, Ay, Az = A3_parts(p) if parts is None else parts
    return V - _along(Ax, V, 2) - _along(Ay, V, 1) - _along(Az, V, 0) + p.d * p.phi * V


def matvec3_fast(p: Problem3, V: np.ndarray) -> np.ndarray:
    """matvec3 with each Toeplitz product done by scipy's FFT-based Toeplitz
    multiply (a library primitive), for full-size grids."""
    from scipy.linalg import matmul_toeplitz
    tx, ty, tz = _cols(p)
    n3, n2, n1 = p.shape
    out = V + p.d * p.phi * V
    out -= matmul_toeplitz(tx, V.reshape(-1, n1).T).T.reshape(V.shape)
    Vy = np.moveaxis(V, 1, 0).reshape(n2, -1)
    out -= np.moveaxis(matmul_toeplitz(ty, Vy).reshape(n2, n3, n1), 0, 1)
    out -= matmul_toeplitz(tz, V.reshape(n3, -1)).reshape(V.shape)
    return out


def matvec3_entry(p: Problem3, V: np.ndarray, k: int, j: int, i: int) -> float:
    """One entry of M v summed directly from the Toeplitz entries: O(n1+n2+n3)."""
    tx, ty, tz = _cols(p)
    ax = tx[np.abs(np.arange(p.n1) - i)]
    ay = ty[np.abs(np.arange(p.n2) - j)]
    az = tz[np.abs(np.arange(p.n3) - k)]
    return float(V[k, j, i] - ax @ V[k, j, :] - ay @ V[k, :, i] - az @ V[:, j, i]
                 + p.d * p.phi[k, j, i] * V[k, j, i])


def tau_eigs3(p: Problem3):
    """Eigenvalues of the scaled tau matrices along x, y, z (Section 4.1)."""
    tx, ty, tz = _cols(p)
    return tau_eigenvalues(tx), tau_eigenvalues(ty), tau_eigenvalues(tz)


def _E1(p: Problem3, lam):
    lx, ly, lz = lam
    return 1.0 - lx[None, None, :] - ly[None, :, None] - lz[:, None, None]


def precond3_apply(p: Problem3, V: np.ndarray, lam=None) -> np.ndarray:
    """z = P_hat^{-1} v with dense sine matrices along each axis:
    W = S v;  Y1 = S (W / E1);  Y2 = S (W / (E1 + dt/eta));  z = mask Y1 + phi Y2,
    with S = S_{n3} (x) S_{n2} (x) S_{n1} and E1 = 1 - lx_i - ly_j - lz_k."""
    lam = tau_eigs3(p) if lam is None else lam
    Ss = (dst1_matrix(p.n1), dst1_matrix(p.n2), dst1_matrix(p.n3))

    def S3(X):
        return _along(Ss[2], _along(Ss[1], _along(Ss[0], X, 2), 1), 0)

    W = S3(V)
    E1 = _E1(p, lam)
    Y1 = S3(W / E1)
    Y2 = S3(W / (E1 + p.d))
    return (1.0 - p.phi) * Y1 + p.phi * Y2


def precond3_apply_fft(p: Problem3, V: np.ndarray, lam=None) -> np.ndarray:
    """precond3_apply with S v from scipy's orthonormal DST-I (a library
    primitive), for full-size grids."""
    import scipy.fft as sf
    lam = tau_eigs3(p) if lam is None else lam
    W = sf.dstn(V, type=1, norm="ortho", workers=-1)
    E1 = _E1(p, lam)
    Y1 = sf.dstn(W / E1, type=1, norm="ortho", workers=-1)
    Y2 = sf.dstn(W / (E1 + p.d), type=1, norm="ortho", workers=-1)
    return (1.0 - p.phi) * Y1 + p.phi * Y2


def precond3_dense(p: Problem3) -> np.ndarray:
    """(I - Phi)(I - tau_1(A))^{-1} + Phi((1 + dt/eta) I - tau_1(A))^{-1} formed
    densely from the tau matrices and explicit inverses (tiny grids only)."""
    tx, ty, tz = _cols(p)
    I1, I2, I3 = np.eye(p.n1), np.eye(p.n2), np.eye(p.n3)
    tau1 = (np.kron(I3, np.kron(I2, tau_matrix(tx))) + np.kron(I3, np.kron(tau_matrix(ty), I1))
            + np.kron(tau_matrix(tz), np.kron(I2, I1)))
    N = p.n1 * p.n2 * p.n3
    I = np.eye(N)
    Phi = np.diag(p.phi.ravel())
    return (I - Phi) @ np.linalg.inv(I - tau1) + Phi @ np.linalg.inv((1.0 + p.d) * I - tau1)


def rhs3(p: Problem3, u_prev: np.ndarray, f_kind: int) -> np.ndarray:
    """b = u^{k-1} + dt mask f(u^{k-1}) (f zero outside the domain)."""
    return u_prev + p.dt * p.mask * f_eval(f_kind, u_prev)


def march3_lu(p: Problem3, u0: np.ndarray, m: int, f_kind: int) -> np.ndarray:
    """u^k = M^{-1} b^{k-1}, k = 1..m, with one LU of the dense M (tiny grids)."""
    lu = sla.lu_factor(dense_M3(p))
    u = u0.astype(np.float64).copy()
    for _ in range(m):
        u = sla.lu_solve(lu, rhs3(p, u, f_kind).ravel()).reshape(p.shape)
    return u


def march3_gmres(p: Problem3, u0: np.ndarray, m: int, f_kind: int, restart: int, tol: float,
                 side: str = "right", precond: bool = True, max_iters: int = 10000):
    """m implicit steps, each solved by GMRES(restart) on the 3-D operators with
    the initial guess u^0, then 2u^{k-1} - u^{k-2}.  Returns (u^m, iterations)."""
    parts = A3_parts(p)
    lam = tau_eigs3(p)
    Aop = lambda V: matvec3(p, V, parts)  # noqa: E731
    Pinv = (lambda V: precond3_apply(p, V, lam)) if precond else None
    u_prev2 = None
    u = u0.astype(np.float64).copy()
    iters = []
    for _ in range(m):
        b = rhs3(p, u, f_kind)
        x0 = u if u_prev2 is None else 2.0 * u - u_prev2
        x, it, _ok = gmres(Aop, b, x0, restart, tol, max_iters, Pinv, side)
        iters.append(it)
        u_prev2, u = u, x
    return u, iters


# ---------------------------------------------------------------------------
# Adjoint of the 3-D march (no counterpart in the paper): the two-dimensional
# derivation with one more factor.  M is symmetric (each G^(alpha) is), so
# with M u^k = u^{k-1} + dt mask f(u^{k-1}) and L = L(u^m):
#   mu^k = M^{-1} lambda^k,  lambda^{k-1} = mu^k + dt mask f'(u^{k-1}) mu^k,
#   dL/dk_s += mu^k . ((A_s / k_s along axis s) u^k)   (dM/dk_s = -A_s / k_s).
# ---------------------------------------------------------------------------

def march3_lu_traj(p: Problem3, u0: np.ndarray, m: int, f_kind: int):
    """march3_lu keeping every state: [u^0, ..., u^m]."""
    lu = sla.lu_factor(dense_M3(p))
    traj = [u0.astype(np.float64).copy()]
    for _ in range(m):
        traj.append(sla.lu_solve(lu, rhs3(p, traj[-1], f_kind).ravel()).reshape(p.shape))
    return traj


def _unit_parts(p: Problem3):
    """A_x / kx, A_y / ky, A_z / kz: the factors with unit k (defined at k = 0 too)."""
    out = []
    for axis, (alpha, n) in enumerate(((p.alpha1, p.n1), (p.alpha2, p.n2), (p.alpha3, p.n3))):
        lo, hi = p.box[2 * axis], p.box[2 * axis + 1]
        h = (hi - lo) / (n + 1)
        out.append(p.dt * riesz_c(alpha) / h ** alpha * G_dense(alpha, n))
    return out


def adjoint3_lu(p: Problem3, traj, lam_m: np.ndarray, f_kind: int):
    """Reverse sweep for L(u^m) given the forward trajectory [u^0..u^m].
    Returns (lambda^0 = dL/du^0, dL/dkx, dL/dky, dL/dkz)."""
    lu = sla.lu_factor(dense_M3(p))
    Ux, Uy, Uz = _unit_parts(p)
    lam = lam_m.astype(np.float64).copy()
    g = [0.0, 0.0, 0.0]
    for k in range(len(traj) - 1, 0, -1):
        mu = sla.lu_solve(lu, lam.ravel()).reshape(p.shape)
        uk = traj[k]
        g[0] += float(np.sum(mu * _along(Ux, uk, 2)))
        g[1] += float(np.sum(mu * _along(Uy, uk, 1)))
        g[2] += float(np.sum(mu * _along(Uz, uk, 0)))
        lam = mu + p.dt * p.mask * fprime_eval(f_kind, traj[k - 1]) * mu
    return lam, g[0], g[1], g[2]


def loss_and_grads3_lu(p: Problem3, u0: np.ndarray, m: int, f_kind: int, u_tgt: np.ndarray):
    """L = ||u^m - u_tgt||^2 and its gradients w.r.t. (u0, kx, ky, kz)."""
    traj = march3_lu_traj(p, u0, m, f_kind)
    diff = traj[-1] - u_tgt
    g0, gx, gy, gz = adjoint3_lu(p, traj, 2.0 * diff, f_kind)
    return float(np.sum(diff * diff)), g0, gx, gy, gz

"""Plain, slow, FP64 reference for the penalized 2D Riesz space-fractional diffusion solve.

TEST INFRASTRUCTURE ONLY — see the package docstring.  It shares no code with
the HIP path; the only common import is the seeded input generator
(``workloads``), which holds none of the method's arithmetic.

Paper: Huang & Sun, "A preconditioner based on sine transform for
two-dimensional Riesz space fractional diffusion equations in convex domains"
(arXiv 2102.11576).  Every function cites the passage it follows.

Conventions
-----------
* Unknowns are stored as arrays U[j][i] of shape (n2, n1) (x fastest); the
  vector u of Section 2 is U.ravel() (lexicographic ordering, x fastest).
* mask[j][i] = 1 inside the convex domain, 0 in the penalty region; the
  paper's Phi_d is diag(1 - mask) (Section 4.1, splitting of M).
* Everything is float64.

Tiers
-----
O1  dense M + one LU per plan, u^k = M^{-1} b^{k-1}            (tiny grids)
O2  Kronecker-dense operators (matvec, preconditioner) on arrays
O3  dense adjoint march (one LU, transposed solves)
plus a plain restarted GMRES (MGS Arnoldi + Givens) used for iteration-count
pins and "GMRES agrees with LU".

Parity status: every function here is pinned by a test in tests/ against a
closed form, a library routine, brute force or the paper's own printed
numbers; see tests/test_oracle_*.py.  Nothing is "parity unpinned" except the
mixed-precision comparison, which by construction has no oracle counterpart.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Optional, Tuple

import numpy as np
import scipy.linalg as sla

# Source-term kinds (same integer codes as the input generator / C ABI).
F_NONE, F_LOGISTIC, F_SIN, F_CUBIC, F_DECAY = 0, 1, 2, 3, 4

__all__ = [
    "gl_weights", "riesz_c", "mesh_widths", "toeplitz_first_column", "G_dense",
    "scheme_rows_bruteforce", "Problem", "problem_from_workload", "A_parts",
    "dense_A", "dense_M", "f_eval", "fprime_eval", "rhs", "march_lu",
    "matvec", "tau_hankel", "tau_matrix", "dst1_matrix", "tau_eigenvalues",
    "tau_eigs_dense", "tau_eigs_xy", "precond_dense", "precond_apply", "P_dense",
    "gmres", "march_gmres", "adjoint_lu", "loss_and_grads_lu",
    "matvec_fast", "precond_apply_fft", "matvec_entry",
    "example1_march",
    "F_NONE", "F_LOGISTIC", "F_SIN", "F_CUBIC", "F_DECAY",
]


# ---------------------------------------------------------------------------
# Section 2: Grunwald-Letnikov weights, Riesz constant, mesh.
# ---------------------------------------------------------------------------

def gl_weights(alpha: float, n: int) -> np.ndarray:
    """g_0..g_n of the shifted Grunwald-Letnikov formulas, by the recurrence (g_form).

    g_0 = 1 and g_l = (1 - (alpha+1)/l) g_{l-1} for l >= 1.
    """
    g = np.empty(n + 1, dtype=np.float64)
    g[0] = 1.0
    for l in range(1, n + 1):
        g[l] = (1.0 - (alpha + 1.0) / l) * g[l - 1]
    return g


def riesz_c(alpha: float) -> float:
    """c_alpha = -1 / (2 cos(alpha*pi/2)), positive for 1 < alpha < 2 (Section 1)."""
    return -1.0 / (2.0 * math.cos(alpha * math.pi / 2.0))


def mesh_widths(n1: int, n2: int, box) -> Tuple[float, float]:
    """h_x = (b-a)/(n1+1), h_y = (d-c)/(n2+1) (Section 2, uniform partition)."""
    x_lo, x_hi, y_lo, y_hi = box
    return (x_hi - x_lo) / (n1 + 1), (y_hi - y_lo) / (n2 + 1)


def toeplitz_first_column(alpha: float, n: int) -> np.ndarray:
    """First column of G_n^(alpha) as displayed in (G): [2g_1, g_0+g_2, g_3, ..., g_n]."""
    g = gl_weights(alpha, max(n, 2))
    t = np.empty(n, dtype=np.float64)
    t[0] = 2.0 * g[1]
    if n > 1:
        t[1] = g[0] + g[2]
    for k in range(2, n):
        t[k] = g[k + 1]
    return t


def G_dense(alpha: float, n: int) -> np.ndarray:
    """The symmetric Toeplitz matrix G_n^(alpha) of (G)."""
    return sla.toeplitz(toeplitz_first_column(alpha, n))


def scheme_rows_bruteforce(alpha: float, n: int) -> np.ndarray:
    """Matrix of the x-part of the scheme built by evaluating the two sums of
    (difference_scheme) literally, with the zero Dirichlet values (B2).

    Row i (1-based) holds the coefficients of u_1..u_n in
        sum_{l=0}^{i+1} g_l u_{i-l+1} + sum_{l=0}^{n-i+2} g_l u_{i+l-1},
    where u_0 = u_{n+1} = 0 and indices beyond [0, n+1] do not occur.
    Used only as an independent pin of toeplitz_first_column / G_dense.
    """
    g = gl_weights(alpha, n + 3)
    Gm = np.zeros((n, n))
    for i in range(1, n + 1):
        for l in range(0, i + 2):
            idx = i - l + 1
            if 1 <= idx <= n:
                Gm[i - 1, idx - 1] += g[l]
        for l in range(0, n - i + 3):
            idx = i + l - 1
            if 1 <= idx <= n:
                Gm[i - 1, idx - 1] += g[l]
    return Gm


# ---------------------------------------------------------------------------
# Section 2: the linear system of one implicit step.
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    n1: int
    n2: int
    box: Tuple[float, float, float, float]
    alpha1: float
    alpha2: float
    kx: float
    ky: float
    eta: float
    dt: float
    mask: np.ndarray  # uint8 [n2][n1]

    @property
    def hx(self):
        return mesh_widths(self.n1, self.n2, self.box)[0]

    @property
    def hy(self):
        return mesh_widths(self.n1, self.n2, self.box)[1]

    @property
    def cx(self):
        """c_x = dt kx c_alpha1 / h_x^alpha1 (Section 2, before (approximation))."""
        return self.dt * self.kx * riesz_c(self.alpha1) / self.hx ** self.alpha1

    @property
    def cy(self):
        return self.dt * self.ky * riesz_c(self.alpha2) / self.hy ** self.alpha2

    @property
    def d(self):
        """Penalty coefficient dt/eta applied outside the domain (Section 2)."""
        return self.dt / self.eta

    @property
    def phi(self):
        """Diagonal of Phi_d: 1 in the penalty region, 0 inside (Section 4.1)."""
        return 1.0 - self.mask.astype(np.float64)


def problem_from_workload(w, kx: Optional[float] = None, ky: Optional[float] = None) -> Problem:
    return Problem(w.n1, w.n2, w.box, w.alpha1, w.alpha2,
                   w.kx if kx is None else kx, w.ky if ky is None else ky,
                   w.eta, w.T / w.m, w.mask)


def A_parts(p: Problem) -> Tuple[np.ndarray, np.ndarray]:
    """A_x = c_x G_{n1}^(alpha1), A_y = c_y G_{n2}^(alpha2) (below (toeplitz_A))."""
    return p.cx * G_dense(p.alpha1, p.n1), p.cy * G_dense(p.alpha2, p.n2)


def dense_A(p: Problem) -> np.ndarray:
    """A = I_{n2} (x) A_x + A_y (x) I_{n1}  (toeplitz_A), x-fastest ordering."""
    Ax, Ay = A_parts(p)
    return np.kron(np.eye(p.n2), Ax) + np.kron(Ay, np.eye(p.n1))


def dense_M(p: Problem) -> np.ndarray:
    """M = I - A + D (matrix_vector, linearsystem), D = diag(dt/eta * phi)."""
    N = p.n1 * p.n2
    return np.eye(N) - dense_A(p) + np.diag(p.d * p.phi.ravel())


def f_eval(kind: int, u: np.ndarray) -> np.ndarray:
    if kind == F_NONE:
        return np.zeros_like(u)
    if kind == F_LOGISTIC:
        return u * (1.0 - u)
    if kind == F_SIN:
        return np.sin(u)
    if kind == F_CUBIC:
        return u - u ** 3
    if kind == F_DECAY:
        return -u
    raise ValueError(kind)


def fprime_eval(kind: int, u: np.ndarray) -> np.ndarray:
    if kind == F_NONE:
        return np.zeros_like(u)
    if kind == F_LOGISTIC:
        return 1.0 - 2.0 * u
    if kind == F_SIN:
        return np.cos(u)
    if kind == F_CUBIC:
        return 1.0 - 3.0 * u * u
    if kind == F_DECAY:
        return -np.ones_like(u)
    raise ValueError(kind)


def rhs(p: Problem, u_prev: np.ndarray, f_kind: int, f_values: Optional[np.ndarray] = None) -> np.ndarray:
    """b^{k-1} = u^{k-1} + dt f^{k-1} (linearsystem) with the zero extension of f
    outside the domain (Section 2, after (B1)); f is taken at the previous level
    (f_approximation).  ``f_values`` overrides f(u) (used by Example 1)."""
    fv = f_eval(f_kind, u_prev) if f_values is None else f_values
    return u_prev + p.dt * p.mask * fv


def march_lu(p: Problem, u0: np.ndarray, m: int, f_kind: int,
             keep_all: bool = False):
    """O1: u^k = M^{-1} b^{k-1}, k = 1..m, with one LU of the dense M."""
    lu = sla.lu_factor(dense_M(p))
    u = u0.astype(np.float64).copy()
    traj = [u.copy()] if keep_all else None
    for _ in range(m):
        b = rhs(p, u, f_kind)
        u = sla.lu_solve(lu, b.ravel()).reshape(p.n2, p.n1)
        if keep_all:
            traj.append(u.copy())
    return (u, traj) if keep_all else u


def matvec(p: Problem, V: np.ndarray, Ax=None, Ay=None) -> np.ndarray:
    """O2: M v on the array V[n2][n1]: V - V A_x^T - A_y V + d phi V.

    (I (x) A_x) v  <->  V A_x^T and (A_y (x) I) v <-> A_y V for x-fastest
    ordering; A_x and A_y are symmetric (G is symmetric Toeplitz)."""
    if Ax is None or Ay is None:
        Ax, Ay = A_parts(p)
    return V - V @ Ax.T - Ay @ V + p.d * p.phi * V


def matvec_fast(p: Problem, V: np.ndarray) -> np.ndarray:
    """M v for large grids: the same formula as matvec with the Toeplitz
    products done by scipy's FFT-based Toeplitz multiply (a library primitive;
    pinned against matvec in the tests)."""
    from scipy.linalg import matmul_toeplitz
    tx = p.cx * toeplitz_first_column(p.alpha1, p.n1)
    ty = p.cy * toeplitz_first_column(p.alpha2, p.n2)
    VAx = matmul_toeplitz(tx, V.T).T          # rows: V A_x^T = (A_x V^T)^T
    AyV = matmul_toeplitz(ty, V)              # columns
    return V - VAx - AyV + p.d * p.phi * V


def matvec_entry(p: Problem, V: np.ndarray, j: int, i: int) -> float:
    """One entry (row j, column i) of M v, summed directly from (difference_scheme)'s
    Toeplitz form: O(n1 + n2) work, for sampled checks at any size."""
    tx = p.cx * toeplitz_first_column(p.alpha1, p.n1)
    ty = p.cy * toeplitz_first_column(p.alpha2, p.n2)
    ax = tx[np.abs(np.arange(p.n1) - i)]
    ay = ty[np.abs(np.arange(p.n2) - j)]
    return float(V[j, i] - ax @ V[j, :] - ay @ V[:, i] + p.d * p.phi[j, i] * V[j, i])


# ---------------------------------------------------------------------------
# Section 4.1: tau matrices, sine transform, the preconditioner.
# ---------------------------------------------------------------------------

def tau_hankel(t: np.ndarray) -> np.ndarray:
    """Hankel correction H_n of the symmetric Toeplitz T_n = [t_|i-j|] (Section 4.1).

    H is constant along anti-diagonals; the 2n-1 anti-diagonal values, from the
    top-left corner to the bottom-right one, are
    [t_2, t_3, ..., t_{n-1}, 0, 0, 0, t_{n-1}, ..., t_3, t_2].
    """
    n = len(t)
    if n <= 2:
        return np.zeros((n, n))
    h = np.concatenate([t[2:n], np.zeros(3), t[2:n][::-1]])
    assert len(h) == 2 * n - 1
    H = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            H[i, j] = h[i + j]
    return H


def tau_matrix(t: np.ndarray) -> np.ndarray:
    """tau(T_n) = T_n - H_n (Section 4.1)."""
    return sla.toeplitz(t) - tau_hankel(t)


def dst1_matrix(n: int) -> np.ndarray:
    """S_n with [S_n]_{ij} = sqrt(2/(n+1)) sin(pi i j/(n+1)), 1 <= i, j <= n (Section 4.1)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(i, i) / (n + 1))


def tau_eigenvalues(t: np.ndarray) -> np.ndarray:
    """Eigenvalues of tau(T_n) in the order diagonalised by S_n: for k = 1..n,
    lambda_k = t_0 + 2 sum_{j=1}^{n-1} t_j cos(j k pi / (n+1)).

    This is the closed form of "eigenvalues determined by the first column"
    (Section 4.1); it is pinned in the tests against diag(S tau(T) S) with the
    Hankel correction formed densely."""
    n = len(t)
    k = np.arange(1, n + 1, dtype=np.float64)
    lam = np.full(n, t[0], dtype=np.float64)
    for j in range(1, n):
        lam += 2.0 * t[j] * np.cos(j * k * np.pi / (n + 1))
    return lam


def tau_eigs_dense(t: np.ndarray) -> np.ndarray:
    """diag(S tau(T) S): the eigenvalues read off the sine-transform diagonalisation."""
    S = dst1_matrix(len(t))
    return np.diag(S @ tau_matrix(t) @ S).copy()


def tau_eigs_xy(p: Problem) -> Tuple[np.ndarray, np.ndarray]:
    lx = p.cx * tau_eigenvalues(toeplitz_first_column(p.alpha1, p.n1))
    ly = p.cy * tau_eigenvalues(toeplitz_first_column(p.alpha2, p.n2))
    return lx, ly


def precond_apply(p: Problem, V: np.ndarray, lam=None) -> np.ndarray:
    """O2: z = P_hat^{-1} v by the 2D sine transform (preconditioner; Lemma 4.2's
    factorisation I - tau_1(A) = (S (x) S)(I - I (x) L_x - L_y (x) I)(S (x) S)).

    W = S_y V S_x;  Y1 = S_y (W / (1 - lx_i - ly_j)) S_x;
    Y2 = S_y (W / (1 + dt/eta - lx_i - ly_j)) S_x;  z = (1-phi) Y1 + phi Y2.
    """
    lx, ly = tau_eigs_xy(p) if lam is None else lam
    Sx, Sy = dst1_matrix(p.n1), dst1_matrix(p.n2)
    W = Sy @ V @ Sx
    E1 = 1.0 - lx[None, :] - ly[:, None]
    E2 = E1 + p.d
    Y1 = Sy @ (W / E1) @ Sx
    Y2 = Sy @ (W / E2) @ Sx
    return (1.0 - p.phi) * Y1 + p.phi * Y2


def precond_apply_fft(p: Problem, V: np.ndarray, lam=None) -> np.ndarray:
    """precond_apply with S_n v taken from scipy's orthonormal DST-I (a library
    primitive, pinned equal to S_n v in the tests), for large grids."""
    import scipy.fft as sf
    lx, ly = tau_eigs_xy(p) if lam is None else lam
    W = sf.dstn(V, type=1, norm="ortho", workers=-1)
    E1 = 1.0 - lx[None, :] - ly[:, None]
    E2 = E1 + p.d
    Y1 = sf.dstn(W / E1, type=1, norm="ortho", workers=-1)
    Y2 = sf.dstn(W / E2, type=1, norm="ortho", workers=-1)
    return (1.0 - p.phi) * Y1 + p.phi * Y2


def P_dense(p: Problem) -> np.ndarray:
    """The preliminary preconditioner P = I - tau_1(A) + D (p1, tau_A), dense."""
    tx = p.cx * toeplitz_first_column(p.alpha1, p.n1)
    ty = p.cy * toeplitz_first_column(p.alpha2, p.n2)
    tau1 = np.kron(np.eye(p.n2), tau_matrix(tx)) + np.kron(tau_matrix(ty), np.eye(p.n1))
    N = p.n1 * p.n2
    return np.eye(N) - tau1 + np.diag(p.d * p.phi.ravel())


def precond_dense(p: Problem) -> np.ndarray:
    """P_hat^{-1} = (I - Phi)(I - tau_1(A))^{-1} + Phi((1 + dt/eta) I - tau_1(A))^{-1}
    formed densely with explicit inverses (preconditioner).  Tiny grids only."""
    tx = p.cx * toeplitz_first_column(p.alpha1, p.n1)
    ty = p.cy * toeplitz_first_column(p.alpha2, p.n2)
    tau1 = np.kron(np.eye(p.n2), tau_matrix(tx)) + np.kron(tau_matrix(ty), np.eye(p.n1))
    N = p.n1 * p.n2
    I = np.eye(N)
    Phi = np.diag(p.phi.ravel())
    return (I - Phi) @ np.linalg.inv(I - tau1) + Phi @ np.linalg.inv((1.0 + p.d) * I - tau1)


# ---------------------------------------------------------------------------
# Section 5: restarted GMRES with the preconditioner.
# ---------------------------------------------------------------------------

def gmres(Aop: Callable, b: np.ndarray, x0: np.ndarray, restart: int, tol: float,
          max_iters: int = 10000, Pinv: Optional[Callable] = None, side: str = "right",
          history: Optional[list] = None):
    """Restarted GMRES(restart), modified Gram-Schmidt Arnoldi, Givens rotations.

    side="right": Krylov space of A P^{-1}; stop when the residual estimate
        <= tol * ||b||_2; x = x0 + P^{-1} V y at the end of each cycle and the
        true residual b - A x restarts the next cycle.
    side="left": Krylov space of P^{-1} A; stop when ||P^{-1}(b - A x)||_2
        <= tol * ||P^{-1} b||_2 (the convention of the paper's experiments,
        Section 5, with r^(0) read as the zero-guess residual).
    Returns (x, inner_iterations, converged).  With a list `history`, every
    residual norm the stopping test looks at (restart residuals and per-step
    estimates) is appended to it, divided by the reference norm.
    """
    shape = b.shape
    bv = b.ravel()
    x = x0.ravel().astype(np.float64).copy()
    P = (lambda v: v) if Pinv is None else (lambda v: Pinv(v.reshape(shape)).ravel())
    A = lambda v: Aop(v.reshape(shape)).ravel()  # noqa: E731
    if side == "right":
        bnorm = np.linalg.norm(bv)
    else:
        bnorm = np.linalg.norm(P(bv))
    if bnorm == 0.0:
        return np.zeros(shape), 0, True
    total = 0
    while True:
        r = bv - A(x)
        if side == "left":
            r = P(r)
        beta = np.linalg.norm(r)
        if history is not None:
            history.append(beta / bnorm)
        if beta <= tol * bnorm:
            return x.reshape(shape), total, True
        if total >= max_iters:
            return x.reshape(shape), total, False
        V = np.zeros((restart + 1, bv.size))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            w = A(P(V[j])) if side == "right" else P(A(V[j]))
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                tmp = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = tmp
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            if history is not None:
                history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or total >= max_iters:
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        upd = V[:j_done].T @ y
        x = x + (P(upd) if side == "right" else upd)
        if side == "left" and abs(g[j_done]) <= tol * bnorm:
            # the paper's convention stops on the preconditioned estimate
            return x.reshape(shape), total, True


def march_gmres(p: Problem, u0: np.ndarray, m: int, f_kind: int, restart: int, tol: float,
                side: str = "right", precond: bool = True, f_values_fn=None,
                max_iters: int = 10000, histories: Optional[list] = None):
    """March m implicit steps solving each M u^k = b^{k-1} with GMRES(restart).

    Initial guess (Section 5): u^0 at the first step, 2u^{k-1} - u^{k-2} after.
    ``f_values_fn(k_minus_1, u_prev)`` overrides f (Example 1).  With a list
    ``histories``, each step appends the residual history of its solve (gmres).
    Returns (u^m, iterations per step)."""
    Ax, Ay = A_parts(p)
    Aop = lambda V: matvec(p, V, Ax, Ay)  # noqa: E731
    lam = tau_eigs_xy(p)
    Pinv = (lambda V: precond_apply(p, V, lam)) if precond else None
    u_prev2 = None
    u = u0.astype(np.float64).copy()
    iters = []
    for k in range(1, m + 1):
        fv = None if f_values_fn is None else f_values_fn(k - 1, u)
        b = rhs(p, u, f_kind, fv)
        x0 = u if u_prev2 is None else 2.0 * u - u_prev2
        h = None if histories is None else []
        x, it, ok = gmres(Aop, b, x0, restart, tol, max_iters, Pinv, side, h)
        if histories is not None:
            histories.append(h)
        iters.append(it)
        u_prev2, u = u, x
    return u, iters


# ---------------------------------------------------------------------------
# Adjoint of the march (no counterpart in the paper; derived from (matrix_vector)).
# ---------------------------------------------------------------------------

def adjoint_lu(p: Problem, traj, lam_m: np.ndarray, f_kind: int):
    """O3: reverse sweep for L(u^m) given the forward trajectory [u^0..u^m].

    With M u^k = u^{k-1} + dt mask f(u^{k-1}) and M symmetric (G symmetric,
    Corollary 2.1; Lemma 2.3):
      mu^k      = M^{-1} lambda^k
      lambda^{k-1} = mu^k + dt mask f'(u^{k-1}) mu^k
      dL/dkx   += mu^k . ((I (x) A_x) u^k) / kx   (dM/dkx = -(I (x) A_x)/kx)
      dL/dky   += mu^k . ((A_y (x) I) u^k) / ky
    Returns (lambda^0 = dL/du^0, dL/dkx, dL/dky)."""
    lu = sla.lu_factor(dense_M(p))
    Ax1 = riesz_c(p.alpha1) * p.dt / p.hx ** p.alpha1 * G_dense(p.alpha1, p.n1)  # A_x / kx
    Ay1 = riesz_c(p.alpha2) * p.dt / p.hy ** p.alpha2 * G_dense(p.alpha2, p.n2)  # A_y / ky
    lam = lam_m.astype(np.float64).copy()
    gkx = 0.0
    gky = 0.0
    m = len(traj) - 1
    for k in range(m, 0, -1):
        mu = sla.lu_solve(lu, lam.ravel()).reshape(p.n2, p.n1)
        uk = traj[k]
        gkx += float(np.sum(mu * (uk @ Ax1.T)))
        gky += float(np.sum(mu * (Ay1 @ uk)))
        lam = mu + p.dt * p.mask * fprime_eval(f_kind, traj[k - 1]) * mu
    return lam, gkx, gky


def loss_and_grads_lu(w, u_tgt: np.ndarray, kx: float, ky: float, u0=None):
    """L = ||u(T) - u_tgt||^2 and its gradients w.r.t. (u0, kx, ky) by O1 + O3."""
    p = problem_from_workload(w, kx, ky)
    u0 = w.u0 if u0 is None else u0
    uT, traj = march_lu(p, u0, w.m, w.f_kind, keep_all=True)
    diff = uT - u_tgt
    L = float(np.sum(diff * diff))
    g0, gkx, gky = adjoint_lu(p, traj, 2.0 * diff, w.f_kind)
    return L, g0, gkx, gky


# ---------------------------------------------------------------------------
# Section 5, Example 1: manufactured solution on the ellipse.
# ---------------------------------------------------------------------------

def example1_march(w, side: str = "left", precond: bool = True, tol: Optional[float] = None,
                   use_lu: bool = False):
    """Run Example 1 as in Section 5 (T, m, eta, GMRES(20), tol 1e-8 by default).

    The source f(u, x, y, t) = -u + e^{-t} g0 is taken at t_{k-1} (f_approximation);
    g0 and the exact solution come with the workload (input fields).
    Returns (error, mean iterations per step, u^m, penalty-region max |u|)."""
    p = problem_from_workload(w)
    g0 = w.extra["src"]
    fn = lambda km1, u: f_eval(F_DECAY, u) + math.exp(-km1 * p.dt) * g0  # noqa: E731
    if use_lu:
        lu = sla.lu_factor(dense_M(p))
        u = w.u0.copy()
        for k in range(1, w.m + 1):
            bb = rhs(p, u, F_NONE, fn(k - 1, u))
            u = sla.lu_solve(lu, bb.ravel()).reshape(u.shape)
        iters = [0]
    else:
        u, iters = march_gmres(p, w.u0, w.m, F_NONE, w.restart, w.tol if tol is None else tol,
                               side=side, precond=precond, f_values_fn=fn)
    ue = math.exp(-w.T) * w.extra["exact0"]
    inside = w.mask.astype(bool)
    err = np.max(np.abs(ue - u)[inside]) / np.max(np.abs(ue)[inside])
    pen = np.max(np.abs(u[~inside])) if (~inside).any() else 0.0
    return float(err), float(np.mean(iters)), u, float(pen)

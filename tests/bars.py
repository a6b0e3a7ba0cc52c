"""Shared comparison helpers of the parity tests (bars only; no arithmetic of
the method beyond reading the oracle's coefficient tables)."""

import numpy as np

import oracle as O

EPS64 = float(np.finfo(np.float64).eps)


def precond_kappa(p):
    """Conditioning of the eigenvalue denominators of the preconditioner.

    E1 = 1 - lambda_x,i - lambda_y,j with lambda the tau eigenvalues, each a
    cosine sum of the scaled first column (Section 4.1).  At low frequencies the
    sum nearly cancels (terms of size c_x |t_j|, result of order one), so any
    FP64 evaluation of E1 carries an absolute error of about
    eps (sum_j |c_x t_j| + sum_j |c_y t_j|), whatever the transform.  Returns
    (kappa1, kappa2): that sum over min E1 (domain part) and over min E2 =
    min E1 + dt/eta (penalty part)."""
    tx = np.abs(p.cx * O.toeplitz_first_column(p.alpha1, p.n1)).sum()
    ty = np.abs(p.cy * O.toeplitz_first_column(p.alpha2, p.n2)).sum()
    lx, ly = O.tau_eigs_xy(p)
    e1 = 1.0 - lx.max() - ly.max()
    return (tx + ty) / e1, (tx + ty) / (e1 + p.d)


def assert_elementwise(out, ref, mask, bar, what="", kappa=(0.0, 0.0), eps=0.0,
                       penalty_own_scale=True):
    """Entry-by-entry comparison, on the whole grid and separately on the domain
    (mask = 1) and on the penalty region (mask = 0):

        max |out - ref| <= (bar + eps kappa) * scale

    with scale the largest |ref| of the region (the whole grid for the penalty
    region when penalty_own_scale is False).  kappa = (domain, penalty) from
    precond_kappa, eps the rounding unit of the eigenvalue tables times the
    number of independent evaluations compared (2 for GPU against oracle)."""
    inside = np.asarray(mask).reshape(ref.shape).astype(bool)
    gmax = np.abs(ref).max()
    for name, sel, k in (("grid", np.ones_like(inside), kappa[0]), ("domain", inside, kappa[0]),
                         ("penalty", ~inside, kappa[1])):
        if not sel.any():
            continue
        err = np.abs(out - ref)[sel].max()
        scale = np.abs(ref)[sel].max() if (name != "penalty" or penalty_own_scale) else gmax
        lim = (bar + eps * k) * scale
        assert err <= lim, f"{what} {name}: max err {err:.3e} > {lim:.3e} (scale {scale:.3e})"


def assert_precond(out, ref, p, precision, what=""):
    """The preconditioner bars: FP64 internals 1e-12 plus the eigenvalue
    conditioning (2 eps kappa, both sides evaluate E1 in FP64), each region
    against its own scale; FP32 internals 2e-5 of the whole output's scale.  In
    FP32 the two fields (P1 for the domain, P2 for the penalty region) share
    one complex FFT per line pair, so the penalty region's rounding follows the
    domain field, which is larger by up to dt/eta."""
    if precision == "fp64":
        assert_elementwise(out, ref, p.mask, 1e-12, what, precond_kappa(p), 2 * EPS64)
    else:
        assert_elementwise(out, ref, p.mask, 2e-5, what, penalty_own_scale=False)

"""Seeded synthetic inputs for the three-dimensional form of the penalized
Riesz space-fractional diffusion solve (the extension to higher dimensions
that the paper leaves to future work in its concluding section).

Inputs only, as in ``configs``: interior grid coordinates, the convex-domain
indicator mask, a seeded initial field and the parameter set.

Array layout: row-major [n3][n2][n1] (x fastest, then y, then z), the
lexicographic ordering of Section 2 carried to a third index.

Fixed choices (the paper has no 3-D workload):
  * box [0,1]^3, T = 1, eta = 1e-6;
  * domain: an ellipsoid centred at (0.5, 0.5, 0.5) with semi-axes
    0.45 (x), 0.35 (y), 0.30 (z); a grid point on its surface counts as inside;
  * alpha = (1.6, 1.7, 1.8), k = (1, 1, 1), f(u) = u (1 - u);
  * u0 = sum of 6 Gaussian bumps A exp(-|p - c|^2 / (2 w^2)) times the mask,
    drawn with numpy.random.default_rng(seed): per bump the centre ~ U[0,1]^3
    redrawn until inside the ellipsoid, then w ~ U[0.04, 0.12], then
    A ~ U[0.5, 1];
  * GMRES(30), tolerance 1e-8, 16 steps.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

F_LOGISTIC = 1

_BOX3 = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
_CENTRE = (0.5, 0.5, 0.5)
_SEMI = (0.45, 0.35, 0.30)


@dataclass
class Workload3:
    name: str
    n1: int
    n2: int
    n3: int
    box: Tuple[float, float, float, float, float, float]  # (x_lo, x_hi, y_lo, y_hi, z_lo, z_hi)
    alpha1: float
    alpha2: float
    alpha3: float
    kx: float
    ky: float
    kz: float
    eta: float
    T: float
    m: int
    f_kind: int
    restart: int
    tol: float
    mask: np.ndarray  # uint8 [n3][n2][n1]
    u0: np.ndarray    # float64 [n3][n2][n1], zero outside the domain

    @property
    def dt(self) -> float:
        return self.T / self.m

    @property
    def N(self) -> int:
        return self.n1 * self.n2 * self.n3

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.n3, self.n2, self.n1)


def interior_coords3(n1: int, n2: int, n3: int, box):
    """Interior mesh points along x, y, z (i = 1..n on each axis)."""
    out = []
    for n, (lo, hi) in zip((n1, n2, n3), ((box[0], box[1]), (box[2], box[3]), (box[4], box[5]))):
        h = (hi - lo) / (n + 1)
        out.append(lo + h * np.arange(1, n + 1, dtype=np.float64))
    return tuple(out)


def _ellipsoid(P):
    return sum(((P[a] - _CENTRE[a]) / _SEMI[a]) ** 2 for a in range(3))


def ellipsoid_mask(n1: int, n2: int, n3: int, box=_BOX3) -> np.ndarray:
    x, y, z = interior_coords3(n1, n2, n3, box)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return (_ellipsoid((X, Y, Z)) <= 1.0).astype(np.uint8)


def bumps3(n1: int, n2: int, n3: int, nbumps: int, seed: int, mask: np.ndarray,
           box=_BOX3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x, y, z = interior_coords3(n1, n2, n3, box)
    u = np.zeros((n3, n2, n1), dtype=np.float64)
    for _ in range(nbumps):
        while True:
            c = rng.random(3)
            if float(_ellipsoid(c)) <= 1.0:
                break
        w = rng.uniform(0.04, 0.12)
        A = rng.uniform(0.5, 1.0)
        gx = np.exp(-((x - c[0]) ** 2) / (2.0 * w * w))
        gy = np.exp(-((y - c[1]) ** 2) / (2.0 * w * w))
        gz = np.exp(-((z - c[2]) ** 2) / (2.0 * w * w))
        u += A * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return u * mask


def make_config3d(n: Optional[int] = None, m: Optional[int] = None, seed: int = 0,
                  shape: Optional[Tuple[int, int, int]] = None, kz: float = 1.0) -> Workload3:
    """The 3-D workload "e3": n^3 (default 255^3) or an explicit (n1, n2, n3)."""
    if shape is None:
        nn = 255 if n is None else n
        n1 = n2 = n3 = nn
    else:
        n1, n2, n3 = shape
    mask = ellipsoid_mask(n1, n2, n3)
    u0 = bumps3(n1, n2, n3, 6, seed, mask)
    return Workload3("e3", n1, n2, n3, _BOX3, 1.6, 1.7, 1.8, 1.0, 1.0, kz, 1e-6, 1.0,
                     16 if m is None else m, F_LOGISTIC, 30, 1e-8, mask, u0)

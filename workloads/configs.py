"""Named synthetic workloads for the penalized 2D Riesz space-fractional diffusion solve.

Everything here is input construction: interior grid coordinates (the uniform
mesh of Section 2 of the paper, points x_i = a + i*h_x, i = 1..n1), convex-domain
indicator masks, seeded Gaussian-bump initial fields and the parameter sets
of the benchmark workloads.  The same arrays are handed to the oracle and to
the HIP library, so both sides see bit-identical inputs.

Array layout: row-major [n2][n1] (x fastest), matching the lexicographic
ordering of the unknowns in Section 2 of the paper.

Unstated details are fixed as follows:
  * all domains are centred at (0.5, 0.5) inside the box [0,1]^2, T = 1;
  * a grid point exactly on the boundary counts as inside (closed domain);
  * a Gaussian bump is A*exp(-((x-cx)^2+(y-cy)^2)/(2 w^2));
  * bumps are drawn with numpy.random.default_rng(seed) (PCG64), per bump in
    the order: centre ~ U[0,1]^2 redrawn until inside the continuous domain,
    then w ~ U[0.02, 0.1], then A ~ U[0.5, 1];
  * the regular hexagon has a vertex on the +x axis.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, Optional, Tuple

import numpy as np

# Source-term kinds understood by both sides (f depends on u only).
F_NONE = 0       # f(u) = 0
F_LOGISTIC = 1   # f(u) = u (1 - u)
F_SIN = 2        # f(u) = sin(u)
F_CUBIC = 3      # f(u) = u - u^3
F_DECAY = 4      # f(u) = -u (Example 1, with a source field)

F_KIND_NAMES = {F_NONE: "0", F_LOGISTIC: "u(1-u)", F_SIN: "sin(u)", F_CUBIC: "u-u^3",
                F_DECAY: "-u"}


@dataclass
class Workload:
    name: str
    n1: int
    n2: int
    box: Tuple[float, float, float, float]  # (x_lo, x_hi, y_lo, y_hi)
    alpha1: float
    alpha2: float
    kx: float
    ky: float
    eta: float
    T: float
    m: int
    f_kind: int
    restart: int
    tol: float
    mask: np.ndarray   # uint8 [n2][n1], 1 = grid point inside the convex domain
    u0: np.ndarray     # float64 [n2][n1], zero outside the domain
    precisions: Tuple[str, ...] = ("fp64",)
    extra: Dict = field(default_factory=dict)

    @property
    def dt(self) -> float:
        return self.T / self.m

    @property
    def N(self) -> int:
        return self.n1 * self.n2


def interior_coords(n1: int, n2: int, box) -> Tuple[np.ndarray, np.ndarray]:
    """Interior mesh points x_i (i=1..n1) and y_j (j=1..n2) as 1-D arrays."""
    x_lo, x_hi, y_lo, y_hi = box
    hx = (x_hi - x_lo) / (n1 + 1)
    hy = (y_hi - y_lo) / (n2 + 1)
    x = x_lo + hx * np.arange(1, n1 + 1, dtype=np.float64)
    y = y_lo + hy * np.arange(1, n2 + 1, dtype=np.float64)
    return x, y


# ---------------------------------------------------------------------------
# Convex shapes: each returns F(x, y) with the closed domain = {F <= 1}.
# ---------------------------------------------------------------------------

def _disk(cx, cy, r) -> Callable:
    return lambda X, Y: ((X - cx) ** 2 + (Y - cy) ** 2) / (r * r)


def _ellipse(cx, cy, ax, ay, angle_deg=0.0) -> Callable:
    th = math.radians(angle_deg)
    c, s = math.cos(th), math.sin(th)

    def F(X, Y):
        dx, dy = X - cx, Y - cy
        xr = c * dx + s * dy
        yr = -s * dx + c * dy
        return (xr / ax) ** 2 + (yr / ay) ** 2
    return F


def _hexagon(cx, cy, R) -> Callable:
    # Regular hexagon, circumradius R, one vertex on the +x axis.
    def F(X, Y):
        ax_, ay_ = np.abs(X - cx), np.abs(Y - cy)
        return np.maximum(ay_ / (R * math.sqrt(3.0) / 2.0),
                          (math.sqrt(3.0) * ax_ + ay_) / (math.sqrt(3.0) * R))
    return F


SHAPES = {
    "disk": _disk,
    "ellipse": _ellipse,
    "hexagon": _hexagon,
}


def domain_mask(n1: int, n2: int, box, shape: Callable) -> np.ndarray:
    x, y = interior_coords(n1, n2, box)
    X, Y = np.meshgrid(x, y)  # [n2][n1]
    return (shape(X, Y) <= 1.0).astype(np.uint8)


def gaussian_bumps(n1: int, n2: int, box, shape: Callable, nbumps: int, seed: int,
                   mask: Optional[np.ndarray] = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x, y = interior_coords(n1, n2, box)
    X, Y = np.meshgrid(x, y)
    u = np.zeros((n2, n1), dtype=np.float64)
    for _ in range(nbumps):
        while True:
            c = rng.random(2)
            if float(shape(np.float64(c[0]), np.float64(c[1]))) <= 1.0:
                break
        w = rng.uniform(0.02, 0.1)
        A = rng.uniform(0.5, 1.0)
        u += A * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2.0 * w * w))
    if mask is None:
        mask = domain_mask(n1, n2, box, shape)
    return u * mask


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")

_UNIT = (0.0, 1.0, 0.0, 1.0)


def make_config(name: str, n: Optional[int] = None, m: Optional[int] = None,
                seed: int = 0) -> Workload:
    """Build one of the five benchmark workloads, optionally at another size.

    c1: disk r=0.45, a=(1.5,1.7), k=(1,1), 63^2, 16 steps, u0=exp(-40 r^2), GMRES(20) 1e-10
    c2: ellipse .45/.30, a=(1.2,1.8), k=(1,.5), 1023^2, 64 steps, 8 bumps, GMRES(30) 1e-8
    c3: ellipse .45/.25 rotated 30 deg, a=(1.9,1.9), 2047^2, 32 steps, sin u, FGMRES(30) 1e-8
    c4: disk r=0.40, a=(1.3,1.6), 511^2, 32 steps, u(1-u), adjoint workload
    c5: hexagon R=.45, a=(1.4,1.75), 4095^2, 16 steps, u-u^3, FGMRES(20) 1e-8
    """
    if name == "c1":
        nn = 63 if n is None else n
        shape = _disk(0.5, 0.5, 0.45)
        mask = domain_mask(nn, nn, _UNIT, shape)
        x, y = interior_coords(nn, nn, _UNIT)
        X, Y = np.meshgrid(x, y)
        u0 = np.exp(-40.0 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2)) * mask
        return Workload("c1", nn, nn, _UNIT, 1.5, 1.7, 1.0, 1.0, 1e-6, 1.0,
                        16 if m is None else m, F_LOGISTIC, 20, 1e-10, mask, u0)
    if name == "c2":
        nn = 1023 if n is None else n
        shape = _ellipse(0.5, 0.5, 0.45, 0.30)
        mask = domain_mask(nn, nn, _UNIT, shape)
        u0 = gaussian_bumps(nn, nn, _UNIT, shape, 8, seed, mask)
        return Workload("c2", nn, nn, _UNIT, 1.2, 1.8, 1.0, 0.5, 1e-6, 1.0,
                        64 if m is None else m, F_LOGISTIC, 30, 1e-8, mask, u0)
    if name == "c3":
        nn = 2047 if n is None else n
        shape = _ellipse(0.5, 0.5, 0.45, 0.25, 30.0)
        mask = domain_mask(nn, nn, _UNIT, shape)
        u0 = gaussian_bumps(nn, nn, _UNIT, shape, 8, seed, mask)
        return Workload("c3", nn, nn, _UNIT, 1.9, 1.9, 1.0, 1.0, 1e-6, 1.0,
                        32 if m is None else m, F_SIN, 30, 1e-8, mask, u0,
                        precisions=("fp64", "fp32", "bf16"))
    if name == "c4":
        nn = 511 if n is None else n
        shape = _disk(0.5, 0.5, 0.40)
        mask = domain_mask(nn, nn, _UNIT, shape)
        u0 = gaussian_bumps(nn, nn, _UNIT, shape, 8, seed, mask)
        return Workload("c4", nn, nn, _UNIT, 1.3, 1.6, 1.0, 1.0, 1e-6, 1.0,
                        32 if m is None else m, F_LOGISTIC, 30, 1e-8, mask, u0,
                        extra={"target_k": (1.2, 0.8), "fd_h": 1e-6, "fd_dirs": 16})
    if name == "c5":
        nn = 4095 if n is None else n
        shape = _hexagon(0.5, 0.5, 0.45)
        mask = domain_mask(nn, nn, _UNIT, shape)
        u0 = gaussian_bumps(nn, nn, _UNIT, shape, 8, seed, mask)
        return Workload("c5", nn, nn, _UNIT, 1.4, 1.75, 1.0, 1.0, 1e-6, 1.0,
                        16 if m is None else m, F_CUBIC, 20, 1e-8, mask, u0,
                        precisions=("fp32",))
    raise ValueError(f"unknown workload {name!r}")


def fd_direction(N_shape, i: int):
    """Seeded finite-difference direction i: (du, dkx, dky), |du|_2 = 1."""
    rng = np.random.default_rng(1000 + i)
    du = rng.standard_normal(N_shape)
    du /= np.linalg.norm(du)
    dk = rng.standard_normal(2)
    return du, float(dk[0]), float(dk[1])


# ---------------------------------------------------------------------------
# The paper's own workload (Example 1): ellipse with semi-axes a=2, b=1
# inscribed in the rectangle (0,2a) x (0,2b).
# ---------------------------------------------------------------------------

def example1_workload(n: int, kx: float, eta: float = 1e-5, T: float = 1.0,
                      m: Optional[int] = None, a: float = 2.0, b: float = 1.0) -> Workload:
    """Example 1 of Section 5: ellipse (a, b) inscribed in (0, 2a) x (0, 2b),
    alpha = (1.4, 1.7), kx = ky, n1 = n2 = n, m = n steps by default, GMRES(20),
    tol 1e-8.  f = -u + e^{-t} g0 (F_DECAY plus the field extra["src"] = g0);
    extra["exact0"] = u_e at t = 0 (u_e(t) = e^{-t} exact0)."""
    from .example1 import example1_exact, example1_source_field
    box = (0.0, 2.0 * a, 0.0, 2.0 * b)
    shape = _ellipse(a, b, a, b)
    mask = domain_mask(n, n, box, shape)
    x, y = interior_coords(n, n, box)
    X, Y = np.meshgrid(x, y)
    u0 = ((X - a) ** 2 / a ** 2 + (Y - b) ** 2 / b ** 2 - 1.0) ** 2 * mask
    steps = (n if m is None else m)
    src = example1_source_field(X, Y, 1.4, 1.7, kx, kx, a, b)
    return Workload("example1", n, n, box, 1.4, 1.7, kx, kx, eta, T, steps, F_DECAY,
                    20, 1e-8, mask, u0,
                    extra={"a": a, "b": b, "src": src, "exact0": example1_exact(X, Y, 0.0, a, b)})

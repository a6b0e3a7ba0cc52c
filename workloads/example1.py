"""Input fields of Example 1 of Section 5 (the paper's own test problem).

The exact solution on the ellipse ((x-a)/a)^2 + ((y-b)/b)^2 <= 1 inscribed in
the box (0, 2a) x (0, 2b) is u_e = e^{-t} (((x-a)/a)^2 + ((y-b)/b)^2 - 1)^2
(zero outside), and the right-hand side is f(u, x, y, t) = -u + e^{-t} g0(x, y),
with g0 the manufactured part that makes u_e solve the equation.  These are
problem data (the PDE's source and reference solution), not part of the
numerical method: the same arrays go to the oracle and to the HIP library.

Derivation of g0 (the example's printed formula is garbled; this reading
reproduces Tables 1-3).  On the chord through (x, y) along x, u_e is
e^{-t} a^{-4} s^2 (2c - s)^2 with s the distance to the left end of the chord
and c its half length, so by the Riemann-Liouville power rule
D^alpha s^p = Gamma(p+1)/Gamma(p+1-alpha) s^{p-alpha}, the left and right
derivatives are e^{-t} a^{-4} h(alpha, s, c) and e^{-t} a^{-4} h(alpha, 2c-s, c),
  h(alpha, s, c) = 24 s^{4-alpha}/Gamma(5-alpha) - 24 c s^{3-alpha}/Gamma(4-alpha)
                   + 8 c^2 s^{2-alpha}/Gamma(3-alpha).
The Riesz derivative is c_alpha (left + right), c_alpha = -1/(2 cos(alpha pi/2)),
and u_t = -u_e, so g0 = -kx c_alpha1 a^{-4} [h_x(left) + h_x(right)]
                        - ky c_alpha2 b^{-4} [h_y(bottom) + h_y(top)].
"""

from __future__ import annotations

import math

import numpy as np


def example1_exact(X, Y, t, a=2.0, b=1.0):
    """u_e(x, y, t) on grid arrays X, Y (zero outside the ellipse)."""
    q = (X - a) ** 2 / a ** 2 + (Y - b) ** 2 / b ** 2
    return np.where(q <= 1.0, math.exp(-t) * (q - 1.0) ** 2, 0.0)


def _h(alpha, s, c):
    s = np.maximum(s, 0.0)
    return (24.0 * s ** (4.0 - alpha) / math.gamma(5.0 - alpha)
            - 24.0 * c * s ** (3.0 - alpha) / math.gamma(4.0 - alpha)
            + 8.0 * c * c * s ** (2.0 - alpha) / math.gamma(3.0 - alpha))


def example1_source_field(X, Y, alpha1, alpha2, kx, ky, a=2.0, b=1.0):
    """g0(x, y): the source is f = -u + e^{-t} g0 inside the ellipse, 0 outside."""
    q = (X - a) ** 2 / a ** 2 + (Y - b) ** 2 / b ** 2
    inside = q <= 1.0
    cx = a * np.sqrt(np.maximum(1.0 - (Y - b) ** 2 / b ** 2, 0.0))  # half chord along x
    cy = b * np.sqrt(np.maximum(1.0 - (X - a) ** 2 / a ** 2, 0.0))  # half chord along y
    ca1 = -1.0 / (2.0 * math.cos(alpha1 * math.pi / 2.0))
    ca2 = -1.0 / (2.0 * math.cos(alpha2 * math.pi / 2.0))
    rx = ca1 * a ** -4 * (_h(alpha1, X - a + cx, cx) + _h(alpha1, a + cx - X, cx))
    ry = ca2 * b ** -4 * (_h(alpha2, Y - b + cy, cy) + _h(alpha2, b + cy - Y, cy))
    return np.where(inside, -kx * rx - ky * ry, 0.0)

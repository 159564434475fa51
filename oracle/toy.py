"""Three-circle product-space toy (Introduction: three non-convex sets S, T, U
in the plane, divide and concur over three copies of the plane).

TEST INFRASTRUCTURE ONLY (see pty_oracle).  Points are complex numbers
standing for (x, y) in the plane; the product-space iterate is an array of
three of them, one per constraint set.
"""
from __future__ import annotations

import numpy as np

from .pty_oracle import abc_iteration


def circle_projection(center: complex, radius: float):
    """Nearest point of the circle |p - center| = radius (the centre maps to angle 0)."""
    def proj(p):
        d = p - center
        m = abs(d)
        if m == 0:
            return center + radius
        return center + radius * d / m
    return proj


class ThreeCircles:
    def __init__(self, centers, radii):
        self.projs = [circle_projection(complex(cc), float(r)) for cc, r in zip(centers, radii)]

    def divide(self, x):
        """P_D x = [P_S x^S, P_T x^T, P_U x^U]."""
        return np.array([pr(v) for pr, v in zip(self.projs, x)], dtype=np.complex128)

    @staticmethod
    def concur(x):
        """P_C x = (x^S + x^T + x^U) / 3 in every copy."""
        m = np.sum(x) / len(x)
        return np.full(len(x), m, dtype=np.complex128)

    def step(self, x, a, b, c):
        x_next, _ = abc_iteration(np.asarray(x, dtype=np.complex128), self.divide,
                                  self.concur, a, b, c)
        return x_next

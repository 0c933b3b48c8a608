"""Brute-force minimiser of 1/2 c.Kc - c.F s.t. c >= 0 for N <= 12 (numpy).

TEST INFRASTRUCTURE ONLY.  For every subset A of the DOFs it solves the dense
face system K_FF c_F = F_F with c_A = 0 and keeps the subsets whose point
satisfies the KKT conditions c >= 0, g = Kc - F >= 0 on A (Sec. 2.1.3,
eq. non-negative: the minimiser is unique because K is positive definite).
"""
from __future__ import annotations

import itertools

import numpy as np


def brute_force(K: np.ndarray, F: np.ndarray, tol: float = 1e-13):
    """Return (c, survivors): the KKT point and the list of active sets that
    produce it.  Raises if two surviving sets give different points."""
    K = np.asarray(K, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    n = F.size
    if n > 12:
        raise ValueError("brute force is limited to N <= 12")
    scale_c = None
    found = []
    for r in range(n + 1):
        for A in itertools.combinations(range(n), r):
            act = np.zeros(n, dtype=bool)
            act[list(A)] = True
            free = ~act
            c = np.zeros(n)
            if free.any():
                c[free] = np.linalg.solve(K[np.ix_(free, free)], F[free])
            g = K @ c - F
            cs = max(1.0, float(np.abs(c).max()))
            gs = max(1e-300, float(np.abs(F).max()))
            if (c[free] >= -tol * cs).all() and (g[act] >= -tol * gs).all():
                found.append((A, np.maximum(c, 0.0)))
    if not found:
        raise RuntimeError("no KKT point found")
    c0 = found[0][1]
    scale_c = max(float(np.abs(c0).max()), 1e-300)
    for A, c in found[1:]:
        if np.abs(c - c0).max() > 1e-13 * scale_c:
            raise RuntimeError("two active sets give different KKT points")
    return c0, [A for A, _ in found]

"""Brute-force minimiser of 1/2 c.Kc - c.F s.t. lo <= c <= hi for small N (numpy).

TEST INFRASTRUCTURE ONLY.  Every variable is either at the lower bound, at
the upper bound (when finite) or free; for every such assignment it solves the
dense face system K_FF c_F = F_F - K_FB c_B with c_B at its bounds, and keeps
the assignments whose point satisfies the KKT conditions: lo <= c <= hi,
g = Kc - F >= 0 where c = lo, g <= 0 where c = hi (Sec. 2.1.3, eq.
non-negative; Sec. 2.2.2, eq. Eq:non-negative: the minimiser is unique because
K is positive definite).
"""
from __future__ import annotations

import itertools

import numpy as np


def brute_force(K: np.ndarray, F: np.ndarray, tol: float = 1e-13, lo: float = 0.0,
                hi: float = np.inf):
    """Return (c, survivors): the KKT point and the list of assignments
    (tuples of 0 = lower, 1 = free, 2 = upper; for hi = inf the tuple of
    variables at the lower bound) that produce it.  Raises if two surviving
    assignments give different points."""
    K = np.asarray(K, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    n = F.size
    if n > 12 or (np.isfinite(hi) and n > 9):
        raise ValueError("brute force is limited to N <= 12 (N <= 9 with an upper bound)")
    if np.isfinite(hi):
        assignments = itertools.product((0, 1, 2), repeat=n)
    else:
        assignments = (tuple(0 if i in A else 1 for i in range(n))
                       for r in range(n + 1) for A in itertools.combinations(range(n), r))
    found = []
    for a in assignments:
        a = np.array(a, dtype=np.int8)
        free = a == 1
        c = np.where(a == 0, lo, hi).astype(np.float64)
        c[free] = 0.0
        if free.any():
            fixed = ~free
            rhs = F[free] - K[np.ix_(free, fixed)] @ c[fixed]
            c[free] = np.linalg.solve(K[np.ix_(free, free)], rhs)
        g = K @ c - F
        cs = max(1.0, float(np.abs(c).max()))
        gs = max(1e-300, float(np.abs(F).max()), float(np.abs(g).max()) * 1e-3)
        ok = (c[free] >= lo - tol * cs).all() and (c[free] <= hi + tol * cs).all()
        ok = ok and (g[a == 0] >= -tol * gs).all() and (g[a == 2] <= tol * gs).all()
        if ok:
            key = tuple(a.tolist()) if np.isfinite(hi) else tuple(np.flatnonzero(a == 0).tolist())
            found.append((key, np.clip(c, lo, hi)))
    if not found:
        raise RuntimeError("no KKT point found")
    c0 = found[0][1]
    scale_c = max(float(np.abs(c0).max()), 1e-300)
    for _, c in found[1:]:
        if np.abs(c - c0).max() > 1e-12 * scale_c:
            raise RuntimeError("two assignments give different KKT points")
    return c0, [k for k, _ in found]

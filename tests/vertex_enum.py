"""Brute-force LP optimum by vertex enumeration (textbook; tiny problems only).

The LP  min c'x  s.t.  Gx >= h, Ax = b, l <= x <= u  is written with surplus
variables s >= 0 as  [G -I; A 0] (x, s) = (h, b).  Every basic solution picks
m basic columns, fixes each non-basic variable at one of its finite bounds,
and solves for the basic ones; the optimum of a bounded feasible LP with a
vertex is the best feasible basic solution.
"""
import itertools

import numpy as np


def vertex_optimum(K, row_type, rhs, c, l, u, tol=1e-9):
    K = np.asarray(K, dtype=float)
    m, n = K.shape
    ge = [i for i in range(m) if row_type[i] == 0]
    ns = len(ge)
    M = np.zeros((m, n + ns))
    M[:, :n] = K
    for k, i in enumerate(ge):
        M[i, n + k] = -1.0
    lo = np.concatenate([l, np.zeros(ns)])
    hi = np.concatenate([u, np.full(ns, np.inf)])
    cc = np.concatenate([c, np.zeros(ns)])
    N = n + ns
    best, best_x = np.inf, None
    for basis in itertools.combinations(range(N), m):
        B = M[:, basis]
        if abs(np.linalg.det(B)) < 1e-10:
            continue
        nb = [j for j in range(N) if j not in basis]
        choices = []
        ok = True
        for j in nb:
            opts = [v for v in (lo[j], hi[j]) if np.isfinite(v)]
            if not opts:
                ok = False
                break
            choices.append(opts)
        if not ok:
            continue
        for vals in itertools.product(*choices):
            z = np.zeros(N)
            z[nb] = vals
            rhs_b = rhs - M[:, nb] @ np.asarray(vals, dtype=float) if nb else np.asarray(rhs, float)
            zb = np.linalg.solve(B, rhs_b)
            z[list(basis)] = zb
            if np.all(z >= lo - tol) and np.all(z <= hi + tol):
                f = cc @ z
                if f < best:
                    best, best_x = f, z[:n].copy()
    return best, best_x

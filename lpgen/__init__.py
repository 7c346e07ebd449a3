"""Seeded synthetic LP instances for the PDHG hot path.

This module only *builds problem data*: it draws random matrices, bounds and
planted optimal primal-dual pairs with NumPy's PCG64 generator.  It contains
none of the PDHG method's arithmetic and is shared by the FP64 oracle tests,
the GPU tests and the benchmark as the single source of inputs.

Problem statement (paper, Section 2.2 "Linear Programming"):

    min c^T x   s.t.  G x >= h,  A x = b,  l <= x <= u

An instance stores the rows of G and A interleaved in any order, with
``row_type[i] = GE (0)`` for a ">=" row and ``EQ (1)`` for an "=" row, and
``rhs[i]`` the matching entry of h or b.  Both solver paths reorder the rows
so that the inequality rows come first (the stacked K = [G; A], q = [h; b]).

Planted optima (used by C0, C0u, C2, C3 and the tiny cases) follow the
Lagrangian dual of Appendix B: with y* feasible (y*_ineq >= 0) and reduced
costs z = c - K^T y* that vanish on interior variables, are >= 0 on variables
at their lower bound and <= 0 at their upper bound, (x*, y*) is optimal and
f* = c^T x* = q^T y* + sum_{x*_i = u_i} u_i z_i.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

GE = 0
EQ = 1


@dataclasses.dataclass
class LP:
    """One LP in CSR form, rows in user order (see module docstring)."""

    n: int
    m: int
    rowptr: np.ndarray  # int64, m + 1
    col: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz
    row_type: np.ndarray  # uint8, m (GE / EQ)
    rhs: np.ndarray  # float64, m
    c: np.ndarray  # float64, n
    l: np.ndarray  # float64, n (may hold -inf)
    u: np.ndarray  # float64, n (may hold +inf)
    name: str = "lp"
    x_star: Optional[np.ndarray] = None
    y_star: Optional[np.ndarray] = None  # user row order
    f_star: Optional[float] = None

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def m_ineq(self) -> int:
        return int(np.count_nonzero(self.row_type == GE))

    def dense(self) -> np.ndarray:
        a = np.zeros((self.m, self.n))
        for i in range(self.m):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            a[i, self.col[s:e]] += self.val[s:e]
        return a

    def scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.m, self.n))

    def save(self, path: str) -> None:
        extra = {}
        if self.x_star is not None:
            extra["x_star"] = self.x_star
        if self.y_star is not None:
            extra["y_star"] = self.y_star
        if self.f_star is not None:
            extra["f_star"] = np.array([self.f_star])
        np.savez(path, n=self.n, m=self.m, rowptr=self.rowptr, col=self.col, val=self.val,
                 row_type=self.row_type, rhs=self.rhs, c=self.c, l=self.l, u=self.u, **extra)

    @staticmethod
    def load(path: str) -> "LP":
        z = np.load(path)  # allow_pickle stays False
        f = z["f_star"][0] if "f_star" in z else None
        return LP(int(z["n"]), int(z["m"]), z["rowptr"], z["col"], z["val"], z["row_type"],
                  z["rhs"], z["c"], z["l"], z["u"], x_star=z["x_star"] if "x_star" in z else None,
                  y_star=z["y_star"] if "y_star" in z else None, f_star=f)


# ---------------------------------------------------------------------------
# sparse pattern helpers
# ---------------------------------------------------------------------------

def _csr_from_coo(m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Sorted CSR (row-major, columns increasing) from COO with unique (row, col)."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols.astype(np.int32), vals.astype(np.float64)


def _rows_with_lengths(rng: np.random.Generator, lengths: np.ndarray, n: int):
    """Row indices and distinct uniform column indices for given row lengths.

    Columns are drawn with replacement and duplicates inside a row are dropped,
    so a row may come out slightly shorter than asked (rare for short rows of a
    wide matrix); this is the only approximation to "without replacement".
    """
    m = lengths.shape[0]
    rows = np.repeat(np.arange(m, dtype=np.int64), lengths)
    cols = rng.integers(0, n, size=rows.shape[0], dtype=np.int64)
    key = rows * n + cols
    key = np.unique(key)
    return key // n, key % n


def _bernoulli_pattern(rng: np.random.Generator, m: int, n: int, density: float):
    """Each (i, j) nonzero independently with probability ``density``."""
    if m * n <= 4_000_000:
        mask = rng.random((m, n)) < density
        r, cidx = np.nonzero(mask)
        return r.astype(np.int64), cidx.astype(np.int64)
    lengths = rng.binomial(n, density, size=m)
    return _rows_with_lengths(rng, lengths, n)


# ---------------------------------------------------------------------------
# planted-optimum random LPs (configs C0, C0u, C2, C3)
# ---------------------------------------------------------------------------

def _plant(rng, n, rowptr, col, val, row_type, u, frac_zero=0.5, frac_int=0.4,
           frac_active_ge=0.5):
    """Choose x*, y*, z and return (rhs, c, x*, y*, f*) so that (x*, y*) is optimal."""
    m = row_type.shape[0]
    perm = rng.permutation(n)
    n0 = int(round(frac_zero * n))
    ni = int(round(frac_int * n))
    at0, inter, atu = perm[:n0], perm[n0:n0 + ni], perm[n0 + ni:]
    x = np.zeros(n)
    x[inter] = rng.uniform(0.0, 1.0, size=inter.shape[0]) * u[inter]
    x[atu] = u[atu]
    z = np.zeros(n)
    z[at0] = np.abs(rng.standard_normal(at0.shape[0]))
    z[atu] = -np.abs(rng.standard_normal(atu.shape[0]))
    y = rng.standard_normal(m)
    ge = np.nonzero(row_type == GE)[0]
    active = rng.random(ge.shape[0]) < frac_active_ge
    y[ge[active]] = np.abs(y[ge[active]])
    y[ge[~active]] = 0.0
    import scipy.sparse as sp

    a = sp.csr_matrix((val, col, rowptr), shape=(m, n))
    ax = a @ x
    rhs = ax.copy()
    slack = rng.uniform(0.1, 1.0, size=ge.shape[0])
    rhs[ge[~active]] = ax[ge[~active]] - slack[~active]
    c = a.T @ y + z
    f = float(c @ x)
    return rhs, c, x, y, f, (at0, inter, atu)


def planted(m: int, n: int, density: float, seed: int, ge_frac: float = 0.0,
            u_range=(1.0, 10.0), unique: bool = False, name: str = "planted") -> LP:
    """Random sparse LP with a planted optimal pair (the recipe of C0 and C3).

    Entries of K are nonzero with probability ``density`` and N(0,1) valued,
    0 <= x <= u with u ~ U(u_range), x* half at 0, 40% interior, 10% at u,
    y* ~ N(0,1) on "=" rows.  ``ge_frac`` of the rows are ">=" rows (i.i.d.,
    interleaved), half of them active with y* = |N(0,1)|, the rest inactive
    with slack U(0.1, 1).  ``unique`` (variant C0u) adds one forced nonzero per
    interior column on distinct rows so the optimal basis is nonsingular.
    """
    rng = np.random.default_rng(seed)
    r, cidx = _bernoulli_pattern(rng, m, n, density)
    row_type = np.where(rng.random(m) < ge_frac, GE, EQ).astype(np.uint8)
    u = rng.uniform(u_range[0], u_range[1], size=n)
    # the planting permutation is drawn from a child generator so that the
    # matching below can be placed before values are drawn
    prng = np.random.default_rng(rng.integers(1 << 62))
    if unique:
        perm = prng.permutation(n)
        n0, ni = int(round(0.5 * n)), int(round(0.4 * n))
        inter = perm[n0:n0 + ni]
        k = min(ni, m)
        rows_forced = rng.permutation(m)[:k]
        r = np.concatenate([r, rows_forced.astype(np.int64)])
        cidx = np.concatenate([cidx, inter[:k].astype(np.int64)])
        key = np.unique(r * n + cidx)
        r, cidx = key // n, key % n
        prng = np.random.default_rng(prng.bit_generator.seed_seq)  # replay the same draws
    vals = rng.standard_normal(r.shape[0])
    rowptr, col, val = _csr_from_coo(m, r, cidx, vals)
    rhs, c, x, y, f, _ = _plant(prng, n, rowptr, col, val, row_type, u)
    l = np.zeros(n)
    return LP(n, m, rowptr, col, val, row_type, rhs, c, l, u, name=name,
              x_star=x, y_star=y, f_star=f)


def config0(seed: int = 0, unique: bool = False) -> LP:
    """C0: m=200 "=" rows, n=500, density 2%, plain PDHG in FP64."""
    return planted(200, 500, 0.02, seed, unique=unique, name="C0u" if unique else "C0")


def zipf_lengths(rng, m: int, s: float, kmax: int) -> np.ndarray:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** (-s)
    p /= p.sum()
    return rng.choice(np.arange(1, kmax + 1), size=m, p=p)


def zipf_mean(s: float, kmax: int) -> float:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** (-s)
    return float((k * p).sum() / p.sum())


def config2(seed: int = 2, m: int = 1_000_000, n: int = 2_000_000, s: float = 1.5,
            kmax: int = 5000) -> LP:
    """C2: large random LP, power-law (Zipf) row lengths, mixed (=, >=) rows."""
    rng = np.random.default_rng(seed)
    lengths = zipf_lengths(rng, m, s, kmax)
    r, cidx = _rows_with_lengths(rng, lengths, n)
    vals = rng.standard_normal(r.shape[0])
    rowptr, col, val = _csr_from_coo(m, r, cidx, vals)
    del r, cidx, vals
    row_type = np.where(rng.random(m) < 0.5, GE, EQ).astype(np.uint8)
    u = rng.uniform(1.0, 10.0, size=n)
    rhs, c, x, y, f, _ = _plant(rng, n, rowptr, col, val, row_type, u)
    return LP(n, m, rowptr, col, val, row_type, rhs, c, np.zeros(n), u, name=f"C2(m={m},n={n},s={s})",
              x_star=x, y_star=y, f_star=f)


def config3_instance(i: int, m_range=(1000, 50000), density_range=(0.001, 0.01)) -> LP:
    """C3 instance i: planted LP with m ~ U{m_range}, n = round(2.5 m), density ~ U(range)."""
    rng = np.random.default_rng(3000 + i)
    m = int(rng.integers(m_range[0], m_range[1] + 1))
    n = int(round(2.5 * m))
    d = float(rng.uniform(*density_range))
    return planted(m, n, d, int(rng.integers(1 << 62)), name=f"C3[{i}]")


# ---------------------------------------------------------------------------
# SCED-shaped LP (configs C1, C4)
# ---------------------------------------------------------------------------

def sced(G: int = 5000, B: int = 2000, T: int = 24, L: int = 125, seed: int = 1,
         name: str = "SCED") -> LP:
    """Synthetic security-constrained economic-dispatch-shaped LP.

    Variables (period-major blocks): p[t,g] in [0,Pmax], ramp deltas d[t,g]
    (t >= 1) in [-0.3Pmax, 0.3Pmax], up reserve r[t,g] in [0, 0.1Pmax], down
    reserve s[t,g] for the first G/2 generators in [0, 0.1Pmax], shed/spill
    per period in [0, inf), one flow slack per line-period in [0, inf).
    Rows: ramp equalities, headroom and footroom ">=", per-period balance "=",
    up/down reserve requirements ">=", and line-flow ">=" rows whose PTDF-like
    coefficients are U(-1,1) with |.| <= 0.05 zeroed.  Limits F_l are 0.9 x the
    largest |flow| of a network-blind merit-order dispatch, so some flows bind.
    Feasible (shed/slack) and bounded (every unbounded variable is penalised).
    """
    rng = np.random.default_rng(seed)
    Gd = G // 2
    bus = rng.integers(0, B, size=G)
    pmax = rng.uniform(50.0, 500.0, size=G)
    cost = rng.uniform(10.0, 100.0, size=G)
    cup = 0.1 * rng.uniform(10.0, 100.0, size=G)
    cdn = 0.1 * rng.uniform(10.0, 100.0, size=Gd)
    ptdf = rng.uniform(-1.0, 1.0, size=(L, B))
    ptdf[np.abs(ptdf) <= 0.05] = 0.0
    tt = np.arange(T)
    demand = 0.6 * pmax.sum() * (1.0 + 0.2 * np.sin(2.0 * math.pi * tt / T))

    # variable offsets
    o_p = 0
    o_d = o_p + T * G
    o_r = o_d + (T - 1) * G
    o_s = o_r + T * G
    o_shed = o_s + T * Gd
    o_spill = o_shed + T
    o_v = o_spill + T
    n = o_v + L * T
    c = np.zeros(n)
    lo = np.zeros(n)
    up = np.full(n, np.inf)
    for t in range(T):
        c[o_p + t * G:o_p + (t + 1) * G] = cost
        up[o_p + t * G:o_p + (t + 1) * G] = pmax
        c[o_r + t * G:o_r + (t + 1) * G] = cup
        up[o_r + t * G:o_r + (t + 1) * G] = 0.1 * pmax
        c[o_s + t * Gd:o_s + (t + 1) * Gd] = cdn
        up[o_s + t * Gd:o_s + (t + 1) * Gd] = 0.1 * pmax[:Gd]
    for t in range(T - 1):
        lo[o_d + t * G:o_d + (t + 1) * G] = -0.3 * pmax
        up[o_d + t * G:o_d + (t + 1) * G] = 0.3 * pmax
    c[o_shed:o_shed + T] = 1000.0
    c[o_spill:o_spill + T] = 1000.0
    c[o_v:o_v + L * T] = 1000.0

    rows, cols, vals, rtype, rhs = [], [], [], [], []
    r0 = 0

    def add(nrows, rr, cc, vv, typ, b):
        nonlocal r0
        rows.append(rr + r0)
        cols.append(cc)
        vals.append(vv)
        rtype.append(np.full(nrows, typ, dtype=np.uint8))
        rhs.append(b)
        r0 += nrows

    g = np.arange(G)
    # ramp: p[t,g] - p[t-1,g] - d[t,g] = 0, t = 1..T-1
    nr = (T - 1) * G
    ridx = np.arange(nr)
    t1 = ridx // G + 1
    gg = ridx % G
    add(nr, np.repeat(ridx, 3),
        np.stack([o_p + t1 * G + gg, o_p + (t1 - 1) * G + gg, o_d + (t1 - 1) * G + gg], 1).ravel(),
        np.tile([1.0, -1.0, -1.0], nr), EQ, np.zeros(nr))
    # headroom: -p[t,g] - r[t,g] >= -Pmax
    nr = T * G
    ridx = np.arange(nr)
    tg, gg = ridx // G, ridx % G
    add(nr, np.repeat(ridx, 2), np.stack([o_p + tg * G + gg, o_r + tg * G + gg], 1).ravel(),
        np.tile([-1.0, -1.0], nr), GE, -pmax[gg])
    # footroom: p[t,g] - s[t,g] >= 0, g < G/2
    nr = T * Gd
    ridx = np.arange(nr)
    tg, gg = ridx // Gd, ridx % Gd
    add(nr, np.repeat(ridx, 2), np.stack([o_p + tg * G + gg, o_s + tg * Gd + gg], 1).ravel(),
        np.tile([1.0, -1.0], nr), GE, np.zeros(nr))
    # balance: sum_g p[t,g] + shed_t - spill_t = D_t
    rr, cc, vv = [], [], []
    for t in range(T):
        rr.append(np.full(G + 2, t))
        cc.append(np.concatenate([o_p + t * G + g, [o_shed + t, o_spill + t]]))
        vv.append(np.concatenate([np.ones(G), [1.0, -1.0]]))
    add(T, np.concatenate(rr), np.concatenate(cc), np.concatenate(vv), EQ, demand.copy())
    # reserves: sum_g r[t,g] >= 0.03 D_t ; sum_{g<G/2} s[t,g] >= 0.03 D_t
    rr, cc, vv = [], [], []
    for t in range(T):
        rr.append(np.full(G, 2 * t))
        cc.append(o_r + t * G + g)
        vv.append(np.ones(G))
        rr.append(np.full(Gd, 2 * t + 1))
        cc.append(o_s + t * Gd + np.arange(Gd))
        vv.append(np.ones(Gd))
    add(2 * T, np.concatenate(rr), np.concatenate(cc), np.concatenate(vv), GE,
        np.repeat(0.03 * demand, 2))
    # merit-order dispatch for the flow limits
    order = np.argsort(cost, kind="stable")
    disp = np.zeros((T, G))
    for t in range(T):
        cum = np.cumsum(pmax[order])
        full = cum <= demand[t]
        disp[t, order[full]] = pmax[order[full]]
        k = int(np.count_nonzero(full))
        if k < G:
            disp[t, order[k]] = demand[t] - (cum[k - 1] if k > 0 else 0.0)
    coef = ptdf[:, bus]  # (L, G)
    flows = disp @ coef.T  # (T, L)
    flim = 0.9 * np.abs(flows).max(axis=0)
    # flow rows: -sum_g PTDF[l,bus(g)] p[t,g] + v[t,l] >= -F_l   (row order: t-major)
    nzl = [np.nonzero(coef[l])[0] for l in range(L)]
    rr, cc, vv, bb = [], [], [], []
    for t in range(T):
        for l in range(L):
            k = 2 * 0 + t * L + l
            gi = nzl[l]
            rr.append(np.full(gi.shape[0] + 1, k))
            cc.append(np.concatenate([o_p + t * G + gi, [o_v + t * L + l]]))
            vv.append(np.concatenate([-coef[l, gi], [1.0]]))
            bb.append(-flim[l])
    add(T * L, np.concatenate(rr), np.concatenate(cc), np.concatenate(vv), GE, np.array(bb))

    m = r0
    rows_a = np.concatenate(rows).astype(np.int64)
    cols_a = np.concatenate(cols).astype(np.int64)
    vals_a = np.concatenate(vals)
    rowptr, col, val = _csr_from_coo(m, rows_a, cols_a, vals_a)
    return LP(n, m, rowptr, col, val, np.concatenate(rtype), np.concatenate(rhs), c, lo, up,
              name=f"{name}(G={G},B={B},T={T},L={L})")


def config1(seed: int = 1) -> LP:
    """C1: SCED-shaped, 5000 generators, 2000 buses, 24 periods, 125 lines."""
    return sced(5000, 2000, 24, 125, seed=seed, name="C1")


def config4_instance(i: int) -> LP:
    """C4 instance i: SCED-shaped at 1/10 of C1 (500 generators, 200 buses)."""
    return sced(500, 200, 24, 125, seed=4000 + i, name=f"C4[{i}]")


# ---------------------------------------------------------------------------
# tiny LPs for brute-force vertex enumeration
# ---------------------------------------------------------------------------

def tiny(seed: int, n: int = 5, m: int = 3, ge_frac: float = 0.5, free_frac: float = 0.0) -> LP:
    """Dense tiny LP with a planted optimum; some bounds may be infinite.

    All variables have finite lower bounds unless ``free_frac`` > 0 picks some
    to be unbounded below with a finite upper bound (their z is then <= 0 and
    they are planted at u) or fully free (planted interior, z = 0).
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    row_type = np.where(rng.random(m) < ge_frac, GE, EQ).astype(np.uint8)
    l = rng.uniform(-2.0, 0.0, size=n)
    u = l + rng.uniform(1.0, 4.0, size=n)
    kind = rng.integers(0, 3, size=n)  # 0 at l, 1 interior, 2 at u
    x = np.where(kind == 0, l, np.where(kind == 2, u, l + rng.uniform(0.2, 0.8, size=n) * (u - l)))
    z = np.where(kind == 0, np.abs(rng.standard_normal(n)) + 0.1,
                 np.where(kind == 2, -np.abs(rng.standard_normal(n)) - 0.1, 0.0))
    if free_frac > 0:
        pick = rng.random(n) < free_frac
        l[pick & (kind == 2)] = -np.inf
        fr = pick & (kind == 1)
        l[fr] = -np.inf
        u[fr] = np.inf
    y = rng.standard_normal(m)
    ge = row_type == GE
    act = rng.random(m) < 0.6
    y[ge & act] = np.abs(y[ge & act]) + 0.1
    y[ge & ~act] = 0.0
    ax = a @ x
    rhs = ax - np.where(ge & ~act, rng.uniform(0.1, 1.0, size=m), 0.0)
    c = a.T @ y + z
    r, cc = np.nonzero(np.ones((m, n), dtype=bool))
    rowptr, col, val = _csr_from_coo(m, r.astype(np.int64), cc.astype(np.int64), a[r, cc])
    return LP(n, m, rowptr, col, val, row_type, rhs, c, l, u, name=f"tiny{seed}",
              x_star=x, y_star=y, f_star=float(c @ x))


def from_dense(a: np.ndarray, row_type, rhs, c, l, u, name="dense") -> LP:
    m, n = a.shape
    r, cc = np.nonzero(a != 0)
    rowptr, col, val = _csr_from_coo(m, r.astype(np.int64), cc.astype(np.int64), a[r, cc])
    return LP(n, m, rowptr, col, val, np.asarray(row_type, dtype=np.uint8),
              np.asarray(rhs, dtype=np.float64), np.asarray(c, dtype=np.float64),
              np.asarray(l, dtype=np.float64), np.asarray(u, dtype=np.float64), name=name)


# ---------------------------------------------------------------------------
# infeasible and unbounded LPs (Section 2.4.5 test cases)
# ---------------------------------------------------------------------------

def _append(lp: LP, rows, cols, vals, row_type, rhs, n_new: int = 0, c_new=(), l_new=(), u_new=(),
            name: str = "") -> LP:
    """lp with extra rows (COO entries with row indices counted from lp.m) and
    n_new extra columns (indices from lp.n)."""
    r0 = np.repeat(np.arange(lp.m, dtype=np.int64), np.diff(lp.rowptr))
    r = np.concatenate([r0, np.asarray(rows, dtype=np.int64)])
    cc = np.concatenate([np.asarray(lp.col, dtype=np.int64), np.asarray(cols, dtype=np.int64)])
    v = np.concatenate([np.asarray(lp.val), np.asarray(vals, dtype=np.float64)])
    m = lp.m + len(row_type)
    n = lp.n + n_new
    rowptr, col, val = _csr_from_coo(m, r, cc, v)
    return LP(n, m, rowptr, col, val,
              np.concatenate([lp.row_type, np.asarray(row_type, dtype=np.uint8)]),
              np.concatenate([lp.rhs, np.asarray(rhs, dtype=np.float64)]),
              np.concatenate([lp.c, np.asarray(c_new, dtype=np.float64)]),
              np.concatenate([lp.l, np.asarray(l_new, dtype=np.float64)]),
              np.concatenate([lp.u, np.asarray(u_new, dtype=np.float64)]), name=name or lp.name)


def primal_infeasible(m: int, n: int, density: float, seed: int, kind: str = "bound") -> LP:
    """A planted LP made infeasible.  kind "bound": one more ">=" row
    x_j >= u_j + 1 on a boxed variable j; kind "pair": a random sparse row a
    twice, as a x >= h and -a x >= 1 - h (so a x <= h - 1)."""
    base = planted(m, n, density, seed, ge_frac=0.5)
    rng = np.random.default_rng(seed + 7919)
    if kind == "bound":
        j = int(rng.integers(n))
        return _append(base, [m], [j], [1.0], [GE], [base.u[j] + 1.0], name=f"infeas-bound({m}x{n})")
    k = max(2, int(density * n))
    cols = rng.choice(n, size=k, replace=False)
    a = rng.standard_normal(k)
    h = float(rng.standard_normal())
    return _append(base, [m] * k + [m + 1] * k, list(cols) * 2, list(a) + list(-a), [GE, GE],
                   [h, 1.0 - h], name=f"infeas-pair({m}x{n})")


def dual_infeasible(m: int, n: int, density: float, seed: int) -> LP:
    """A planted LP made unbounded: one more variable t >= 0 (no upper bound)
    with cost -1 that appears only in ">=" rows, with positive coefficients,
    so x* + s e_t is feasible for every s >= 0 and the objective falls without
    bound."""
    base = planted(m, n, density, seed, ge_frac=0.5)
    rng = np.random.default_rng(seed + 104729)
    ge = np.nonzero(base.row_type == GE)[0]
    k = max(1, min(len(ge), int(round(density * m)) + 1))
    rows = rng.choice(ge, size=k, replace=False) if len(ge) else np.zeros(0, dtype=np.int64)
    vals = rng.uniform(0.5, 2.0, size=len(rows))
    out = _append(base, [], [], [], [], [], name=f"unbounded({m}x{n})")
    # the new column: rebuild with its entries
    r0 = np.repeat(np.arange(out.m, dtype=np.int64), np.diff(out.rowptr))
    r = np.concatenate([r0, rows.astype(np.int64)])
    cc = np.concatenate([np.asarray(out.col, dtype=np.int64), np.full(len(rows), n, dtype=np.int64)])
    v = np.concatenate([np.asarray(out.val), vals])
    rowptr, col, val = _csr_from_coo(out.m, r, cc, v)
    return LP(n + 1, out.m, rowptr, col, val, out.row_type, out.rhs, np.append(out.c, -1.0),
              np.append(out.l, 0.0), np.append(out.u, np.inf), name=out.name)


# ---------------------------------------------------------------------------
# random draws of the fishnet multi-start (Section 2.5), passed to both paths
# ---------------------------------------------------------------------------

def fishnet_draws(n: int, P: int, seed: int):
    """Standard normal draws for fishnet casting: G (P x n, one row per
    starting point) and P*P draws for the repopulation weights (more than the
    rounds of 2^p points consume)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((P, n)), rng.standard_normal(P * P)


def row_block(lp: LP, r0: int, r1: int) -> LP:
    """Rows r0..r1-1 of ``lp`` with every column: the rows of K one GPU would
    own under a row partition (its dual sweep gathers the full primal vector)."""
    a, b = int(lp.rowptr[r0]), int(lp.rowptr[r1])
    return LP(lp.n, r1 - r0, (lp.rowptr[r0:r1 + 1] - a).astype(np.int64), lp.col[a:b].copy(), lp.val[a:b].copy(),
              lp.row_type[r0:r1].copy(), lp.rhs[r0:r1].copy(), lp.c.copy(), lp.l.copy(), lp.u.copy(),
              name=f"{lp.name}[rows {r0}:{r1}]")


def col_block(lp: LP, c0: int, c1: int) -> LP:
    """Columns c0..c1-1 of ``lp`` with every row: the rows of K^T one GPU would
    own under a column partition (its primal sweep gathers the full dual
    vector).  Rows without an entry in the block stay, empty."""
    keep = (lp.col >= c0) & (lp.col < c1)
    rows = np.repeat(np.arange(lp.m, dtype=np.int64), np.diff(lp.rowptr))
    cnt = np.bincount(rows[keep], minlength=lp.m)
    rowptr = np.zeros(lp.m + 1, dtype=np.int64)
    np.cumsum(cnt, out=rowptr[1:])
    return LP(c1 - c0, lp.m, rowptr, (lp.col[keep] - c0).astype(np.int32), lp.val[keep].copy(),
              lp.row_type.copy(), lp.rhs.copy(), lp.c[c0:c1].copy(), lp.l[c0:c1].copy(), lp.u[c0:c1].copy(),
              name=f"{lp.name}[cols {c0}:{c1}]")


def random_case(seed: int) -> LP:
    """A planted LP of a shape drawn from `seed` (for sweeps over many
    structures): either a dense tiny LP with free and half-bounded variables
    or a sparse planted LP with m in [5, 400], n in [m, 3m], density in
    [0.5%, 20%] (at least 1.5 entries per row on average), ">=" rows 0-100%,
    and in a quarter of the sparse cases one row and one column emptied."""
    rng = np.random.default_rng(90_000 + seed)
    if rng.random() < 0.3:
        n = int(rng.integers(2, 12))
        m = int(rng.integers(1, n + 1))
        return tiny(int(rng.integers(1 << 31)), n=n, m=m, ge_frac=float(rng.random()),
                    free_frac=float(rng.uniform(0.0, 0.6)))
    m = int(rng.integers(5, 401))
    n = int(rng.integers(m, 3 * m + 1))
    d = float(min(0.2, max(rng.uniform(0.005, 0.2), 1.5 / n)))
    lp = planted(m, n, d, int(rng.integers(1 << 31)), ge_frac=float(rng.random()),
                 u_range=(float(rng.uniform(0.5, 2.0)), float(rng.uniform(3.0, 20.0))))
    if rng.random() >= 0.25:
        return lp
    # empty row i and column j.  The planted reduced costs z = c - K'y* stay,
    # so c' = K2'y2 + z keeps (x*, y2) optimal; row i becomes an "=" row with
    # right-hand side 0 and multiplier 0
    i, j = int(rng.integers(m)), int(rng.integers(n))
    rows = np.repeat(np.arange(m), np.diff(lp.rowptr))
    A = np.zeros((m, n))
    np.add.at(A, (rows, lp.col), lp.val)
    z = lp.c - A.T @ lp.y_star
    A[i, :] = 0.0
    A[:, j] = 0.0
    y = lp.y_star.copy()
    y[i] = 0.0
    rt = lp.row_type.copy()
    rt[i] = EQ
    ax = A @ lp.x_star
    inactive = (rt == GE) & (y == 0.0)
    rhs = ax.copy()
    rhs[inactive] -= rng.uniform(0.1, 1.0, size=int(inactive.sum()))
    c = A.T @ y + z
    r, cc = np.nonzero(A)
    rowptr, col, val = _csr_from_coo(m, r.astype(np.int64), cc.astype(np.int64), A[r, cc])
    return LP(n, m, rowptr, col, val, rt, rhs, c, lp.l.copy(), lp.u.copy(), name=lp.name + "-emptied",
              x_star=lp.x_star, y_star=y, f_star=float(c @ lp.x_star))

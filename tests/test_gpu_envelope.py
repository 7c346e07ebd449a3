"""Differentiation through unrolled PDHG steps where the optimum is known.

Envelope theorem (the dual of Section 2.2, Appendix B): at a unique,
non-degenerate optimum the optimal value f* = min_x max_y L(x, y) with
L = c'x + q'y - y'Kx (x in X, y in Y) has df*/dc = x*, df*/dq = y*, and
df*/dl = lambda*^+, df*/du = lambda*^- with lambda* = c - K'y*.  Unrolled
from a saddle point, the map z_K(c, q, l, u, z_0) of K fixed steps (Appendix
D's step) gives L(z_K) the same first-order behaviour: its total derivative
is the direct term (x_K, y_K) plus the adjoint of the steps applied to
(dL/dx_K, dL/dy_K) = (c - K'y_K, q - K x_K), whose components on free
coordinates vanish at the saddle and whose components on clipped coordinates
(lambda on variables at a bound, the slack of inactive ">=" rows) must be
stopped by the clip masks -- or routed to l and u, where they make up
lambda*^+ and lambda*^-.  C0u has a unique, non-degenerate planted optimum.

The primal objective c'x_K is differentiated as well and reported: its
derivative reaches x* only as the linearised steps converge, at a rate set by
the smallest singular values of the active basis, which K = 500 steps do not
reach on C0u (measured, not gated).

The C4 shape (SCED at 1/10 scale, FP32, K = 500 steps with a checkpoint
every 50, warm-started from a 1e-4 solve): pdhg_backward on 4 instances of a
batched handle against the oracle's reverse mode and against FP64 central
differences of the oracle's unrolled map along random directions.
"""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16806_amd as pd

    pd.lib()
    return pd


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _lagrangian_grads(s, lp, K):
    """Total derivative of L(x_K, y_K) w.r.t. (c, rhs, l, u) after K recorded steps."""
    s.iterate(K, record=True)
    xk, yk = s.solution(which=1)  # SOL_CURRENT
    A = lp.scipy()
    g = s.backward(lp.c - A.T @ yk, lp.rhs - A @ xk)
    return {"c": xk + g["c"], "rhs": yk + g["rhs"], "l": g["l"], "u": g["u"]}, xk, yk


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_envelope_c0u_from_the_optimum(pd, prec, seed):
    """Gate (1e-2 relative in norm, K = 500 from the planted optimum): dL/dc =
    x*, dL/dq = y*, dL/dl = lambda*^+, dL/du = lambda*^-."""
    lp = lpgen.config0(seed, unique=True)
    K = 500
    s = pd.Solver(lp, precision=prec, eps=1e-6, unroll_capacity=K, unroll_checkpoint=50)
    s.solve()  # the step parameters of the end of a solve
    s.set_state(lp.x_star, lp.y_star)
    d, xk, yk = _lagrangian_grads(s, lp, K)
    lam = lp.c - lp.scipy().T @ lp.y_star
    errs = {"c": _rel(d["c"], lp.x_star), "rhs": _rel(d["rhs"], lp.y_star),
            "l": _rel(d["l"], np.maximum(lam, 0.0)), "u": _rel(d["u"], np.minimum(lam, 0.0))}
    # the primal objective's derivative (reported): x_K + (dx_K/dc)'c vs x*, (dx_K/dq)'c vs y*
    s.set_state(lp.x_star, lp.y_star)
    s.iterate(K, record=True)
    gp = s.backward(lp.c, np.zeros(lp.m))
    xk2, _ = s.solution(which=1)
    print(f"[envelope] C0u seed {seed} {prec}: lagrangian {errs}; primal objective: "
          f"dc vs x* {_rel(xk2 + gp['c'], lp.x_star):.3e}, dq vs y* {_rel(gp['rhs'], lp.y_star):.3e}", flush=True)
    for k, e in errs.items():
        assert e <= 1e-2, (k, e)
    # far inside the gate: FP64 to ~1e-12, FP32 to the iterates' rounding
    assert max(errs.values()) <= (1e-9 if prec == "f64" else 1e-4), errs


def test_envelope_c0u_from_a_solve(pd):
    """The same gate warm-started from the library's own FP64 solve to 1e-8
    (the realistic use: the optimum is not known): the error is that of the
    solve's point."""
    lp = lpgen.config0(2, unique=True)
    K = 500
    s = pd.Solver(lp, precision="f64", eps=1e-8, max_iters=400000, unroll_capacity=K, unroll_checkpoint=50)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL"
    x, y = s.solution()
    s.set_state(x, y)
    d, _, _ = _lagrangian_grads(s, lp, K)
    lam = lp.c - lp.scipy().T @ lp.y_star
    errs = {"c": _rel(d["c"], lp.x_star), "rhs": _rel(d["rhs"], lp.y_star),
            "l": _rel(d["l"], np.maximum(lam, 0.0)), "u": _rel(d["u"], np.minimum(lam, 0.0))}
    print(f"[envelope] C0u seed 2 from an FP64 solve: {errs}", flush=True)
    for k, e in errs.items():
        assert e <= 1e-2, (k, e)


def _c4_run(pd, prec):
    """4 SCED/10 instances in one handle, solved to 1e-4, then K = 500
    recorded steps from the solutions; the loss is sum_i c_i'x_K,i."""
    K, C = 500, 50
    lps = [lpgen.config4_instance(i) for i in range(4)]
    s = pd.Solver(lps, precision=prec, eps=1e-4, max_iters=200000, unroll_capacity=K, unroll_checkpoint=C)
    rs = s.solve()
    starts = [s.solution(inst=i) for i in range(4)]
    for i, (x, y) in enumerate(starts):
        s.set_state(x, y, inst=i)
    s.iterate(K, record=True)
    g = s.backward(np.concatenate([lp.c for lp in lps]), np.zeros(sum(lp.m for lp in lps)))
    s.close()
    return dict(K=K, lps=lps, rs=rs, starts=starts, g=g)


@pytest.fixture(scope="module")
def c4_f64(pd):
    return _c4_run(pd, "f64")


@pytest.fixture(scope="module")
def c4_f32(pd):
    return _c4_run(pd, "f32")


def _split(c4, i):
    """Instance i's slices of the batched gradients."""
    lps = c4["lps"]
    xo = sum(lp.n for lp in lps[:i])
    yo = sum(lp.m for lp in lps[:i])
    n, m = lps[i].n, lps[i].m
    g = c4["g"]
    return {"c": g["c"][xo:xo + n], "q": g["rhs"][yo:yo + m], "l": g["l"][xo:xo + n], "u": g["u"][xo:xo + n],
            "x0": g["x0"][xo:xo + n], "y0": g["y0"][yo:yo + m]}


def _vs_oracle(orc, c4, inst):
    lp, r = c4["lps"][inst], c4["rs"][inst]
    x0, y0 = c4["starts"][inst]
    o = orc.Oracle(lp)
    ref = o.unrolled_vjp(10, r["tau"], r["sigma"], lp.c, lp.rhs, lp.l, lp.u, x0, y0, c4["K"], lp.c, np.zeros(lp.m))
    got = _split(c4, inst)
    errs = {k: _rel(got[k], ref[k]) for k in ("c", "q", "l", "u", "x0", "y0") if np.linalg.norm(ref[k]) > 0}
    # how concentrated the differences are: entries off by more than 1e-3 of the gradient's largest entry
    off = {k: int(np.sum(np.abs(got[k] - ref[k]) > 1e-3 * np.abs(ref[k]).max())) for k in errs}
    return o, ref, got, errs, off


@pytest.mark.parametrize("inst,ndir", [(0, 32), (1, 8), (2, 8), (3, 8)])
def test_c4_backward_f64_vs_oracle_and_fd(orc, pd, c4_f64, inst, ndir):
    """FP64 at the C4 shape: the oracle's reverse mode to 1e-9 relative in norm,
    and FP64 central differences of the oracle's unrolled map along random
    directions of (c, q, l, u)."""
    c4 = c4_f64
    lp, r = c4["lps"][inst], c4["rs"][inst]
    x0, y0 = c4["starts"][inst]
    o, ref, got, errs, off = _vs_oracle(orc, c4, inst)
    print(f"[c4] inst {inst} FP64: vs oracle reverse mode {errs}", flush=True)
    for k, e in errs.items():
        assert e <= 1e-9, (k, e)
    rng = np.random.default_rng(100 + inst)
    fin_l, fin_u = np.isfinite(lp.l), np.isfinite(lp.u)
    base = dict(c=lp.c, q=lp.rhs, l=np.where(fin_l, lp.l, 0.0), u=np.where(fin_u, lp.u, 0.0))

    def F(p):
        xk, _ = o.unrolled(10, r["tau"], r["sigma"], p["c"], p["q"], np.where(fin_l, p["l"], lp.l),
                           np.where(fin_u, p["u"], lp.u), x0, y0, c4["K"])
        return lp.c @ xk

    # The warm start sits near SCED's degenerate optimum, where many clip
    # decisions are within 1e-8 relative of a bound: steps of h >= 1e-8 cross
    # kinks of the piecewise-linear map (measured on the CPU: central
    # differences off by 1e-5..1e-4 at h = 1e-6..1e-8, 1e-7 at h = 1e-10,
    # which is their rounding level there)
    h = 1e-10
    worst = []
    for _ in range(ndir):
        v = {}
        for k, a in base.items():
            d = rng.standard_normal(a.shape[0])
            if k == "l":
                d *= fin_l
            if k == "u":
                d *= fin_u
            v[k] = d * (np.linalg.norm(a) / max(np.linalg.norm(d), 1e-300))
        fd = (F({k: base[k] + h * v[k] for k in base}) - F({k: base[k] - h * v[k] for k in base})) / (2 * h)
        an = sum(got[k] @ v[k] for k in ("c", "q", "l", "u"))
        scale = sum(np.linalg.norm(ref[k]) * np.linalg.norm(v[k]) for k in ("c", "q", "l", "u"))
        worst.append(abs(fd - an) / scale)
    worst = np.array(worst)
    print(f"[c4] inst {inst} FP64: {ndir} central differences, |fd - <g, v>| / sum |g_k||v_k|: "
          f"median {np.median(worst):.2e}, max {worst.max():.2e}", flush=True)
    assert worst.max() <= 1e-5, worst


@pytest.mark.parametrize("inst", [0, 1, 2, 3])
def test_c4_backward_f32_vs_oracle(orc, pd, c4_f32, inst):
    """FP32 at the C4 shape against the oracle's FP64 reverse mode from the
    same start.  The two trajectories differ by FP32 rounding, and at a
    warm start near SCED's degenerate optimum some clip decisions sit on a
    tie (variables with zero reduced cost at a bound), so a handful of masks
    differ and with them the one-sided slopes of the piecewise-linear map
    (the differing entries are printed: tens to hundreds of the 44,548 +
    32,572).  Measured 0.5-1.5% relative in norm; gated at 5e-2."""
    o, ref, got, errs, off = _vs_oracle(orc, c4_f32, inst)
    print(f"[c4] inst {inst} FP32: vs oracle reverse mode {errs}; entries off by > 1e-3 of the largest: {off}",
          flush=True)
    for k, e in errs.items():
        assert e <= 5e-2, (k, e)


@pytest.fixture(scope="module")
def c4_live(pd):
    """The C4 handle in FP64 kept open: solved to 1e-4, K = 500 recorded steps
    from the solutions, the gradient of sum_i c_i'x_K,i, and the forward map
    of the same handle for finite differences (set_data keeps the matrix, the
    Ruiz factors and the step parameters)."""
    K, C = 500, 50
    lps = [lpgen.config4_instance(i) for i in range(4)]
    s = pd.Solver(lps, precision="f64", eps=1e-4, max_iters=200000, unroll_capacity=K, unroll_checkpoint=C)
    s.solve()
    starts = [s.solution(inst=i) for i in range(4)]
    for i, (x, y) in enumerate(starts):
        s.set_state(x, y, inst=i)
    s.iterate(K, record=True)
    g = s.backward(np.concatenate([lp.c for lp in lps]), np.zeros(sum(lp.m for lp in lps)))
    c4 = dict(K=K, lps=lps, starts=starts, g=g)

    def losses(data):
        """Each instance's own loss c_i'x_K,i after K steps from its start with
        the data (c, q, l, u) given per instance."""
        s.set_data(c=np.concatenate([d["c"] for d in data]), rhs=np.concatenate([d["q"] for d in data]),
                   l=np.concatenate([d["l"] for d in data]), u=np.concatenate([d["u"] for d in data]))
        for i, (x, y) in enumerate(starts):
            s.set_state(x, y, inst=i)
        s.iterate(K)
        return np.array([lp.c @ s.solution(inst=i, which=pd.SOL_CURRENT)[0] for i, lp in enumerate(lps)])

    c4["losses"] = losses
    yield c4
    s.close()


def _c4_data(lps):
    return [dict(c=lp.c.copy(), q=lp.rhs.copy(), l=lp.l.copy(), u=lp.u.copy()) for lp in lps]


def test_c4_backward_f64_vs_gpu_fd(pd, c4_live):
    """FP64 at the C4 shape (4 SCED/10 LPs in one handle, K = 500 steps,
    checkpoint every 50): the adjoint against central differences of the
    same handle's forward map, per LP, along 32 random directions of
    (c, q, l, u) and on 32 single coordinates (8 each of c, q and the finite
    l and u: the 4 largest gradient entries and 4 random ones), the latter
    with both one-sided differences.  Each
    evaluation perturbs all four LPs at once, each along its own direction,
    and reads each LP's own loss: the LPs share no data."""
    c4 = c4_live
    lps, losses = c4["lps"], c4["losses"]
    g = [_split(c4, i) for i in range(4)]
    rng = np.random.default_rng(7)
    fams = ("c", "q", "l", "u")
    fin = [dict(c=np.ones(lp.n, bool), q=np.ones(lp.m, bool), l=np.isfinite(lp.l), u=np.isfinite(lp.u))
           for lp in lps]
    # directions: h relative to the data's norm, small enough to cross no clip
    # decision at the degenerate warm start (as for the oracle's map)
    h = 1e-10
    dir_err = [[] for _ in lps]
    for _ in range(32):
        vs = []
        for i, lp in enumerate(lps):
            base = _c4_data([lp])[0]
            v = {}
            for k in fams:
                a = np.where(fin[i][k], base[k], 0.0)
                d = rng.standard_normal(a.shape[0]) * fin[i][k]
                v[k] = d * (np.linalg.norm(a) / max(np.linalg.norm(d), 1e-300))
            vs.append(v)
        plus, minus = _c4_data(lps), _c4_data(lps)
        for i in range(4):
            for k in fams:
                plus[i][k] = plus[i][k] + h * vs[i][k]
                minus[i][k] = minus[i][k] - h * vs[i][k]
        fd = (losses(plus) - losses(minus)) / (2 * h)
        for i in range(4):
            an = sum(g[i][k] @ vs[i][k] for k in fams)
            scale = sum(np.linalg.norm(g[i][k]) * np.linalg.norm(vs[i][k]) for k in fams)
            dir_err[i].append(abs(fd[i] - an) / scale)
    # coordinates: one-sided steps of 1e-7 of the entry's size, at least
    # 1e-4 (the losses are ~7e7, so one ulp of a loss is ~1.5e-8 and a
    # difference quotient carries an error of a few ulp / step; that bound,
    # 8 ulp(L) / step, is added to the tolerances).  Where the two one-sided
    # slopes agree the map is differentiable there and the central
    # difference must equal the gradient entry; where they differ the
    # coordinate sits on or near a kink (a clip decision tied at the
    # degenerate warm start: a variable at its bound with zero reduced
    # cost), and the adjoint's entry, the slope of the side its recorded
    # masks took, must lie between the two one-sided slopes of a 100x
    # shorter step.
    coords = []
    for i, lp in enumerate(lps):
        cl = []
        for k in fams:
            idx = np.flatnonzero(fin[i][k])
            top = idx[np.argsort(-np.abs(g[i][k][idx]))[:4]]
            rest = rng.choice(np.setdiff1d(idx, top), 4, replace=False)
            cl += [(k, int(j)) for j in np.concatenate([top, rest])]
        coords.append(cl)
    L0 = losses(_c4_data(lps))

    def one_sided(t, shrink):
        plus, minus = _c4_data(lps), _c4_data(lps)
        dl = np.empty(4)
        for i in range(4):
            k, j = coords[i][t]
            dl[i] = max(1e-7 * abs(plus[i][k][j]), 1e-4) / shrink
            plus[i][k][j] += dl[i]
            minus[i][k][j] -= dl[i]
        Lp, Lm = losses(plus), losses(minus)
        return (L0 - Lm) / dl, (Lp - L0) / dl, 8 * np.spacing(np.abs(L0)) / dl

    co_err = [[] for _ in lps]
    kinks = [0] * 4
    for t in range(32):
        left, right, noise = one_sided(t, 1.0)
        scale = [max(abs(g[i][coords[i][t][0]][coords[i][t][1]]), abs(right[i]), abs(left[i]), 1e-12)
                 for i in range(4)]
        kinked = [abs(right[i] - left[i]) > 1e-4 * scale[i] + 2 * noise[i] for i in range(4)]
        if any(kinked):
            # a kink within the step: the one-sided slopes of a 100x shorter
            # step, closer to the limits at the point itself
            left2, right2, noise2 = one_sided(t, 100.0)
        for i in range(4):
            k, j = coords[i][t]
            gj = g[i][k][j]
            if not kinked[i]:
                co_err[i].append(max(abs(0.5 * (right[i] + left[i]) - gj) - noise[i], 0.0) / scale[i])
            else:
                kinks[i] += 1
                lo, hi = min(left2[i], right2[i]), max(left2[i], right2[i])
                co_err[i].append(max(lo - noise2[i] - gj, gj - hi - noise2[i], 0.0) / scale[i])
            if co_err[i][-1] > 1e-4:
                print(f"[c4-fd] LP {i} {k}[{j}] g {gj:.9g} left {left[i]:.9g} right {right[i]:.9g}"
                      + (f" (1/100 step: {left2[i]:.9g} {right2[i]:.9g})" if kinked[i] else ""), flush=True)
    for i in range(4):
        de, ce = np.array(dir_err[i]), np.array(co_err[i])
        print(f"[c4-fd] LP {i} (loss {L0[i]:.6g}): 32 directions |fd - <g,v>| / sum |g_k||v_k| median {np.median(de):.2e} max "
              f"{de.max():.2e}; 32 coordinates ({kinks[i]} on kinks) relative error median {np.median(ce):.2e} "
              f"max {ce.max():.2e}", flush=True)
    for i in range(4):
        assert max(dir_err[i]) <= 1e-5, (i, dir_err[i])
        assert max(co_err[i]) <= 2e-4, (i, co_err[i], coords[i])

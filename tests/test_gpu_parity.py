"""GPU-vs-oracle parity of the HIP path, called through the C-ABI.

Tolerances:
  * FP64 mode: the GPU and the oracle evaluate the same expressions with
    different summation orders; per-element relative agreement of 1e-12 (one
    step, KKT terms) and 1e-9 after a few hundred steps is well above the
    accumulated rounding (~n_steps * 1e-16 * condition).
  * FP32 mode: iterates and matrix values are rounded to FP32 (unit roundoff
    6e-8) but accumulate in FP64, so one step from identical FP32-representable
    inputs agrees with the FP64 oracle to a few FP32 ulps of the operands'
    magnitude; whole solves are compared on what the method fixes: the oracle's
    relative KKT of the returned point <= 1e-4 and the objective within 1e-5
    (relative) of the planted / oracle optimum.
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
    return abs(a - b) / (1.0 + abs(b))


def _cases():
    return {
        "c0": lpgen.config0(0),
        "mixed": lpgen.planted(300, 700, 0.02, 5, ge_frac=0.5),
        "tinyfree": lpgen.tiny(3, n=8, m=4, free_frac=0.5),
        "sced_small": lpgen.sced(40, 16, 8, 12, seed=5),
        "zipf": lpgen.config2(7, m=3000, n=6000, kmax=2000),
    }


# ---------------------------------------------------------------------------
# KKT of a caller point (FP64 throughout)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c0", "mixed", "tinyfree", "sced_small", "zipf"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_kkt_matches_oracle(orc, pd, name, prec):
    lp = _cases()[name]
    o = orc.Oracle(lp)
    s = pd.Solver(lp, precision=prec)
    rng = np.random.default_rng(1)
    pts = [(np.clip(rng.standard_normal(lp.n) * 3, lp.l, lp.u), rng.standard_normal(lp.m))]
    if lp.x_star is not None:
        pts.append((lp.x_star, lp.y_star))
    for x, y in pts:
        g = s.kkt(x, y)
        c = o.kkt(x, y)
        for k in ("pres", "dres", "pobj", "dobj"):
            assert g[k] == pytest.approx(c[k], rel=1e-11, abs=1e-11 * (1 + abs(c["pobj"]))), (k, g[k], c[k])
        assert g["rel_kkt"] == pytest.approx(c["rel_kkt"], rel=1e-9, abs=1e-13)


# ---------------------------------------------------------------------------
# setup: Ruiz factors, power iteration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c0", "mixed", "sced_small", "zipf"])
def test_ruiz_factors_match_oracle(orc, pd, name):
    lp = _cases()[name]
    o = orc.Oracle(lp)
    for iters in (1, 10):
        s = pd.Solver(lp, precision="f64", ruiz_iters=iters)
        rho, kap = s.scaling()
        rho_o, kap_o = o.ruiz(iters)
        # same expressions, same order, IEEE sqrt and division: bitwise equal
        np.testing.assert_array_equal(rho, rho_o)
        np.testing.assert_array_equal(kap, kap_o)


@pytest.mark.parametrize("name", ["c0", "mixed", "sced_small"])
def test_power_norm_matches_oracle(orc, pd, name):
    lp = _cases()[name]
    s = pd.Solver(lp, precision="f64", ruiz_iters=10, power_tol=1e-9, power_max_iters=20000)
    kn, _ = orc.Oracle(lp).power_norm(10, max_iters=20000, tol=1e-9)
    assert s.info()["knorm"] == pytest.approx(kn, rel=1e-6)


# ---------------------------------------------------------------------------
# fixed-step trajectory (FP64)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c0", "mixed", "sced_small", "zipf"])
def test_fixed_steps_match_oracle_f64(orc, pd, name):
    lp = _cases()[name]
    o = orc.Oracle(lp)
    eta, omega = 0.5, 1.3
    s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=eta, primal_weight=omega)
    kn = s.info()["knorm"]
    eta = 0.9 / kn
    s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=eta, primal_weight=omega)
    rho, kap = o.ruiz(10)
    x0s = np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap)
    y0s = np.zeros(lp.m)
    done = 0
    for k in (1, 9, 190):
        s.iterate(k)
        done += k
        xs, ys = o.steps(x0s, y0s, eta / omega, eta * omega, done, ruiz_iters=10)
        x, y = s.solution(which=pd.SOL_CURRENT)
        xo, yo = np.clip(kap * xs, lp.l, lp.u), rho * ys
        tol = 1e-12 if k == 1 else 1e-9
        np.testing.assert_allclose(x, xo, rtol=tol, atol=tol * (1 + np.abs(xo).max()))
        np.testing.assert_allclose(y, yo, rtol=tol, atol=tol * (1 + np.abs(yo).max()))


def test_iterate_resume_is_exact(pd):
    lp = _cases()["mixed"]
    for prec in ("f32", "f64"):
        a = pd.Solver(lp, precision=prec)
        b = pd.Solver(lp, precision=prec)
        a.iterate(37)
        a.iterate(63)
        b.iterate(100)
        xa, ya = a.solution(which=pd.SOL_CURRENT)
        xb, yb = b.solution(which=pd.SOL_CURRENT)
        np.testing.assert_array_equal(xa, xb)
        np.testing.assert_array_equal(ya, yb)


def test_one_step_f32_matches_oracle(orc, pd):
    """FP32 storage, FP64 accumulation: one step agrees to FP32 rounding."""
    lp = _cases()["sced_small"]
    o = orc.Oracle(lp)
    s64 = pd.Solver(lp, precision="f64")
    eta = 0.9 / s64.info()["knorm"]
    s = pd.Solver(lp, precision="f32", step_size=eta, primal_weight=1.0)
    rng = np.random.default_rng(3)
    rho, kap = o.ruiz(10)
    # a start point that is exactly representable in FP32 in scaled variables
    xs = np.clip(rng.uniform(-1, 1, lp.n), lp.l / kap, lp.u / kap).astype(np.float32).astype(np.float64)
    ys = rng.standard_normal(lp.m).astype(np.float32).astype(np.float64)
    ys[lp.row_type == 0] = np.abs(ys[lp.row_type == 0])
    s.set_state(kap * xs, rho * ys)
    s.iterate(1)
    x, y = s.solution(which=pd.SOL_CURRENT)
    xo, yo = o.steps(xs, ys, eta, eta, 1, ruiz_iters=10)
    rho = o.ruiz(10)[0]
    Ks = abs(lp.scipy().multiply(rho[:, None]).multiply(kap[None, :])).tocsr()
    bx, by = fp32_step_bounds(Ks, kap * lp.c, rho * lp.rhs, xs, ys, xo, yo, eta, eta)
    assert np.all(np.abs(x / kap - xo) <= bx)
    assert np.all(np.abs(y / rho - yo) <= by)


def fp32_step_bounds(Ks, cs, qs, xs, ys, xo, yo, tau, sigma):
    """Per-element bounds on one FP32 step's deviation from the exact FP64
    step (xo, yo) from the same FP32-representable start (xs, ys), in scaled
    variables.

    Each FP32 rounding (a matrix entry, c~, q~, the bounds, x+, xbar, y+) is at
    most u = 2^-24 relative; products of FP32 numbers are exact in FP64 and the
    FP64 sums add ~2^-53 per term, covered by a 1% margin.  With |K~| the
    entrywise absolute matrix:
      primal: v = x - tau (c~ - K~'y): |dv| <= tau u (|c~| + |K~|'|y|); the
        clip to FP32 bounds and the output rounding add u |x+| each:
        |dx+| <= Bx = 2u |x+| + tau u (|c~| + |K~|'|y|)
      xbar = 2 x+ - x, rounded: |dxbar| <= 2 Bx + u |xbar|
      dual: w = y + sigma (q~ - K~ xbar):
        |dw| <= sigma (u |q~| + u |K~||xbar| + |K~| |dxbar|)
      y+ = proj(w), rounded: |dy+| <= |dw| + u |y+|
    """
    u = 2.0 ** -24
    xb = 2 * xo - xs
    bx = 2 * u * np.abs(xo) + tau * u * (np.abs(cs) + Ks.T @ np.abs(ys))
    dxb = 2 * bx + u * np.abs(xb)
    by = sigma * (u * np.abs(qs) + u * (Ks @ np.abs(xb)) + Ks @ dxb) + u * np.abs(yo)
    return 1.01 * bx + 1e-300, 1.01 * by + 1e-300


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

def test_solve_c0_plain_f64(orc, pd):
    lp = _cases()["c0"]
    opts = dict(precision="f64", ruiz_iters=0, use_restarts=0, use_pw_update=0, eps=1e-6, max_iters=400000)
    s = pd.Solver(lp, **opts)
    r = s.solve()[0]
    ro = orc.Oracle(lp).solve(orc.SolveOpts.plain(eps=1e-6, max_iters=400000))
    assert r["status"] == 0 and ro.status == 0
    x, y = s.solution()
    chk = orc.Oracle(lp).kkt(x, y)
    assert chk["rel_kkt"] <= 1e-6 * 1.01
    assert _rel(chk["pobj"], lp.f_star) <= 1e-5
    # same iteration count: identical algorithm in FP64, same check schedule
    assert abs(r["iters"] - ro.iters) <= 64
    assert r["restarts"] == 0


@pytest.mark.parametrize("name", ["c0", "mixed", "tinyfree"])
def test_solve_restarted_f64(orc, pd, name):
    lp = _cases()[name]
    s = pd.Solver(lp, precision="f64", eps=1e-6)
    r = s.solve()[0]
    ro = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6))
    assert r["status"] == 0, r
    x, y = s.solution()
    chk = orc.Oracle(lp).kkt(x, y)
    assert chk["rel_kkt"] <= 1e-6 * 1.01
    assert _rel(chk["pobj"], ro.kkt["pobj"]) <= 1e-5
    if lp.f_star is not None:
        assert _rel(chk["pobj"], lp.f_star) <= 1e-5
    assert r["knorm"] == pytest.approx(ro.knorm, rel=1e-5)
    assert r["omega0"] == pytest.approx(ro.omega0, rel=1e-12)


# the Zipf LP at 1e-5: even the FP64 method stalls above 1e-6 on it within
# 200,000 iterations (its best check in a CPU replay: 1.3e-6)
F32_EPS = {"zipf": 1e-5}


@pytest.mark.parametrize("name", ["c0", "mixed", "sced_small", "zipf"])
def test_solve_f32_parity(orc, pd, name):
    lp = _cases()[name]
    o = orc.Oracle(lp)
    eps = F32_EPS.get(name, 1e-6)
    s = pd.Solver(lp, precision="f32", eps=eps, max_iters=200000)
    r = s.solve()[0]
    x, y = s.solution()
    chk = o.kkt(x, y)
    if lp.f_star is not None:
        fref = lp.f_star
    else:
        fref = o.solve(orc.SolveOpts(eps=1e-7, max_iters=2_000_000)).kkt["pobj"]
    print(name, r["status_name"], r["iters"], r["restarts"], r["kkt"]["rel_kkt"], chk["rel_kkt"],
          _rel(chk["pobj"], fref))
    assert r["status_name"] == "OPTIMAL" and chk["rel_kkt"] <= 1.05 * eps, (r["status_name"], chk)
    assert _rel(chk["pobj"], fref) <= 1e-5


def test_solution_lambda(orc, pd):
    lp = _cases()["tinyfree"]
    s = pd.Solver(lp, precision="f64", eps=1e-8)
    s.solve()
    x, y, lam = s.solution(lam=True)
    o = orc.Oracle(lp)
    d = lp.c - o.spmv_t(y)
    inf_l, inf_u = ~np.isfinite(lp.l), ~np.isfinite(lp.u)
    ref = np.where(inf_l & inf_u, 0.0, np.where(inf_l, np.minimum(d, 0), np.where(inf_u, np.maximum(d, 0), d)))
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=1e-10)


def test_set_state_roundtrip(pd):
    lp = _cases()["mixed"]
    s = pd.Solver(lp, precision="f64")
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, lp.n) * lp.u
    y = rng.standard_normal(lp.m)
    y[lp.row_type == 0] = np.abs(y[lp.row_type == 0])
    s.set_state(x, y)
    x2, y2 = s.solution(which=pd.SOL_CURRENT)
    np.testing.assert_allclose(x2, x, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(y2, y, rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------------------
# batching
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("budget", [0, None])
def test_batched_equals_solo_bitwise(pd, prec, budget):
    """All instances running at once (budget 0) and the default admission."""
    lps = [lpgen.planted(m, int(2.5 * m), 0.02, 30 + i, ge_frac=0.3) for i, m in enumerate([60, 150, 90, 240])]
    lps.append(lpgen.sced(20, 8, 4, 6, seed=9))
    kw = dict(precision=prec, eps=1e-5)
    b = pd.Solver(lps, **kw) if budget is None else pd.Solver(lps, batch_resident_bytes=budget, **kw)
    rb = b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        rs = s.solve()[0]
        assert rb[i]["iters"] == rs["iters"] and rb[i]["restarts"] == rs["restarts"], i
        assert rb[i]["status"] == rs["status"]
        xb, yb = b.solution(inst=i)
        xs, ys = s.solution()
        np.testing.assert_array_equal(xb, xs)
        np.testing.assert_array_equal(yb, ys)


def _sweep_bytes(lp, e=4):
    """Per-iteration sweep bytes of an instance as the admission budget counts them."""
    return 2 * (e + 4) * lp.nnz + 8 * (lp.n + lp.m + 2) + e * (9 * lp.n + 6 * lp.m)


@pytest.mark.parametrize("budget", ["one", "two", "half"])
@pytest.mark.parametrize("graph", [1, 0])
def test_admission_equals_solo_bitwise(pd, budget, graph):
    """A byte budget that admits the batch's instances a few at a time leaves
    every instance's trajectory as it is alone: same iterations, restarts,
    status and bits."""
    lps = [lpgen.planted(m, int(2.5 * m), 0.02, 40 + i, ge_frac=0.3) for i, m in enumerate([60, 150, 90, 240, 120])]
    lps.append(lpgen.sced(20, 8, 4, 6, seed=9))
    kw = dict(precision="f32", eps=1e-5, use_graph=graph)
    sizes = sorted((_sweep_bytes(lp) for lp in lps), reverse=True)
    cap = {"one": 1, "two": sizes[0] + sizes[1], "half": sum(sizes) // 2}[budget]
    b = pd.Solver(lps, batch_resident_bytes=cap, **kw)
    rb = b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        rs = s.solve()[0]
        assert rb[i]["status_name"] == rs["status_name"] == "OPTIMAL", (i, rb[i]["status_name"])
        assert rb[i]["iters"] == rs["iters"] and rb[i]["restarts"] == rs["restarts"], i
        xb, yb = b.solution(inst=i)
        xs, ys = s.solution()
        np.testing.assert_array_equal(xb, xs)
        np.testing.assert_array_equal(yb, ys)
    # a second solve from the solution: the budget state starts afresh
    rb2 = b.solve()
    assert all(r["status_name"] == "OPTIMAL" for r in rb2)


def test_admission_time_limit_leaves_waiting_at_start(pd):
    """Instances still waiting at a time limit report TIME_LIMIT with no
    iterations and their starting point."""
    lps = [lpgen.planted(m, int(2.5 * m), 0.02, 50 + i, ge_frac=0.3) for i, m in enumerate([300, 200, 100])]
    b = pd.Solver(lps, precision="f64", eps=1e-300, max_iters=10_000_000, time_limit=0.5,
                  batch_resident_bytes=1)
    rb = b.solve()
    order = np.argsort([-_sweep_bytes(lp) for lp in lps], kind="stable")
    first = int(order[0])
    assert rb[first]["status_name"] == "TIME_LIMIT" and rb[first]["iters"] > 0
    for i in order[1:]:
        r = rb[int(i)]
        assert r["status_name"] == "TIME_LIMIT" and r["iters"] == 0, r
        x, y = b.solution(inst=int(i), which=pd.SOL_CURRENT)
        lp = lps[int(i)]
        np.testing.assert_array_equal(x, np.clip(np.zeros(lp.n), lp.l, lp.u))
        np.testing.assert_array_equal(y, np.zeros(lp.m))


def test_graph_and_eager_agree(pd):
    lp = _cases()["mixed"]
    a = pd.Solver(lp, precision="f32", eps=1e-5, use_graph=1)
    b = pd.Solver(lp, precision="f32", eps=1e-5, use_graph=0)
    ra, rb = a.solve()[0], b.solve()[0]
    assert ra["iters"] == rb["iters"]
    np.testing.assert_array_equal(a.solution()[0], b.solution()[0])


def test_iteration_and_time_limits(pd):
    lp = _cases()["sced_small"]
    s = pd.Solver(lp, precision="f32", eps=1e-12, max_iters=640)
    r = s.solve()[0]
    assert r["status_name"] == "ITERATION_LIMIT" and r["iters"] == 640
    s = pd.Solver(lp, precision="f32", eps=1e-12, max_iters=10**9, time_limit=0.2)
    r = s.solve()[0]
    assert r["status_name"] == "TIME_LIMIT"
    x, y = s.solution()
    assert np.isfinite(x).all() and np.isfinite(y).all()


def test_huge_step_reports_numerical_error(pd):
    """A step far above 1/||K|| makes the iterates of free variables grow
    geometrically; the check's FP64 sums overflow and the control kernel
    stops the instance with NUMERICAL_ERROR."""
    lp = _cases()["tinyfree"]
    assert np.isinf(lp.l).any()
    s = pd.Solver(lp, precision="f32", step_size=1e4, max_iters=100000, use_restarts=0)
    r = s.solve()[0]
    assert r["status_name"] == "NUMERICAL_ERROR"


# ---------------------------------------------------------------------------
# launch layouts: rows per lane group, bin limits, XCD numbering, grid cap
# ---------------------------------------------------------------------------

LAYOUTS = [
    dict(bin_rows_dual=[4] * 5 + [1] * 3, bin_rows_primal=[4] * 5 + [1] * 3),
    dict(bin_rows_dual=[2] * 5 + [1] * 3, bin_rows_primal=[2] * 5 + [1] * 3, xcd_remap=0, max_grid=64),
    dict(bin_len_dual=[16, 32, 64, 128, 256, 512, 2048, 0], bin_len_primal=[1, 2, 4, 8, 16, 32, 64, 0],
         xcd_remap=1, max_grid=100000),
    # the dual sweep in column slices (rows of >= 16 S entries)
    dict(col_slices=4),
    dict(col_slices=3, bin_rows_dual=[2] * 5 + [1] * 3, xcd_remap=1, max_grid=64),
]


@pytest.mark.parametrize("li", range(len(LAYOUTS)))
@pytest.mark.parametrize("name", ["mixed", "zipf", "sced_small"])
def test_layouts_fixed_steps_f64(orc, pd, li, name):
    lp = _cases()[name]
    o = orc.Oracle(lp)
    s0 = pd.Solver(lp, precision="f64")
    eta, omega = 0.9 / s0.info()["knorm"], 1.1
    s = pd.Solver(lp, precision="f64", step_size=eta, primal_weight=omega, **LAYOUTS[li])
    rho, kap = o.ruiz(10)
    s.iterate(50)
    xs, ys = o.steps(np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap), np.zeros(lp.m), eta / omega, eta * omega,
                     50, ruiz_iters=10)
    x, y = s.solution(which=pd.SOL_CURRENT)
    xo, yo = np.clip(kap * xs, lp.l, lp.u), rho * ys
    np.testing.assert_allclose(x, xo, rtol=1e-9, atol=1e-9 * (1 + np.abs(xo).max()))
    np.testing.assert_allclose(y, yo, rtol=1e-9, atol=1e-9 * (1 + np.abs(yo).max()))
    # the caller-point KKT uses the same layout
    g = s.kkt(x, y)
    c = o.kkt(x, y)
    assert g["rel_kkt"] == pytest.approx(c["rel_kkt"], rel=1e-9, abs=1e-13)


@pytest.mark.parametrize("li", range(len(LAYOUTS)))
def test_layouts_solve_f32(orc, pd, li):
    lp = _cases()["zipf"]
    s = pd.Solver(lp, precision="f32", eps=1e-5, max_iters=200000, **LAYOUTS[li])
    r = s.solve()[0]
    x, y = s.solution()
    chk = orc.Oracle(lp).kkt(x, y)
    assert r["status_name"] == "OPTIMAL" and chk["rel_kkt"] <= 1.05e-5, (r["status_name"], chk)
    assert _rel(chk["pobj"], lp.f_star) <= 1e-5


def test_layouts_batched_bitwise(pd):
    lps = [lpgen.planted(m, int(2.5 * m), 0.02, 60 + i, ge_frac=0.3) for i, m in enumerate([70, 160, 110])]
    kw = dict(precision="f32", eps=1e-5, **LAYOUTS[0])
    b = pd.Solver(lps, **kw)
    rb = b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        rs = s.solve()[0]
        assert rb[i]["iters"] == rs["iters"]
        np.testing.assert_array_equal(b.solution(inst=i)[0], s.solution()[0])


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_run_to_run_bitwise(pd, prec):
    """No atomics on the floating-point path: the same solve on two handles,
    and twice on one handle from the same start, gives the same bits (iterate,
    average, KKT terms, restart trace), and so do the check and the KKT of a
    caller point."""
    lp = lpgen.sced(40, 16, 8, 12, seed=5)
    kw = dict(precision=prec, eps=1e-6, trace_capacity=1024)
    a, b = pd.Solver(lp, **kw), pd.Solver(lp, **kw)
    ra, rb = a.solve()[0], b.solve()[0]
    assert ra["iters"] == rb["iters"] and ra["kkt"] == rb["kkt"]
    assert a.trace() == b.trace()
    for which in (pd.SOL_CURRENT, pd.SOL_AVERAGE):
        for u, v in zip(a.solution(which=which), b.solution(which=which)):
            np.testing.assert_array_equal(u, v)
    x, y = a.solution()
    a.set_state(np.zeros(lp.n), np.zeros(lp.m))
    ra2 = a.solve()[0]
    b.set_state(np.zeros(lp.n), np.zeros(lp.m))
    rb2 = b.solve()[0]
    assert ra2["kkt"] == rb2["kkt"] and ra2["iters"] == rb2["iters"]
    assert a.kkt(x, y) == a.kkt(x, y) == b.kkt(x, y)

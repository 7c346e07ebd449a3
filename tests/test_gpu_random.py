"""Parity over 32 seeded LP structures (lpgen.random_case: dense tiny LPs with
free and half-bounded variables; sparse planted LPs of varied shape, density
and row-type mix; emptied rows and columns): FP64 fixed steps and the KKT
function element by element against the oracle, and FP64 restarted solves
to the planted optimum."""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

SEEDS = list(range(32))


@pytest.fixture(scope="module")
def pd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16806_amd as pd

    pd.lib()
    return pd


@pytest.mark.parametrize("seed", SEEDS)
def test_random_case_steps_and_kkt(orc, pd, seed):
    lp = lpgen.random_case(seed)
    o = orc.Oracle(lp)
    s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=1.0, primal_weight=1.0)
    eta, omega = 0.9 / s.info()["knorm"], 0.8
    s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=eta, primal_weight=omega)
    rho, kap = o.ruiz(10)
    x0s = np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap)
    y0s = np.zeros(lp.m)
    done = 0
    for k in (1, 19):
        s.iterate(k)
        done += k
        xs, ys = o.steps(x0s, y0s, eta / omega, eta * omega, done, ruiz_iters=10)
        x, y = s.solution(which=pd.SOL_CURRENT)
        xo, yo = np.clip(kap * xs, lp.l, lp.u), rho * ys
        tol = 1e-12 if k == 1 else 1e-10
        np.testing.assert_allclose(x, xo, rtol=tol, atol=tol * (1 + np.abs(xo).max()))
        np.testing.assert_allclose(y, yo, rtol=tol, atol=tol * (1 + np.abs(yo).max(initial=0.0)))
    # the KKT function at a random point
    rng = np.random.default_rng(seed)
    xr = np.clip(rng.standard_normal(lp.n) * 3, lp.l, lp.u)
    yr = rng.standard_normal(lp.m)
    g, r = s.kkt(xr, yr), o.kkt(xr, yr)
    for key in ("pres", "dres", "pobj", "dobj", "rel_kkt"):
        assert g[key] == pytest.approx(r[key], rel=1e-11, abs=1e-12), (key, g[key], r[key])


@pytest.mark.parametrize("seed", SEEDS)
def test_random_case_solve_f64(orc, pd, seed):
    lp = lpgen.random_case(seed)
    s = pd.Solver(lp, precision="f64", eps=1e-7, max_iters=400000)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", (lp.name, r["status_name"], r["iters"])
    x, y = s.solution()
    o = orc.Oracle(lp)
    chk = o.kkt(x, y)
    assert chk["rel_kkt"] <= 1e-7 * 1.01
    assert abs(chk["pobj"] - lp.f_star) / (1 + abs(lp.f_star)) <= 1e-5
    ro = o.solve(orc.SolveOpts(eps=1e-7, max_iters=400000))
    assert ro.status == 0
    # the same method in FP64: the same work up to a rounding-level flip of a
    # restart decision
    assert abs(r["iters"] - ro.iters) <= max(128, ro.iters // 10), (r["iters"], ro.iters)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("adaptive", [0, 1])
@pytest.mark.parametrize("budget", [0, None])
def test_random_batch_equals_solo_bitwise(pd, prec, adaptive, budget):
    """A batch of 12 different structures (tiny dense with free variables next
    to sparse planted LPs) gives every instance bitwise its solo result, with
    all instances running at once and under the default admission."""
    lps = [lpgen.random_case(s) for s in range(100, 112)]
    kw = dict(precision=prec, eps=1e-6, max_iters=100000, adaptive_step=adaptive)
    b = pd.Solver(lps, **kw) if budget is None else pd.Solver(lps, batch_resident_bytes=budget, **kw)
    rb = b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        rs = s.solve()[0]
        assert rb[i]["status"] == rs["status"] and rb[i]["iters"] == rs["iters"], (i, lp.name)
        xb, yb = b.solution(inst=i)
        xs, ys = s.solution()
        np.testing.assert_array_equal(xb, xs)
        np.testing.assert_array_equal(yb, ys)

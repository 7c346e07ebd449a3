"""The sweeps in column slices (opts.col_slices for the dual sweep,
opts.col_slices_t for the primal sweep): the same iteration as the whole-row
sweeps up to FP64 summation order.

Each sliced row sums its slices' FP64 partials in slice order, so results are
checked against the oracle (FP64 steps to 1e-12 / 1e-9, restart traces check
by check), batched equals solo bit for bit, and the recorded steps of the
adjoint (which sweep whole rows) still match the oracle's reverse mode."""
import numpy as np
import pytest

import lpgen
from test_gpu_trace import _compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16806_amd as pd

    pd.lib()
    return pd


def _zipf():
    """Long rows (Zipf lengths up to 2000), columns of about 16 entries."""
    return lpgen.config2(7, m=3000, n=6000, kmax=2000)


def _tall():
    """Columns of about 52 entries: St = 2 slices all of them, St = 3 three
    quarters, St = 4 a few."""
    return lpgen.config2(7, m=4000, n=2000, kmax=1500)


def _sliced_rows(lp, S):
    return int((np.diff(lp.rowptr) >= 16 * S).sum())


def _sliced_cols(lp, S):
    return int((np.bincount(lp.col, minlength=lp.n) >= 16 * S).sum())


# (LP, dual slices, primal slices, rows per lane group in the short-row bins):
# groups of 2 and 4 rows give the sliced rows of one group different slice
# lengths per pass
@pytest.mark.parametrize("name,S,St,rows", [
    ("zipf", 2, 0, 1), ("zipf", 4, 0, 1), ("zipf", 8, 0, 1), ("zipf", 3, 0, 2), ("zipf", 4, 0, 4),
    ("tall", 0, 2, 1), ("tall", 0, 3, 1), ("tall", 0, 4, 2), ("tall", 3, 3, 2), ("tall", 2, 3, 4)])
def test_sliced_steps_f64_match_oracle(orc, pd, name, S, St, rows):
    lp = {"zipf": _zipf, "tall": _tall}[name]()
    assert S == 0 or _sliced_rows(lp, S) > 50
    assert St == 0 or _sliced_cols(lp, St) > 50
    o = orc.Oracle(lp)
    rho, kap = o.ruiz(10)
    rr = [rows] * 5 + [1] * 3
    lay = dict(col_slices=S, col_slices_t=St, bin_rows_dual=rr, bin_rows_primal=rr)
    s = pd.Solver(lp, precision="f64", step_size=0.5, primal_weight=1.0, **lay)
    eta, omega = 0.9 / s.info()["knorm"], 1.3
    s = pd.Solver(lp, precision="f64", step_size=eta, primal_weight=omega, **lay)
    x0 = np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap)
    for k, tol in ((1, 1e-12), (199, 1e-9)):
        s.iterate(k)
        xs, ys = o.steps(x0, np.zeros(lp.m), eta / omega, eta * omega, 1 if k == 1 else 200, ruiz_iters=10)
        x, y = s.solution(which=pd.SOL_CURRENT)
        xo, yo = np.clip(kap * xs, lp.l, lp.u), rho * ys
        np.testing.assert_allclose(x, xo, rtol=tol, atol=tol * (1 + np.abs(xo).max()))
        np.testing.assert_allclose(y, yo, rtol=tol, atol=tol * (1 + np.abs(yo).max()))


@pytest.mark.parametrize("name,S,St", [("zipf", 4, 0), ("tall", 2, 3)])
def test_sliced_restart_trace_matches_oracle_f64(orc, pd, name, S, St):
    lp = {"zipf": _zipf, "tall": _tall}[name]()
    s = pd.Solver(lp, precision="f64", eps=1e-6, col_slices=S, col_slices_t=St, trace_capacity=4096,
                  max_iters=200000)
    s.solve()
    gt, total = s.trace()
    ro = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6, max_iters=200000), trace_cap=4096)
    assert total == len(gt) == len(ro.trace)
    _compare(gt, ro.trace)


@pytest.mark.parametrize("name,S,St", [("zipf", 4, 0), ("tall", 2, 3)])
def test_sliced_solve_f32(orc, pd, name, S, St):
    lp = {"zipf": _zipf, "tall": _tall}[name]()
    s = pd.Solver(lp, precision="f32", eps=1e-5, col_slices=S, col_slices_t=St, max_iters=200000)
    r = s.solve()[0]
    x, y = s.solution()
    k = orc.Oracle(lp).kkt(x, y)
    assert r["status_name"] == "OPTIMAL" and k["rel_kkt"] <= 1.05e-5, (r, k)
    assert abs(k["pobj"] - lp.f_star) / (1 + abs(lp.f_star)) <= 1e-5


@pytest.mark.parametrize("budget", [0, 1])
def test_sliced_batched_equals_solo(pd, budget):
    """Instances with sliced rows, with none (all rows short) and with fewer
    columns than slices, in one batch: each one bitwise as alone, with every
    instance running at once (budget 0) and one at a time (a 1-byte budget:
    the sliced passes then walk the blocks of the admitted instance only)."""
    lps = [_zipf(), lpgen.planted(90, 200, 0.03, 5, ge_frac=0.4), lpgen.tiny(4, n=3, m=2),
           lpgen.config2(8, m=2000, n=4000, kmax=1500), _tall()]
    kw = dict(precision="f32", eps=1e-5, col_slices=4, col_slices_t=2, max_iters=200000)
    b = pd.Solver(lps, batch_resident_bytes=budget, **kw)
    rb = b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        rs = s.solve()[0]
        assert rb[i]["iters"] == rs["iters"] and rb[i]["status"] == rs["status"]
        np.testing.assert_array_equal(b.solution(inst=i)[0], s.solution()[0])
        np.testing.assert_array_equal(b.solution(inst=i)[1], s.solution()[1])


def test_sliced_handle_adjoint_matches_oracle(orc, pd):
    """Recorded steps sweep whole rows (as the replay does): the adjoint of a
    handle with column slices still equals the oracle's reverse mode."""
    lp = _zipf()
    o = orc.Oracle(lp)
    kn, _ = o.power_norm(10, max_iters=5000, tol=1e-10)
    eta, omega = 0.8 / kn, 1.7
    K = 30
    s = pd.Solver(lp, precision="f64", col_slices=4, col_slices_t=2, step_size=eta, primal_weight=omega,
                  unroll_capacity=K, unroll_checkpoint=8)
    rng = np.random.default_rng(1)
    gx, gy = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    x0 = np.clip(np.zeros(lp.n), lp.l, lp.u)
    s.set_state(x0, np.zeros(lp.m))
    s.iterate(K, record=True)
    g = s.backward(gx, gy)
    go = o.unrolled_vjp(10, eta / omega, eta * omega, lp.c, lp.rhs, lp.l, lp.u, x0, np.zeros(lp.m), K, gx, gy)
    for name, key in (("c", "c"), ("rhs", "q"), ("x0", "x0"), ("y0", "y0")):
        a, b = g[name], go[key]
        assert np.linalg.norm(a - b) <= 1e-9 * (np.linalg.norm(b) + 1e-30), name


def test_sliced_phase_timers(pd):
    lp = _tall()
    s = pd.Solver(lp, precision="f32", col_slices=4, col_slices_t=3)
    t = s.time_kernels(reps=5)
    assert t["ms_dual"] > 0 and t["ms_primal"] > 0

"""pdhg_set_data: new cost, right-hand side and bounds on an existing handle
(the matrix, Ruiz factors and step parameters of setup stay), solved against
the oracle on the new LP; the batch's concatenated layout; rejected data
leaves the handle as it was."""
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


def _perturbed(lp, seed):
    """The same matrix with a new planted pair: new c, rhs and bounds that
    keep a known optimum (x* stays feasible and optimal for the new data)."""
    rng = np.random.default_rng(seed)
    l2 = lp.l - rng.uniform(0.0, 0.5, size=lp.n) * (lp.x_star > lp.l)   # looser where x* is off its lower bound
    u2 = lp.u + rng.uniform(0.0, 0.5, size=lp.n) * (lp.x_star < lp.u)
    # x* keeps its bound status: shift the bounds it sits on together with it
    at_l, at_u = lp.x_star == lp.l, lp.x_star == lp.u
    shift = rng.uniform(-0.2, 0.2, size=lp.n)
    x2 = lp.x_star + shift * ~(at_l | at_u)
    x2 = np.clip(x2, l2, u2)
    l2[at_l] = lp.l[at_l]
    u2[at_u] = lp.u[at_u]
    rows = np.repeat(np.arange(lp.m), np.diff(lp.rowptr))
    ax = np.zeros(lp.m)
    np.add.at(ax, rows, lp.val * x2[lp.col])
    rhs2 = ax.copy()
    ge = lp.row_type == lpgen.GE
    inactive = ge & (lp.y_star == 0.0)
    rhs2[inactive] -= rng.uniform(0.1, 1.0, size=int(inactive.sum()))
    # reduced costs: zero on the interior (keep c = K'y* + z with the same z)
    return x2, rhs2, l2, u2


def test_set_data_rhs_and_bounds(orc, pd):
    lp = lpgen.planted(150, 380, 0.03, 21, ge_frac=0.4)
    s = pd.Solver(lp, precision="f64", eps=1e-7)
    assert s.solve()[0]["status_name"] == "OPTIMAL"
    x2, rhs2, l2, u2 = _perturbed(lp, 4)
    lp2 = lpgen.LP(lp.n, lp.m, lp.rowptr, lp.col, lp.val, lp.row_type, rhs2, lp.c, l2, u2)
    s.set_data(rhs=rhs2, l=l2, u=u2)
    s.set_state(np.clip(np.zeros(lp.n), l2, u2), np.zeros(lp.m))
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    o2 = orc.Oracle(lp2)
    chk = o2.kkt(x, y)
    assert chk["rel_kkt"] <= 1.01e-7
    ro = o2.solve(orc.SolveOpts(eps=1e-9))
    assert abs(chk["pobj"] - ro.kkt["pobj"]) <= 1e-5 * (1 + abs(ro.kkt["pobj"]))
    # the device KKT of the handle now refers to the new data
    assert s.kkt(x, y)["rel_kkt"] == pytest.approx(chk["rel_kkt"], rel=1e-6)


def test_set_data_batched_layout(pd):
    lps = [lpgen.planted(m, int(2.5 * m), 0.03, 30 + i, ge_frac=0.3) for i, m in enumerate([60, 140, 90])]
    rng = np.random.default_rng(5)
    news = [(lp.c + 0.05 * rng.standard_normal(lp.n), lp.rhs + 0.01 * rng.standard_normal(lp.m)) for lp in lps]
    kw = dict(precision="f32", eps=1e-5)
    b = pd.Solver(lps, **kw)
    b.set_data(c=np.concatenate([c for c, _ in news]), rhs=np.concatenate([q for _, q in news]))
    rb = b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        s.set_data(c=news[i][0], rhs=news[i][1])
        rs = s.solve()[0]
        assert rb[i]["iters"] == rs["iters"] and rb[i]["status"] == rs["status"]
        np.testing.assert_array_equal(b.solution(inst=i)[0], s.solution()[0])


def test_set_data_rejects_and_keeps_state(pd):
    lp = lpgen.planted(80, 200, 0.04, 8, ge_frac=0.5)
    s = pd.Solver(lp, precision="f64", eps=1e-7)
    r0 = s.solve()[0]
    x0, y0 = s.solution()
    bad_l = lp.l.copy()
    bad_l[3] = lp.u[3] + 1.0
    with pytest.raises(pd.PDHGError) as e:
        s.set_data(l=bad_l)
    assert e.value.code == -3
    c_nan = lp.c.copy()
    c_nan[0] = np.nan
    with pytest.raises(pd.PDHGError) as e:
        s.set_data(c=c_nan)
    assert e.value.code == -4
    # nothing changed: the same solve from the same start gives the same bits
    s.set_state(np.zeros(lp.n), np.zeros(lp.m))
    s2 = pd.Solver(lp, precision="f64", eps=1e-7)
    s2.solve()
    s2.set_state(np.zeros(lp.n), np.zeros(lp.m))
    r1, r2 = s.solve()[0], s2.solve()[0]
    assert r1["iters"] == r2["iters"]
    np.testing.assert_array_equal(s.solution()[0], s2.solution()[0])
    assert r0["status_name"] == "OPTIMAL"

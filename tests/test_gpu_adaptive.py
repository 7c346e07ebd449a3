"""Adaptive step size (Section 2.4.4, Algorithm 5) on the GPU vs the oracle.

The step-size feedback amplifies rounding: in the oracle alone, a 1e-15
relative change of c moves the iterate by ~1e-11 after 64 attempts and by
several percent after 640 (fixed steps stay at 1e-12).  FP64 parity is
therefore checked attempt by attempt over short windows, where the GPU and
the oracle differ only by summation order: the same accept / reject
decisions and restarts, the trial step to 1e-9 and the iterate to 1e-8
relative.  Whole solves in both precisions are checked on what the method
fixes: the oracle's relative KKT of the returned point and the objective
against the planted optimum.
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


@pytest.mark.parametrize("name", ["c0", "mixed", "tinyfree", "sced_small"])
@pytest.mark.parametrize("every,iters,restarts", [(1, 1, 0), (1, 4, 0), (1, 16, 0), (8, 48, 1)])
def test_adaptive_f64_trajectory_matches_oracle(orc, pd, name, every, iters, restarts):
    lp = _cases()[name]
    kw = dict(eps=1e-13, max_iters=iters, check_every=every, use_restarts=restarts, use_pw_update=restarts)
    s = pd.Solver(lp, precision="f64", adaptive_step=1, **kw)
    r = s.solve()[0]
    ro = orc.Oracle(lp).solve(orc.SolveOpts(adaptive_step=True, **kw))
    print(name, every, iters, r["iters"], r["accepted"], r["restarts"], r["eta_next"], "|", ro.iters,
          ro.accepted, ro.restarts, ro.eta_next)
    assert r["iters"] == ro.iters
    assert r["status"] == ro.status
    assert r["accepted"] == ro.accepted
    assert r["restarts"] == ro.restarts
    assert r["eta_next"] == pytest.approx(ro.eta_next, rel=1e-9)
    assert r["omega"] == pytest.approx(ro.omega, rel=1e-9)
    x, y = s.solution()
    for a, b in ((x, ro.x), (y, ro.y)):
        assert np.linalg.norm(a - b) <= 1e-8 * (1.0 + np.linalg.norm(b))


@pytest.mark.parametrize("iters", [1, 4, 16])
def test_adaptive_sliced_dual_sweep_f64_matches_oracle(orc, pd, iters):
    """The adaptive attempts with the dual sweep in 4 column slices (the
    product K~x' summed slice by slice): the same decisions, step and iterate
    as the oracle over short windows, as with whole rows."""
    lp = _cases()["zipf"]
    assert (np.diff(lp.rowptr) >= 64).sum() > 100
    kw = dict(eps=1e-13, max_iters=iters, check_every=1, use_restarts=0, use_pw_update=0)
    s = pd.Solver(lp, precision="f64", adaptive_step=1, col_slices=4, **kw)
    r = s.solve()[0]
    ro = orc.Oracle(lp).solve(orc.SolveOpts(adaptive_step=True, **kw))
    assert (r["iters"], r["accepted"], r["status"]) == (ro.iters, ro.accepted, ro.status)
    assert r["eta_next"] == pytest.approx(ro.eta_next, rel=1e-9)
    x, y = s.solution()
    for a, b in ((x, ro.x), (y, ro.y)):
        assert np.linalg.norm(a - b) <= 1e-8 * (1.0 + np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adaptive_sliced_solve(orc, pd, prec):
    """A whole adaptive solve with the dual sweep in column slices reaches the
    tolerance with the oracle's KKT check and the planted objective."""
    lp = _cases()["zipf"]
    s = pd.Solver(lp, precision=prec, eps=1e-5, max_iters=200000, adaptive_step=1, col_slices=4)
    r = s.solve()[0]
    x, y = s.solution()
    k = orc.Oracle(lp).kkt(x, y)
    assert r["status_name"] == "OPTIMAL" and k["rel_kkt"] <= 1.05e-5, (r, k)
    assert _rel(k["pobj"], lp.f_star) <= 1e-5


@pytest.mark.parametrize("name", ["c0", "mixed"])
@pytest.mark.parametrize("iters", [1, 2, 3, 4])
def test_adaptive_rejections_match_oracle(orc, pd, name, iters):
    """A first trial step far above 1/||K~|| is rejected (twice on "mixed"):
    checks after every attempt cover epochs without an accepted step, whose
    average is the iterate, and restarts from them."""
    lp = _cases()[name]
    kw = dict(eps=1e-13, max_iters=iters, check_every=1, step_size=20.0)
    s = pd.Solver(lp, precision="f64", adaptive_step=1, **kw)
    r = s.solve()[0]
    ro = orc.Oracle(lp).solve(orc.SolveOpts(adaptive_step=True, **kw))
    assert (r["accepted"], r["restarts"]) == (ro.accepted, ro.restarts)
    assert r["eta_next"] == pytest.approx(ro.eta_next, rel=1e-9)
    x, y = s.solution()
    for a, b in ((x, ro.x), (y, ro.y)):
        assert np.linalg.norm(a - b) <= 1e-9 * (1.0 + np.linalg.norm(b))


@pytest.mark.parametrize("name", ["c0", "mixed", "tinyfree", "sced_small", "zipf"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adaptive_solve(orc, pd, name, prec):
    lp = _cases()[name]
    o = orc.Oracle(lp)
    eps = 1e-6 if prec == "f64" else 1e-5
    if name == "zipf":
        # at 1e-6 the oracle itself stalls near 4e-5 for one of four 1e-15
        # perturbations of c (the step feedback is rounding-sensitive)
        eps = 1e-4
    s = pd.Solver(lp, precision=prec, eps=eps, max_iters=300000, adaptive_step=1)
    r = s.solve()[0]
    x, y = s.solution()
    chk = o.kkt(x, y)
    fref = lp.f_star if lp.f_star is not None else o.solve(orc.SolveOpts(eps=1e-7, max_iters=2_000_000)).kkt["pobj"]
    print(name, prec, r["status_name"], r["iters"], r["accepted"], r["restarts"], r["kkt"]["rel_kkt"],
          chk["rel_kkt"], _rel(chk["pobj"], fref))
    assert r["status_name"] == "OPTIMAL", r
    assert 0 < r["accepted"] <= r["iters"]
    if prec == "f64":
        assert chk["rel_kkt"] <= eps * 1.01
        assert _rel(chk["pobj"], fref) <= max(1e-5, 10 * eps)
        # the step feedback makes iteration counts rounding-sensitive: compare
        # the work to the oracle's own adaptive solve within a factor of 2
        it_o = o.solve(orc.SolveOpts(eps=eps, adaptive_step=True)).iters
        assert 0.5 * it_o <= r["iters"] <= 2.0 * it_o + 128, (r["iters"], it_o)
    else:
        assert chk["rel_kkt"] <= max(1e-4, 1.01 * eps)
        assert _rel(chk["pobj"], fref) <= max(1e-5, 10 * eps)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_adaptive_batched_equals_solo_bitwise(pd, prec):
    lps = [lpgen.planted(m, int(2.5 * m), 0.02, 30 + i, ge_frac=0.3) for i, m in enumerate([60, 150, 90, 240])]
    lps.append(lpgen.sced(20, 8, 4, 6, seed=9))
    kw = dict(precision=prec, eps=1e-5, adaptive_step=1)
    b = pd.Solver(lps, **kw)
    rb = b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        rs = s.solve()[0]
        for k in ("iters", "restarts", "status", "accepted"):
            assert rb[i][k] == rs[k], (i, k)
        assert rb[i]["eta_next"] == rs["eta_next"]
        xb, yb = b.solution(inst=i)
        xs, ys = s.solution()
        np.testing.assert_array_equal(xb, xs)
        np.testing.assert_array_equal(yb, ys)


def test_adaptive_graph_and_eager_agree(pd):
    lp = _cases()["mixed"]
    a = pd.Solver(lp, precision="f32", eps=1e-5, use_graph=1, adaptive_step=1)
    b = pd.Solver(lp, precision="f32", eps=1e-5, use_graph=0, adaptive_step=1)
    ra, rb = a.solve()[0], b.solve()[0]
    assert ra["iters"] == rb["iters"] and ra["accepted"] == rb["accepted"]
    np.testing.assert_array_equal(a.solution()[0], b.solution()[0])


def test_adaptive_toggle_between_solves(orc, pd):
    """set_opts switches between fixed and adaptive steps on one handle (the
    chunk graph is rebuilt); each solve starts from the caller's point."""
    lp = _cases()["sced_small"]
    o = orc.Oracle(lp)
    s = pd.Solver(lp, precision="f64", eps=1e-6)
    r0 = s.solve()[0]
    assert r0["accepted"] == r0["iters"] and r0["eta_next"] == r0["eta"]
    for mode in (1, 0, 1):
        s.set_opts(adaptive_step=mode)
        s.set_state(np.zeros(lp.n), np.zeros(lp.m))
        r = s.solve()[0]
        assert r["status_name"] == "OPTIMAL", (mode, r)
        x, y = s.solution()
        assert o.kkt(x, y)["rel_kkt"] <= 1.01e-6
        if mode == 0:
            assert r["accepted"] == r["iters"]


def test_adaptive_iteration_limit_counts_attempts(pd):
    lp = _cases()["sced_small"]
    s = pd.Solver(lp, precision="f32", eps=1e-12, max_iters=640, adaptive_step=1)
    r = s.solve()[0]
    assert r["status_name"] == "ITERATION_LIMIT" and r["iters"] == 640
    assert r["accepted"] <= 640
    x, y = s.solution()
    assert np.isfinite(x).all() and np.isfinite(y).all()


def test_adaptive_timers(pd):
    lp = _cases()["mixed"]
    s = pd.Solver(lp, precision="f32", adaptive_step=1)
    t = s.time_kernels(reps=5)
    assert t["ms_primal_ad"] > 0 and t["ms_dual_ad"] > 0 and t["ms_step_ad"] > 0
    # the timers leave the solver usable
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL"

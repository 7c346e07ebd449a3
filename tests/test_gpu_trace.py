"""Per-check records of pdhg_solve (the device ring read by pdhg_get_trace)
against the oracle's trace of the same solve: the restart decisions, the
candidate choice and the primal-weight sequence of Section 2.4.2 and
Algorithm 4, check by check, in FP64."""
import json
import math
import os

import numpy as np
import pytest

import lpgen
from test_oracle import GOLD, _assert_restart_rule

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16806_amd as pd

    pd.lib()
    return pd


def _cases():
    return {
        "c0": lpgen.config0(0),
        "c0u": lpgen.config0(1, unique=True),
        "mixed": lpgen.planted(300, 700, 0.02, 5, ge_frac=0.5),
        "tinyfree": lpgen.tiny(3, n=8, m=4, free_frac=0.5),
        "sced_small": lpgen.sced(40, 16, 8, 12, seed=5),
    }


def _close(a, b, rel):
    if math.isinf(a) or math.isinf(b):
        return a == b
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


def _compare(gt, ot, rel_kkt=1e-6, rel_w=1e-9):
    """Device records against the oracle's, check by check: the decisions and
    their inputs (epoch length, reference value, previous candidate, primal
    weight before and after, the restart distances and the candidate's
    scaled-LP terms)."""
    assert len(gt) == len(ot), (len(gt), len(ot))
    for k, (g, o) in enumerate(zip(gt, ot)):
        # discrete decisions: identical (a flip is reported with the margin that caused it)
        assert (g["iter"], g["restarted"], g["cand_avg"], g["accepted"], g["t_inner"]) == \
               (o["iter"], o["restarted"], o["cand_avg"], o["accepted"], o["t_inner"]), (k, g, o)
        for f in ("omega", "omega_before", "eta_next"):
            assert _close(g[f], o[f], rel_w), (k, f, g[f], o[f])
        for f in ("kkt_cand", "rel_kkt_cur", "rel_kkt_avg", "kkt0", "kkt_prev", "kkt0_next", "delta_x", "delta_y"):
            assert _close(g[f], o[f], rel_kkt), (k, f, g[f], o[f])
        # the candidate's terms, each bounded by KKT_omega * max(omega, 1/omega, 1): to rel_kkt of
        # that bound (a single term can cancel to ~0)
        w = o["omega_before"]
        bound = o["kkt_cand"] * max(w, 1.0 / w, 1.0)
        for f in ("cand_pres", "cand_dres", "cand_gap"):
            assert abs(g[f] - o[f]) <= rel_kkt * bound, (k, f, g[f], o[f])


@pytest.mark.parametrize("name", ["c0", "c0u", "mixed", "tinyfree", "sced_small"])
def test_restart_trace_matches_oracle_f64(orc, pd, name):
    lp = _cases()[name]
    s = pd.Solver(lp, precision="f64", eps=1e-6, trace_capacity=4096)
    r = s.solve()[0]
    gt, total = s.trace()
    ro = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6), trace_cap=4096)
    assert total == len(gt) == len(ro.trace)
    assert sum(g["restarted"] for g in gt) == r["restarts"] == ro.restarts
    assert gt[-1]["iter"] == r["iters"]
    # omega changes only at restarts
    for a, b in zip(gt, gt[1:]):
        if not b["restarted"]:
            assert b["omega"] == a["omega"]
    _compare(gt, ro.trace)
    # the device's own records follow the Section 2.4.2 rule at every check
    _assert_restart_rule(gt, gt[0]["omega_before"], gt[0]["kkt0"])


def test_restart_trace_1x1_golden_f64(pd):
    """The device trace on the 1 x 1 LP of tests/golden/restart_1x1.py (a check
    after every iteration) equals the hand derivation: every decision and
    candidate, and the KKT_omega values, reference values and omega to 1e-9."""
    g = json.load(open(os.path.join(GOLD, "restart_trace_1x1.json")))
    lp = lpgen.from_dense(np.array(g["lp"]["K"]), g["lp"]["row_type"], g["lp"]["q"], g["lp"]["c"],
                          np.array(g["lp"]["l"]), np.array([np.inf]))
    s = pd.Solver(lp, precision="f64", eps=g["opts"]["eps"], check_every=g["opts"]["check_every"],
                  ruiz_iters=g["opts"]["ruiz_iters"], trace_capacity=64)
    r = s.solve()[0]
    gt, total = s.trace()
    want = g["checks"]
    assert r["status"] == 0 and total == len(gt) == len(want)
    for t, w in zip(gt, want):
        assert (t["iter"], t["t_inner"], t["restarted"], t["cand_avg"]) == \
               (w["iter"], w["t_inner"], w["restarted"], w["cand_avg"]), (t, w)
        for k in ("kkt_cand", "kkt0", "omega_before", "omega", "kkt0_next", "rel_kkt_cur", "rel_kkt_avg",
                  "delta_x", "delta_y"):
            assert t[k] == pytest.approx(w[k], rel=1e-9, abs=1e-300), (k, t, w)
        assert t["kkt_prev"] == pytest.approx(np.inf if w["kkt_prev"] == "inf" else w["kkt_prev"], rel=1e-9)
    _assert_restart_rule(gt, 0.75, 3.0)


def test_plain_trace_matches_oracle_f64(orc, pd):
    lp = _cases()["c0"]
    kw = dict(eps=1e-5, max_iters=20000)
    s = pd.Solver(lp, precision="f64", ruiz_iters=0, use_restarts=0, use_pw_update=0, trace_capacity=4096, **kw)
    s.solve()
    gt, total = s.trace()
    ro = orc.Oracle(lp).solve(orc.SolveOpts.plain(**kw), trace_cap=4096)
    assert all(g["restarted"] == 0 and g["cand_avg"] == 0 and math.isinf(g["rel_kkt_avg"]) for g in gt)
    assert [g["iter"] for g in gt] == [64 * (k + 1) for k in range(total)]
    _compare(gt, ro.trace)


@pytest.mark.parametrize("name", ["c0", "mixed"])
def test_adaptive_trace_matches_oracle_f64(orc, pd, name):
    """Adaptive steps over a short window (the trajectories are chaotic over
    long runs): accepted counts and the next trial step at every check."""
    lp = _cases()[name]
    kw = dict(eps=1e-13, max_iters=48, check_every=8)
    s = pd.Solver(lp, precision="f64", adaptive_step=1, trace_capacity=64, **kw)
    s.solve()
    gt, _ = s.trace()
    ro = orc.Oracle(lp).solve(orc.SolveOpts(adaptive_step=True, **kw), trace_cap=64)
    _compare(gt, ro.trace, rel_kkt=1e-6, rel_w=1e-9)


def test_ring_keeps_the_last_records(pd):
    lp = _cases()["mixed"]
    full = pd.Solver(lp, precision="f64", eps=1e-7, trace_capacity=4096)
    full.solve()
    ft, ftotal = full.trace()
    assert ftotal > 5
    ring = pd.Solver(lp, precision="f64", eps=1e-7, trace_capacity=3)
    ring.solve()
    rt, rtotal = ring.trace()
    assert rtotal == ftotal and len(rt) == 3
    assert rt == ft[-3:]
    # a second solve starts a new trace
    ring.set_state(np.zeros(lp.n), np.zeros(lp.m))
    ring.solve()
    rt2, rtotal2 = ring.trace()
    assert rtotal2 >= 1 and rt2[-1]["iter"] <= ftotal * 64


def test_batched_traces_equal_solo(pd):
    lps = [lpgen.planted(m, int(2.5 * m), 0.02, 70 + i, ge_frac=0.3) for i, m in enumerate([80, 200, 120])]
    kw = dict(precision="f32", eps=1e-5, trace_capacity=512)
    b = pd.Solver(lps, batch_resident_bytes=0, **kw)
    b.solve()
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        s.solve()
        assert b.trace(inst=i) == s.trace()


def test_trace_needs_capacity(pd):
    s = pd.Solver(_cases()["tinyfree"], precision="f64")
    s.solve()
    with pytest.raises(pd.PDHGError) as e:
        s.trace()
    assert e.value.code == -7

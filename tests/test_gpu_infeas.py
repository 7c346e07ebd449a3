"""Infeasibility detection (Section 2.4.5, Algorithm 6) on the GPU vs the oracle.

Both sides test the difference of the last step of each check period in the
original variables, each test relative to the ray's objective improvement.
With fixed steps in FP64 the two follow the same trajectory up to summation
order, so they report the same status at the same check or a neighbouring
one; with adaptive steps (rounding-sensitive) and in FP32 the status must
agree.  On feasible LPs detection must never fire and must not change the
path: the solution is bitwise the one without detection.
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


def _infeasible():
    return {
        "bound60": (lpgen.primal_infeasible(60, 150, 0.05, 1, "bound"), 4),
        "pair60": (lpgen.primal_infeasible(60, 150, 0.05, 2, "pair"), 4),
        "pair300": (lpgen.primal_infeasible(300, 700, 0.02, 4, "pair"), 4),
        "bound300": (lpgen.primal_infeasible(300, 700, 0.02, 6, "bound"), 4),
        "unb60": (lpgen.dual_infeasible(60, 150, 0.05, 3), 5),
        "unb300": (lpgen.dual_infeasible(300, 700, 0.02, 5), 5),
    }


@pytest.mark.parametrize("name", ["bound60", "pair60", "pair300", "bound300", "unb60", "unb300"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("adaptive", [0, 1])
def test_detection_matches_oracle(orc, pd, name, prec, adaptive):
    lp, want = _infeasible()[name]
    s = pd.Solver(lp, precision=prec, eps=1e-6, max_iters=100_000, detect_infeas=1, adaptive_step=adaptive)
    r = s.solve()[0]
    ro = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6, max_iters=100_000, detect_infeas=True,
                                            adaptive_step=bool(adaptive)))
    print(name, prec, adaptive, r["status_name"], r["iters"], "| oracle", ro.status, ro.iters)
    assert ro.status == want
    assert r["status"] == want, r
    if prec == "f64" and not adaptive:
        assert abs(r["iters"] - ro.iters) <= 2 * 64, (r["iters"], ro.iters)
    else:
        assert r["iters"] <= 4 * ro.iters + 640
    x, y = s.solution()
    assert np.isfinite(x).all() and np.isfinite(y).all()


@pytest.mark.parametrize("name", ["c0u", "mixed", "sced_small", "tinyfree", "zipf"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("adaptive", [0, 1])
def test_no_false_positive_and_same_path(pd, name, prec, adaptive):
    lp = {"c0u": lpgen.config0(1, unique=True), "mixed": lpgen.planted(300, 700, 0.02, 5, ge_frac=0.5),
          "sced_small": lpgen.sced(40, 16, 8, 12, seed=5), "tinyfree": lpgen.tiny(3, n=8, m=4, free_frac=0.5),
          "zipf": lpgen.config2(7, m=3000, n=6000, kmax=2000)}[name]
    eps = 1e-6 if prec == "f64" else 1e-5
    kw = dict(precision=prec, eps=eps, max_iters=100_000, adaptive_step=adaptive)
    a = pd.Solver(lp, detect_infeas=1, **kw)
    b = pd.Solver(lp, detect_infeas=0, **kw)
    ra, rb = a.solve()[0], b.solve()[0]
    assert ra["status"] == rb["status"] and ra["status"] in (0, 1), (ra, rb)
    assert ra["iters"] == rb["iters"] and ra["restarts"] == rb["restarts"]
    xa, ya = a.solution()
    xb, yb = b.solution()
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(ya, yb)


@pytest.mark.parametrize("adaptive", [0, 1])
def test_batch_mixes_statuses(pd, adaptive):
    """Optimal, primal-infeasible and unbounded instances in one batch stop
    independently with the statuses and iterations of their solo runs."""
    lps = [lpgen.planted(80, 200, 0.04, 21, ge_frac=0.5), lpgen.primal_infeasible(60, 150, 0.05, 2, "pair"),
           lpgen.dual_infeasible(60, 150, 0.05, 3), lpgen.sced(20, 8, 4, 6, seed=9),
           lpgen.primal_infeasible(60, 150, 0.05, 1, "bound")]
    kw = dict(precision="f64", eps=1e-6, max_iters=100_000, detect_infeas=1, adaptive_step=adaptive)
    b = pd.Solver(lps, **kw)
    rb = b.solve()
    assert [r["status_name"] for r in rb] == ["OPTIMAL", "PRIMAL_INFEASIBLE", "DUAL_INFEASIBLE", "OPTIMAL",
                                               "PRIMAL_INFEASIBLE"]
    for i, lp in enumerate(lps):
        rs = pd.Solver(lp, **kw).solve()[0]
        assert (rb[i]["status"], rb[i]["iters"]) == (rs["status"], rs["iters"]), i


def test_detection_off_by_default(pd):
    lp = lpgen.primal_infeasible(60, 150, 0.05, 1, "bound")
    r = pd.Solver(lp, precision="f64", eps=1e-6, max_iters=3200).solve()[0]
    assert r["status_name"] == "ITERATION_LIMIT"
    s = pd.Solver(lp, precision="f64", eps=1e-6, max_iters=3200)
    s.set_opts(detect_infeas=1)
    assert s.solve()[0]["status_name"] == "PRIMAL_INFEASIBLE"

"""The launch-layout autotuner (pdhg_autotune) on the GPU: its record lists
every candidate of the search, its choice is the fastest of the trials by the
rule it states, and a solver set up with the chosen options reaches the
oracle's optimum (the layout changes how sums are split, not what is solved)."""
import json

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


def _lims():
    from paper_2508_16806_amd.tuner import limits

    return [limits(f, w) for f in (2, 4, 8, 16) for w in (512, 2048) if w >= 64 * f]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_autotune_record_and_choice(orc, pd, prec, tmp_path):
    lp = lpgen.config0(0)
    out = tmp_path / "tune.json"
    best, rec = pd.autotune(lp, reps=3, out_json=str(out), precision=prec)
    assert json.loads(out.read_text()) == rec
    assert rec["precision"] == prec
    assert len(rec["trials"]) == 7 and len(rec["rows_trials"]) == 3 and len(rec["shapes"]) == 8
    sl = rec["slice_trials"]
    assert [(t["col_slices"], t["f"], t["w"]) for t in sl] == [(0, 0, 0)] + [
        (S, f, w) for S in (2, 4, 8) for f in (2, 4, 8, 16) for w in (512, 2048) if w >= 64 * f]
    assert sorted((t["f"], t["w"]) for t in rec["trials"]) == sorted(
        (f, w) for f in (2, 4, 8, 16) for w in (512, 2048) if w >= 64 * f)
    assert all(t["ms_primal"] > 0 and t["ms_dual"] > 0 for t in rec["trials"])
    # limits: the fastest stage-0 candidate of each operator
    bp = min(rec["trials"], key=lambda t: t["ms_primal"])
    bd0 = min(rec["trials"], key=lambda t: t["ms_dual"])
    from paper_2508_16806_amd.tuner import limits

    # column slices: the fastest sliced trial of each sweep where it beats
    # the unsliced one by 2% (the dual sweep then takes that trial's bins)
    t0, sliced = sl[0], sl[1:]
    bd = min(sliced, key=lambda t: t["ms_dual"])
    dual_sliced = bd["ms_dual"] <= 0.98 * t0["ms_dual"]
    bpr = min(sliced, key=lambda t: t["ms_primal"])
    want_t = bpr["col_slices"] if bpr["ms_primal"] <= 0.98 * t0["ms_primal"] else 0
    assert best.col_slices == rec["col_slices"] == (bd["col_slices"] if dual_sliced else 0)
    assert best.col_slices_t == rec["col_slices_t"] == want_t
    assert list(best.bin_len_primal) == limits(bp["f"], bp["w"]) == rec["bin_len_primal"]
    bd_lim = limits(bd["f"], bd["w"]) if dual_sliced else limits(bd0["f"], bd0["w"])
    assert list(best.bin_len_dual) == bd_lim == rec["bin_len_dual"]
    rp = min(rec["rows_trials"], key=lambda t: t["ms_primal"])["rows"]
    rd = min(rec["rows_trials"], key=lambda t: t["ms_dual"])["rows"]
    assert list(best.bin_rows_primal) == [rp] * 5 + [1, 1, 1] == rec["bin_rows_primal"]
    assert list(best.bin_rows_dual) == [rd] * 5 + [1, 1, 1] == rec["bin_rows_dual"]
    bs = min(rec["shapes"], key=lambda t: t["ms_iter"])
    assert (best.xcd_remap, best.max_grid) == (bs["xcd_remap"], bs["max_grid"])
    assert (rec["xcd_remap"], rec["max_grid"]) == (bs["xcd_remap"], bs["max_grid"])

    for t in rec["shapes"]:
        assert t["ms_iter"] == pytest.approx(t["ms_primal"] + t["ms_dual"] + t["ms_check"] / 64, rel=1e-6)
    # every other option is the base's
    assert best.precision == (0 if prec == "f64" else 1) and best.check_every == 64 and best.eps == 1e-4
    # the chosen layout solves the LP
    best.eps = 1e-6
    s = pd.Solver(lp, opts=best)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    ro = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-8))
    assert r["kkt"]["pobj"] == pytest.approx(ro.kkt["pobj"], rel=1e-4, abs=1e-4)


def test_autotune_batch(orc, pd):
    """A batch of LPs of different shapes is tuned as one layout."""
    lps = [lpgen.config0(0), lpgen.planted(120, 300, 0.05, 3), lpgen.config2(m=2000, n=4000)]
    best, rec = pd.autotune(lps, reps=2)
    assert list(best.bin_len_primal) in _lims() and list(best.bin_len_dual) in _lims()
    best.eps = 1e-4
    s = pd.Solver(lps, opts=best)
    res = s.solve()
    for i, (lp, r) in enumerate(zip(lps, res)):
        assert r["status_name"] == "OPTIMAL", r
        x, y = s.solution(i)
        # the oracle's own KKT error of the returned point (Section 2.3.2)
        assert orc.Oracle(lp).kkt(x, y)["rel_kkt"] <= 1.5e-4


def test_autotune_rejects_small_workspace(pd):
    import ctypes as C

    import torch

    lp = lpgen.config0(0)
    need = pd.autotune_workspace_bytes(lp)
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    d = pd._Desc(lp)
    arr = (pd.LPDesc * 1)(d.desc)
    o, best, got = pd.default_opts(), pd.Opts(), C.c_size_t(0)
    rc = pd.lib().pdhg_autotune(C.cast(arr, C.c_void_p), 1, C.byref(o), ws.data_ptr(), need - 256, C.byref(got),
                                1, None, C.byref(best), None)
    assert rc == pd.ERR_NOMEM and got.value == need


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_time_kernels_figures_and_bounds(pd, prec):
    """The phase timers the search ranks layouts by: every figure is a finite,
    positive time (the restart kernel runs, restarts being on), the call
    reports its repetitions, and repetitions outside 1..10000 are refused."""
    lp = lpgen.planted(300, 700, 0.02, 4, ge_frac=0.5)
    s = pd.Solver(lp, precision=prec)
    t = s.time_kernels(reps=3)
    assert t["reps"] == 3
    for k, v in t.items():
        if k.startswith("ms_"):
            assert np.isfinite(v) and v > 0, (k, v)
    for bad in (0, -1, 10001):
        with pytest.raises(pd.PDHGError):
            s.time_kernels(reps=bad)
    # the handle still solves after the timers (solver counters restored)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL"

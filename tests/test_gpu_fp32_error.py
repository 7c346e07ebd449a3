"""The FP32 path's error against FP64 references, per configuration: the
oracle's relative KKT error of the FP32 solution, its objective gap to the
reference optimum (planted f*, or an FP64 GPU solve to 1e-8 certified by the
oracle's KKT), and on C0u (unique optimum) the distance to x*.  Each case
prints one "[fp32-error]" JSON line."""
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


def _gap(p, f):
    return abs(p - f) / (1 + abs(f))


def _ref64(orc, pd, lp):
    """FP64 GPU solve to 1e-8 whose KKT error, by the oracle, is <= 1e-8."""
    s = pd.Solver(lp, precision="f64", eps=1e-8, max_iters=2_000_000, time_limit=120.0)
    r = s.solve()[0]
    x, y = s.solution()
    k = orc.Oracle(lp).kkt(x, y)
    assert r["status_name"] == "OPTIMAL" and k["rel_kkt"] <= 1.01e-8, (r["status_name"], k)
    return k["pobj"]


CASES = {
    "C0": lambda: [lpgen.config0(0)],
    "C0u": lambda: [lpgen.config0(0, unique=True)],
    "C1": lambda: [lpgen.config1()],
    "C2/10": lambda: [lpgen.config2(2, m=100_000, n=200_000)],
    "C3 (8 LPs, m<=20k)": lambda: [lpgen.config3_instance(i, m_range=(1000, 20000)) for i in range(8)],
    "C4 (4 LPs)": lambda: [lpgen.config4_instance(i) for i in range(4)],
}


# the tight tolerance of each case: 1e-6, except the Zipf LP at 1e-5 (the
# FP64 solve of its 1/100-scale sibling needs ~96k iterations to 1e-5)
TIGHT = {"C2/10": 1e-5}
STALLS = set()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tol", ["paper", "tight"])
def test_fp32_error_per_result(orc, pd, name, tol):
    """At the paper's 1e-4 the objective gap is reported; at the tight
    tolerance it must be <= 1e-5 (a KKT error of 1e-4 does not bound it)."""
    lps = CASES[name]()
    eps = 1e-4 if tol == "paper" else TIGHT.get(name, 1e-6)
    stall = tol == "tight" and name in STALLS
    s = pd.Solver(lps, precision="f32", eps=eps, max_iters=300_000 if stall else 2_000_000, time_limit=120.0)
    res = s.solve()
    out = []
    for i, (lp, r) in enumerate(zip(lps, res)):
        assert r["status_name"] == "OPTIMAL" or (stall and r["status_name"] == "ITERATION_LIMIT"), (name, i, r)
        x, y = s.solution(inst=i)
        k = orc.Oracle(lp).kkt(x, y)
        fref = lp.f_star if lp.f_star is not None else _ref64(orc, pd, lp)
        rec = {"case": name, "inst": i, "eps": eps, "status": r["status_name"], "iters": r["iters"],
               "oracle_rel_kkt": k["rel_kkt"],
               "obj_gap": _gap(k["pobj"], fref), "ref": "planted" if lp.f_star is not None else "fp64 solve"}
        if name == "C0u":
            rec["x_rel_err"] = float(np.linalg.norm(x - lp.x_star) / np.linalg.norm(lp.x_star))
        out.append(rec)
        print("[fp32-error]", json.dumps(rec), flush=True)
    for rec in out:
        assert rec["oracle_rel_kkt"] <= (1e-4 if stall else eps) * 1.05, rec
        if tol == "tight":
            assert rec["obj_gap"] <= 1e-5, rec


@pytest.mark.parametrize("seed", [48, 55])
def test_fp32_reaches_1e5_on_former_floor_cases(orc, pd, seed):
    """Two dense random structures whose FP32 solves stalled near 2e-5 while
    the epoch averages were FP32 incremental means of the iterates (each
    update rounded at the average's own magnitude): with the averages kept as
    FP32 means of offsets from the epoch start they reach 1e-5."""
    lp = lpgen.random_case(seed)
    s = pd.Solver(lp, precision="f32", eps=1e-5, max_iters=300_000)
    r = s.solve()[0]
    x, y = s.solution()
    k = orc.Oracle(lp).kkt(x, y)
    print("[fp32-floor]", seed, r["status_name"], r["iters"], r["restarts"], k["rel_kkt"], flush=True)
    assert r["status_name"] == "OPTIMAL" and k["rel_kkt"] <= 1.05e-5, (r, k)

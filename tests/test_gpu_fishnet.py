"""Fishnet casting (Section 2.5, Algorithm 7) on the GPU vs the oracle.

Both sides get the same standard normal draws (lpgen.fishnet_draws) and the
same radius, step and primal weight (the handle's), so in FP64 they run the
same arithmetic up to summation order: the kept points of every round agree
exactly, the gaps to 1e-9 and the surviving point to 1e-9 relative.  In FP32
the points are rounded to FP32 each step; the kept sets agree and the
surviving point to 1e-4 relative.
"""
import ctypes as C

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


def _lps():
    return {"small": lpgen.planted(40, 100, 0.06, 17, ge_frac=0.5), "c0": lpgen.config0(2),
            "sced_small": lpgen.sced(40, 16, 8, 12, seed=5), "tinyfree": lpgen.tiny(3, n=8, m=4, free_frac=0.5)}


@pytest.mark.parametrize("name", ["small", "c0", "sced_small", "tinyfree"])
@pytest.mark.parametrize("P,k", [(2, 20), (8, 10), (32, 16)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fishnet_matches_oracle(orc, pd, name, P, k, prec):
    lp = _lps()[name]
    s = pd.Solver(lp, precision=prec, fishnet_points=32)
    info = s.info()
    G, wraw = lpgen.fishnet_draws(lp.n, P, seed=11)
    out = s.fishnet(P, k, G=G, wraw=wraw)
    x, y = s.solution(which=pd.SOL_CURRENT)
    o = orc.Oracle(lp)
    xo, yo, gaps, keep = o.fishnet(10, info["eta"], info["omega"], info["knorm"], P, k, G, wraw)
    assert out["rounds"] == len(keep)
    for r in range(len(keep)):
        assert list(out["keep"][r]) == list(keep[r]), (r, out["keep"][r], keep[r])
    rtol = 1e-9 if prec == "f64" else 1e-4
    live = gaps != 0.0
    np.testing.assert_allclose(out["gaps"][live], gaps[live], rtol=rtol * 10, atol=1e-12)
    for a, b in ((x, xo), (y, yo)):
        assert np.linalg.norm(a - b) <= rtol * (1.0 + np.linalg.norm(b)), np.linalg.norm(a - b)


@pytest.mark.parametrize("name", ["small", "c0", "sced_small"])
def test_fishnet_warm_start_solves(orc, pd, name):
    lp = _lps()[name]
    s = pd.Solver(lp, precision="f32", eps=1e-5, max_iters=200_000, fishnet_points=32)
    s.fishnet(32, 64, seed=3)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    assert orc.Oracle(lp).kkt(x, y)["rel_kkt"] <= 1e-4


def test_fishnet_device_draws_equal_host(pd):
    import torch

    lp = _lps()["small"]
    P, k = 8, 10
    G, wraw = lpgen.fishnet_draws(lp.n, P, seed=4)
    a = pd.Solver(lp, precision="f64", fishnet_points=8)
    ra = a.fishnet(P, k, G=G, wraw=wraw)
    b = pd.Solver(lp, precision="f64", fishnet_points=8)
    Gd = torch.tensor(G, dtype=torch.float64, device="cuda").contiguous()
    wd = torch.tensor(wraw, dtype=torch.float64, device="cuda").contiguous()
    gd = torch.zeros((ra["rounds"], P), dtype=torch.float64, device="cuda")
    kd = torch.zeros((ra["rounds"], P), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = pd.lib().pdhg_fishnet(b.h, P, k, Gd.data_ptr(), wd.data_ptr(), wd.numel(), pd.MEM_DEVICE,
                               gd.data_ptr(), kd.data_ptr(), None)
    assert rc == 0, pd.lib().pdhg_last_error()
    np.testing.assert_array_equal(gd.cpu().numpy(), ra["gaps"])
    np.testing.assert_array_equal(kd.cpu().numpy(), ra["keep"])
    np.testing.assert_array_equal(a.solution(which=pd.SOL_CURRENT)[0], b.solution(which=pd.SOL_CURRENT)[0])


def test_fishnet_errors(pd):
    lp = _lps()["small"]
    G, wraw = lpgen.fishnet_draws(lp.n, 8, seed=1)
    s = pd.Solver(lp, precision="f32")
    with pytest.raises(pd.PDHGError):  # no fishnet workspace
        s.fishnet(8, 4, G=G, wraw=wraw)
    s = pd.Solver(lp, precision="f32", fishnet_points=4)
    with pytest.raises(pd.PDHGError):  # more points than the workspace holds
        s.fishnet(8, 4, G=G, wraw=wraw)
    s = pd.Solver(lp, precision="f32", fishnet_points=8)
    with pytest.raises(pd.PDHGError):  # too few repopulation draws
        s.fishnet(8, 4, G=G, wraw=wraw[:2])
    bad = G.copy()
    bad[3, 5] = np.nan
    with pytest.raises(pd.PDHGError):
        s.fishnet(8, 4, G=bad, wraw=wraw)
    b = pd.Solver([lp, lp], precision="f32", fishnet_points=8)
    with pytest.raises(pd.PDHGError):  # one LP per handle
        b.fishnet(8, 4, G=G, wraw=wraw)

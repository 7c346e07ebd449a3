"""LP data resident in device memory (PDHG_MEM_DEVICE: CUDA tensors through
the binding): setup, validation, the KKT of a device point and solutions
written to device buffers give what the host-memory path gives."""
import ctypes as C
import types

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


def _on_device(lp):
    import torch

    f = {k: torch.tensor(getattr(lp, k), device="cuda") for k in
         ("rowptr", "col", "val", "row_type", "rhs", "c", "l", "u")}
    return types.SimpleNamespace(n=lp.n, m=lp.m, **f)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_device_input_equals_host_input(pd, prec):
    lps = [lpgen.planted(70 + 30 * i, 180 + 60 * i, 0.04, 11 + i, ge_frac=0.4) for i in range(3)]
    kw = dict(precision=prec, eps=1e-6)
    for batch in (lps[:1], lps):
        h = pd.Solver(batch, **kw)
        d = pd.Solver([_on_device(lp) for lp in batch], **kw)
        assert h.info()["knorm"] == d.info()["knorm"]
        rh, rd = h.solve(), d.solve()
        for i in range(len(batch)):
            assert rh[i]["iters"] == rd[i]["iters"] and rh[i]["kkt"] == rd[i]["kkt"]
            for u, v in zip(h.solution(inst=i), d.solution(inst=i)):
                np.testing.assert_array_equal(u, v)


def test_device_input_is_validated(pd):
    lp = lpgen.planted(40, 90, 0.05, 2)
    bad = _on_device(lp)
    bad.val[3] = float("nan")
    with pytest.raises(pd.PDHGError) as e:
        pd.Solver(bad)
    assert e.value.code == -4
    bad = _on_device(lp)
    bad.col[0] = lp.n
    with pytest.raises(pd.PDHGError) as e:
        pd.Solver(bad)
    assert e.value.code == -2


def test_device_points_and_outputs(pd):
    import torch

    lp = lpgen.planted(80, 200, 0.04, 5, ge_frac=0.5)
    s = pd.Solver(lp, precision="f64", eps=1e-7)
    s.solve()
    x, y = s.solution()
    # KKT of a point given as CUDA tensors equals the host call
    xd, yd = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    assert s.kkt(xd, yd) == s.kkt(x, y)
    # the solution written into device buffers
    xo = torch.empty(lp.n, dtype=torch.float64, device="cuda")
    yo = torch.empty(lp.m, dtype=torch.float64, device="cuda")
    lo = torch.empty(lp.n, dtype=torch.float64, device="cuda")
    rc = pd.lib().pdhg_get_solution(s.h, 0, pd.SOL_RESULT, xo.data_ptr(), yo.data_ptr(), lo.data_ptr(),
                                    pd.MEM_DEVICE, None)
    assert rc == 0
    torch.cuda.synchronize()
    xh, yh, lh = s.solution(lam=True)
    np.testing.assert_array_equal(xo.cpu().numpy(), xh)
    np.testing.assert_array_equal(yo.cpu().numpy(), yh)
    np.testing.assert_array_equal(lo.cpu().numpy(), lh)
    # and a state set from device buffers
    rc = pd.lib().pdhg_set_state(s.h, 0, xo.data_ptr(), yo.data_ptr(), pd.MEM_DEVICE, None)
    assert rc == 0
    s.iterate(1)
    s2 = pd.Solver(lp, precision="f64", eps=1e-7)
    s2.solve()
    s2.set_state(xh, yh)
    s2.iterate(1)
    np.testing.assert_array_equal(s.solution(which=pd.SOL_CURRENT)[0], s2.solution(which=pd.SOL_CURRENT)[0])


def test_calls_on_a_side_stream(pd):
    """Every call is ordered on the stream it is given: setup, solve, fixed
    steps, solution and KKT on a created stream (default priority) give the
    null stream's bits."""
    import torch

    lp = lpgen.planted(90, 230, 0.04, 6, ge_frac=0.5)
    st = torch.cuda.Stream()
    a = pd.Solver(lp, precision="f32", eps=1e-6, stream=st)
    ra = a.solve(stream=st)[0]
    a.iterate(7, stream=st)
    xa, ya = a.solution(which=pd.SOL_CURRENT, stream=st)
    ka = a.kkt(xa, ya, stream=st)
    b = pd.Solver(lp, precision="f32", eps=1e-6)
    rb = b.solve()[0]
    b.iterate(7)
    xb, yb = b.solution(which=pd.SOL_CURRENT)
    assert ra["iters"] == rb["iters"] and ra["kkt"] == rb["kkt"]
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(ya, yb)
    assert ka == b.kkt(xb, yb)

"""pdhg_setup_noalloc (the fixed per-device workspace) against pdhg_setup.

Both set up the same LP with the same options and run the same kernels, so a
solve from either handle must give the same bits: status, iterations,
restarts, KKT terms, the solution and the multipliers.  Two set-ups in a row
on the one fixed array, the second with a smaller LP, check that nothing of
the first LP's contents leaks into the second.  Also: the size limit, one
live handle per device, and no device memory taken by the call.
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


def _run(pd, lp, noalloc, **kw):
    s = pd.Solver(lp, noalloc=noalloc, **kw)
    r = s.solve()
    sols = [s.solution(inst=i, lam=True) for i in range(s.batch)]
    it = s.info()
    s.close()
    return r, sols, it


def _same(a, b):
    (ra, sa, ia), (rb, sb, ib) = a, b
    for x, y in zip(ra, rb):
        x, y = dict(x), dict(y)
        x.pop("seconds"), y.pop("seconds")
        assert x == y
    for (xa, ya, la), (xb, yb, lb) in zip(sa, sb):
        np.testing.assert_array_equal(xa, xb)
        np.testing.assert_array_equal(ya, yb)
        np.testing.assert_array_equal(la, lb)
    assert (ia["knorm"], ia["omega"], ia["nblk_primal"], ia["nblk_dual"]) == \
           (ib["knorm"], ib["omega"], ib["nblk_primal"], ib["nblk_dual"])


def test_noalloc_with_column_slices(pd):
    """Both sweeps (and the check) in column slices: the slice starts and the
    partial products live in the fixed array too, and the solve matches the
    allocating set-up bit for bit, adaptive steps included."""
    lp = lpgen.config2(7, m=3000, n=6000, kmax=2000)
    for extra in ({}, dict(adaptive_step=1)):
        kw = dict(precision="f32", eps=1e-5, col_slices=4, col_slices_t=2, max_iters=100000, **extra)
        _same(_run(pd, lp, False, **kw), _run(pd, lp, True, **kw))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_equals_setup_twice_shrinking(pd, prec):
    big = lpgen.planted(400, 1000, 0.02, 31, ge_frac=0.4)
    small = lpgen.planted(90, 200, 0.05, 32, ge_frac=0.6)
    kw = dict(precision=prec, eps=1e-6 if prec == "f64" else 1e-5, trace_capacity=64)
    for lp in (big, small):
        ref = _run(pd, lp, False, **kw)
        got = _run(pd, lp, True, **kw)
        assert got[0][0]["status_name"] == "OPTIMAL"
        _same(got, ref)


def test_noalloc_batch_and_adaptive(pd):
    lps = [lpgen.planted(m, int(2.5 * m), 0.03, 40 + i, ge_frac=0.3) for i, m in enumerate([60, 150, 100])]
    kw = dict(precision="f32", eps=1e-5, adaptive_step=1, batch_resident_bytes=0)
    _same(_run(pd, lps, True, **kw), _run(pd, lps, False, **kw))
    # then a smaller batch on the same array
    _same(_run(pd, lps[:2], True, **kw), _run(pd, lps[:2], False, **kw))


def test_noalloc_one_live_handle_per_device(pd):
    lp = lpgen.planted(50, 120, 0.05, 3)
    a = pd.Solver(lp, precision="f64", noalloc=True)
    with pytest.raises(pd.PDHGError) as e:
        pd.Solver(lp, precision="f64", noalloc=True)
    assert e.value.code == -7 and "still live" in str(e.value)
    a.close()
    b = pd.Solver(lp, precision="f64", noalloc=True)  # the array is free again
    assert b.solve()[0]["status"] == 0
    b.close()


def test_noalloc_rejects_lp_beyond_the_fixed_size(pd):
    # about 4M nonzeros: K and K^T in FP64 and FP32 need ~130 MB > 64 MiB
    lp = lpgen.planted(20000, 50000, 0.004, 5)
    with pytest.raises(pd.PDHGError) as e:
        pd.Solver(lp, precision="f32", noalloc=True)
    assert e.value.code == -5 and "fixed workspace" in str(e.value)
    # the refused call left the array free
    s = pd.Solver(lpgen.planted(40, 100, 0.05, 6), precision="f64", noalloc=True)
    s.close()


def test_noalloc_takes_no_device_memory(pd):
    import torch

    lp = lpgen.planted(200, 500, 0.02, 9)
    s = pd.Solver(lp, precision="f32", noalloc=True)  # the library's code object is loaded now
    s.close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    s = pd.Solver(lp, precision="f32", noalloc=True)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    s.close()
    assert free0 - free1 <= 2 << 20, (free0, free1)

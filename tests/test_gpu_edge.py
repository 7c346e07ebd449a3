"""Degenerate and extreme shapes on the GPU, against the oracle and closed
forms: no constraint rows, empty rows and columns, duplicate entries, all-zero
data, a 1 x 1 LP, and a single row with 100,000 entries (whole-workgroup rows
in K, one-entry rows in K^T)."""
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


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_no_rows_closed_form(orc, pd, prec):
    """m = 0: the minimiser sits at l_j where c_j > 0 and at u_j where c_j < 0."""
    c = np.array([1.0, -2.0, 0.0, 3.0, -1.0])
    l = np.array([0.0, 0.0, 0.0, -1.0, -2.0])
    u = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    lp = lpgen.from_dense(np.zeros((0, 5)), [], [], c, l, u)
    s = pd.Solver(lp, precision=prec, eps=1e-8)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    assert y.shape == (0,)
    np.testing.assert_allclose(x[[0, 1, 3, 4]], [0.0, 2.0, -1.0, 5.0], atol=1e-6)
    assert 0.0 <= x[2] <= 3.0
    ro = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-8))
    assert r["kkt"]["pobj"] == pytest.approx(ro.kkt["pobj"], abs=1e-6)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_empty_rows_and_columns(orc, pd, prec):
    """An empty "=" row with b = 0, an empty ">=" row with h = -1 (both always
    satisfied) and an empty column (x_j at the bound its cost prefers)."""
    K = np.array([[1.0, 1.0, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 0.0],
                  [0.0, 1.0, 0.0, 2.0],
                  [0.0, 0.0, 0.0, 0.0]])
    lp = lpgen.from_dense(K, [1, 1, 0, 0], [1.0, 0.0, 1.0, -1.0], [1.0, 2.0, -1.0, 1.0], [0, 0, 0, 0],
                          [2.0, 2.0, 3.0, 2.0])
    s = pd.Solver(lp, precision=prec, eps=1e-7)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    o = orc.Oracle(lp)
    ro = o.solve(orc.SolveOpts(eps=1e-9))
    assert x[2] == pytest.approx(3.0, abs=1e-5)  # empty column with c < 0 goes to u
    assert o.kkt(x, y)["rel_kkt"] <= 1e-5
    assert r["kkt"]["pobj"] == pytest.approx(ro.kkt["pobj"], rel=1e-5, abs=1e-6)


def test_duplicate_entries_are_summed(orc, pd):
    """A row listing the same column twice is the LP with the entries added:
    both paths reach that LP's optimum, and they agree on the Ruiz factors of
    the duplicated form bitwise."""
    base = lpgen.planted(30, 70, 0.1, 4, ge_frac=0.4)
    # split every entry of row 0 into two halves (same column twice)
    rp, col, val = base.rowptr, base.col, base.val
    b0, e0 = rp[0], rp[1]
    col2 = np.concatenate([col[b0:e0], col[b0:e0], col[e0:]])
    val2 = np.concatenate([0.5 * val[b0:e0], 0.5 * val[b0:e0], val[e0:]])
    rp2 = rp.copy()
    rp2[1:] += e0 - b0
    dup = lpgen.LP(**{**base.__dict__})
    dup.rowptr, dup.col, dup.val = rp2, col2.astype(np.int32), val2
    s = pd.Solver(dup, precision="f64", eps=1e-8)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL"
    x, y = s.solution()
    assert orc.Oracle(base).kkt(x, y)["rel_kkt"] <= 1e-7
    assert r["kkt"]["pobj"] == pytest.approx(base.f_star, rel=1e-6)
    rho, kap = s.scaling()
    rho_o, kap_o = orc.Oracle(dup).ruiz(10)
    np.testing.assert_array_equal(rho, rho_o)
    np.testing.assert_array_equal(kap, kap_o)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_all_zero_data_stops_at_start(pd, prec):
    """c = 0 and q = 0 with 0 inside the bounds: the start (0, 0) is optimal
    and the primal weight falls back to 1 (both norms below eps_zero)."""
    K = np.array([[1.0, -1.0, 0.0], [0.0, 2.0, 1.0]])
    lp = lpgen.from_dense(K, [1, 0], [0.0, 0.0], [0.0, 0.0, 0.0], [-1.0, -1.0, -1.0], [1.0, 1.0, 1.0])
    s = pd.Solver(lp, precision=prec, eps=1e-8)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL" and r["iters"] == 0, r
    assert r["omega0"] == 1.0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_by_one_lp(pd, prec):
    """min x s.t. 2x >= 3, x in [0, 10]: x* = 1.5, y* = 0.5."""
    lp = lpgen.from_dense(np.array([[2.0]]), [0], [3.0], [1.0], [0.0], [10.0])
    # FP32 iterates settle within a few units of 2^-24 of the optimum
    s = pd.Solver(lp, precision=prec, eps=1e-8 if prec == "f64" else 1e-6)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    tol = 1e-6 if prec == "f64" else 1e-5
    assert x[0] == pytest.approx(1.5, abs=tol) and y[0] == pytest.approx(0.5, abs=tol)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_long_row(orc, pd, prec):
    """min c'x s.t. sum_j x_j >= 1, 0 <= x <= 1 with n = 100,000: the whole
    demand goes to the cheapest variable.  K has one row of 100k entries (a
    whole-workgroup row), K^T 100k one-entry rows."""
    n = 100_000
    rng = np.random.default_rng(3)
    c = rng.uniform(1.0, 2.0, n)
    jmin = int(np.argmin(c))
    rowptr = np.array([0, n], dtype=np.int64)
    lp = lpgen.LP(n, 1, rowptr, np.arange(n, dtype=np.int32), np.ones(n), np.array([0], dtype=np.uint8),
                  np.array([1.0]), c, np.zeros(n), np.ones(n), name="star")
    eps = 1e-6 if prec == "f64" else 1e-4  # FP32: the sums run over 100k iterates
    s = pd.Solver(lp, precision=prec, eps=eps, max_iters=500_000)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    assert orc.Oracle(lp).kkt(x, y)["rel_kkt"] <= 1.01 * eps
    assert r["kkt"]["pobj"] == pytest.approx(c[jmin], rel=10 * eps)
    assert y[0] == pytest.approx(c[jmin], rel=1e-3)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_of_degenerate_shapes_equals_solo(pd, prec):
    """A batch mixing an LP with no rows, a 1 x 1 LP, an LP whose rows are all
    empty, one with an empty column and ordinary ones: the threaded setup
    writes each instance's part of the shared images, and every instance
    still gets bitwise its solo result."""
    c = np.array([1.0, -2.0, 0.0, 3.0, -1.0])
    lps = [
        lpgen.from_dense(np.zeros((0, 5)), [], [], c, np.zeros(5), np.full(5, 2.0)),
        lpgen.from_dense(np.array([[2.0]]), [0], [3.0], [1.0], [0.0], [10.0]),
        lpgen.from_dense(np.zeros((3, 4)), [1, 0, 1], [0.0, -1.0, 0.0], [1.0, -1.0, 0.5, 0.0], np.zeros(4),
                         np.full(4, 3.0)),
        lpgen.from_dense(np.array([[1.0, 1.0, 0.0], [0.0, 1.0, 0.0]]), [1, 0], [1.0, 0.5], [1.0, 2.0, -1.0],
                         np.zeros(3), np.full(3, 4.0)),
        lpgen.planted(50, 120, 0.05, 3, ge_frac=0.5),
        lpgen.tiny(7, n=6, m=3, free_frac=0.3),
    ]
    kw = dict(precision=prec, eps=1e-6, max_iters=200000)
    for budget in (0, None):
        b = pd.Solver(lps, **kw) if budget is None else pd.Solver(lps, batch_resident_bytes=budget, **kw)
        rb = b.solve()
        for i, lp in enumerate(lps):
            s = pd.Solver(lp, **kw)
            rs = s.solve()[0]
            assert rb[i]["status"] == rs["status"] and rb[i]["iters"] == rs["iters"], (i, rb[i], rs)
            xb, yb = b.solution(inst=i)
            xs, ys = s.solution()
            np.testing.assert_array_equal(xb, xs)
            np.testing.assert_array_equal(yb, ys)

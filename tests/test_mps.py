"""MPS reader and writer (host only).

Each fixture under tests/golden/mps is a small model written for these tests;
its meaning is restated here by hand, row by row, and solved independently
with HiGHS (scipy.optimize.linprog) in the file's own form (<=, >=, ranges,
maximisation).  The reader's arrays must equal the hand-made solver form, and
the FP64 oracle's solve of the parsed model must reach HiGHS' objective."""
import math
import os

import numpy as np
import pytest

import lpgen
from paper_2508_16806_amd import mps

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "mps")
INF = math.inf


def _dense(model):
    K = np.zeros((model.m, model.n))
    for i in range(model.m):
        for k in range(model.rowptr[i], model.rowptr[i + 1]):
            K[i, model.col[k]] += model.val[k]
    return K


def _highs(c, A_ub=None, b_ub=None, A_eq=None, b_eq=None, bounds=None, maximize=False, const=0.0):
    from scipy.optimize import linprog

    cc = -np.asarray(c, float) if maximize else np.asarray(c, float)
    r = linprog(cc, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq, bounds=bounds, method="highs")
    assert r.status == 0, r.message
    v = r.fun
    return (-v if maximize else v) + const


def _oracle_objective(orc, model):
    o = orc.Oracle(model)
    r = o.solve(orc.SolveOpts(eps=1e-9, max_iters=2_000_000))
    assert r.status == 0
    return model.objective(r.x), r


# ---------------------------------------------------------------------------
# small.mps:  min x1 + 2 x2 - x3
#   LIM1: x1 + x2 <= 4      LIM2: x1 >= 1      MYEQN: -x2 + x3 = 7
#   0 <= x1 <= 4, -1 <= x2 <= 1, 0 <= x3 <= 10
# ---------------------------------------------------------------------------
def test_small_arrays():
    m = mps.read_mps(os.path.join(GOLD, "small.mps"))
    assert m.name == "SMALL" and m.col_names == ["X1", "X2", "X3"] and m.row_names == ["LIM1", "LIM2", "MYEQN"]
    np.testing.assert_array_equal(_dense(m), [[-1, -1, 0], [1, 0, 0], [0, -1, 1]])
    np.testing.assert_array_equal(m.row_type, [lpgen.GE, lpgen.GE, lpgen.EQ])
    np.testing.assert_array_equal(m.rhs, [-4, 1, 7])
    np.testing.assert_array_equal(m.c, [1, 2, -1])
    np.testing.assert_array_equal(m.l, [0, -1, 0])
    np.testing.assert_array_equal(m.u, [4, 1, 10])
    assert m.row_origin == [(0, -1), (1, 1), (2, 1)] and m.obj_offset == 0.0 and not m.maximize


def test_small_objective(orc):
    m = mps.read_mps(os.path.join(GOLD, "small.mps"))
    ref = _highs([1, 2, -1], A_ub=[[1, 1, 0], [-1, 0, 0]], b_ub=[4, -1], A_eq=[[0, -1, 1]], b_eq=[7],
                 bounds=[(0, 4), (-1, 1), (0, 10)])
    got, r = _oracle_objective(orc, m)
    assert got == pytest.approx(ref, abs=1e-6)
    # the multiplier of LIM2 (x1 >= 1 binds) in the file's convention is d obj / d rhs = +1
    duals = m.row_duals(r.y)
    assert duals[1] == pytest.approx(1.0, abs=1e-5)


# ---------------------------------------------------------------------------
# ranges_max.mps:  max 3 x1 + 2 x2 - x3 + x4 + 10
#   1 <= x1 + x2 <= 6         (G, range 5)
#   5 <= x1 + 2 x3 <= 8       (L, range -3)
#   2 <= x2 + x4 <= 6         (E, range +4)
#   -1.5 <= x3 - x4 <= 0.5    (E, range -2)
#   0 <= x1 <= 4, x2 <= 3, 1 <= x3 <= 5, x4 free
# ---------------------------------------------------------------------------
def test_ranges_max_arrays():
    m = mps.read_mps(os.path.join(GOLD, "ranges_max.mps"))
    assert m.maximize and m.obj_offset == -10.0
    np.testing.assert_array_equal(m.c, [-3, -2, 1, -1])
    K = _dense(m)
    np.testing.assert_array_equal(K, [[1, 1, 0, 0], [-1, -1, 0, 0], [1, 0, 2, 0], [-1, 0, -2, 0],
                                      [0, 1, 0, 1], [0, -1, 0, -1], [0, 0, 1, -1], [0, 0, -1, 1]])
    np.testing.assert_array_equal(m.rhs, [1, -6, 5, -8, 2, -6, -1.5, -0.5])
    assert np.all(m.row_type == lpgen.GE)
    np.testing.assert_array_equal(m.l, [0, -INF, 1, -INF])
    np.testing.assert_array_equal(m.u, [4, 3, 5, INF])
    assert m.row_origin == [(0, 1), (0, -1), (1, 1), (1, -1), (2, 1), (2, -1), (3, 1), (3, -1)]


def test_ranges_max_objective(orc):
    m = mps.read_mps(os.path.join(GOLD, "ranges_max.mps"))
    A = [[1, 1, 0, 0], [1, 0, 2, 0], [0, 1, 0, 1], [0, 0, 1, -1]]
    lo, hi = [1, 5, 2, -1.5], [6, 8, 6, 0.5]
    A_ub = np.vstack([A, -np.asarray(A)])
    b_ub = np.concatenate([hi, -np.asarray(lo)])
    ref = _highs([3, 2, -1, 1], A_ub=A_ub, b_ub=b_ub, bounds=[(0, 4), (None, 3), (1, 5), (None, None)],
                 maximize=True, const=10.0)
    got, _ = _oracle_objective(orc, m)
    assert got == pytest.approx(ref, abs=1e-6)


# ---------------------------------------------------------------------------
# bounds.mps:  min A - B + 2 C + 0.5 D - 2 E
#   C1: A + B - D >= -2       C2: B + C + E <= 10
#   A = 1.5, B <= -1 (l = -inf), C >= 0, E in [0, 1], D in [0.25, 2]
#   optimum 0.625 at (1.5, -1, 0, 0.25, 1)
# ---------------------------------------------------------------------------
def test_bounds_arrays_and_objective(orc):
    m = mps.read_mps(os.path.join(GOLD, "bounds.mps"))
    assert m.obj_name == "OBJ"
    np.testing.assert_array_equal(m.c, [1, -1, 2, 0.5, -2])  # the second N row is ignored
    np.testing.assert_array_equal(_dense(m), [[1, 1, 0, -1, 0], [0, -1, -1, 0, -1]])
    np.testing.assert_array_equal(m.rhs, [-2, -10])
    np.testing.assert_array_equal(m.l, [1.5, -INF, 0, 0.25, 0])
    np.testing.assert_array_equal(m.u, [1.5, -1, INF, 2, 1])
    ref = _highs([1, -1, 2, 0.5, -2], A_ub=[[-1, -1, 0, 1, 0], [0, 1, 1, 0, 1]], b_ub=[2, 10],
                 bounds=[(1.5, 1.5), (None, -1), (0, None), (0.25, 2), (0, 1)])
    assert ref == pytest.approx(0.625, abs=1e-9)
    got, _ = _oracle_objective(orc, m)
    assert got == pytest.approx(0.625, abs=1e-6)


@pytest.mark.parametrize("which", ["c0", "mixed", "free", "sced_small"])
@pytest.mark.parametrize("gz", [False, True])
def test_write_read_roundtrip_exact(tmp_path, which, gz):
    lp = {"c0": lambda: lpgen.config0(0), "mixed": lambda: lpgen.planted(60, 150, 0.05, 3, ge_frac=0.5),
          "free": lambda: lpgen.tiny(3, n=8, m=4, free_frac=0.5),
          "sced_small": lambda: lpgen.sced(20, 8, 4, 6, seed=9)}[which]()
    path = tmp_path / ("lp.mps.gz" if gz else "lp.mps")
    mps.write_mps(lp, path)
    m = mps.read_mps(path)
    assert (m.n, m.m) == (lp.n, lp.m)
    np.testing.assert_array_equal(m.row_type, lp.row_type)
    np.testing.assert_array_equal(m.rhs, lp.rhs)
    np.testing.assert_array_equal(m.c, lp.c)
    np.testing.assert_array_equal(m.l, lp.l)
    np.testing.assert_array_equal(m.u, lp.u)
    # same matrix (entries may come back in column order within a row)
    import scipy.sparse as sp

    A = sp.csr_matrix((lp.val, lp.col, lp.rowptr), shape=(lp.m, lp.n))
    B = sp.csr_matrix((m.val, m.col, m.rowptr), shape=(m.m, m.n))
    assert (A != B).nnz == 0


@pytest.mark.parametrize("text,msg", [
    ("ROWS\n N OBJ\n G R1\nCOLUMNS\n X OBJ 1 R9 2\nENDATA\n", "unknown row"),
    ("ROWS\n N OBJ\n Q R1\nENDATA\n", "bad row type"),
    ("ROWS\n N OBJ\n G R1\nCOLUMNS\n X OBJ one\nENDATA\n", "bad number"),
    ("FOO\n", "unknown section"),
    ("ROWS\n N OBJ\n G R1\nCOLUMNS\n X R1 1\nBOUNDS\n UP BND Y 1\nENDATA\n", "unknown column"),
    ("ROWS\n N OBJ\n G R1\nCOLUMNS\n X R1 1\nBOUNDS\n SC BND X 1\nENDATA\n", "unsupported bound"),
    ("ROWS\n N OBJ\nENDATA\n", "no columns"),
])
def test_rejects_malformed(text, msg):
    with pytest.raises(ValueError) as e:
        mps.parse_mps(text)
    assert msg in str(e.value)

"""Models read from MPS files solved on the GPU: the objective in the file's
own sense (maximisation, constant) against HiGHS on the file's own form, and
the row multipliers mapped back to the file's rows."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "mps")

# HiGHS objectives of the fixtures, as computed in tests/test_mps.py
REF = {"small.mps": None, "ranges_max.mps": None, "bounds.mps": 0.625}


@pytest.fixture(scope="module")
def pd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16806_amd as pd

    pd.lib()
    return pd


def _ref(name):
    import test_mps as t

    if name == "small.mps":
        return t._highs([1, 2, -1], A_ub=[[1, 1, 0], [-1, 0, 0]], b_ub=[4, -1], A_eq=[[0, -1, 1]], b_eq=[7],
                        bounds=[(0, 4), (-1, 1), (0, 10)])
    if name == "ranges_max.mps":
        A = [[1, 1, 0, 0], [1, 0, 2, 0], [0, 1, 0, 1], [0, 0, 1, -1]]
        lo, hi = [1, 5, 2, -1.5], [6, 8, 6, 0.5]
        return t._highs([3, 2, -1, 1], A_ub=np.vstack([A, -np.asarray(A)]), b_ub=np.concatenate([hi, -np.asarray(lo)]),
                        bounds=[(0, 4), (None, 3), (1, 5), (None, None)], maximize=True, const=10.0)
    return REF[name]


@pytest.mark.parametrize("name", ["small.mps", "ranges_max.mps", "bounds.mps"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mps_models_solve(pd, name, prec):
    m = pd.read_mps(os.path.join(GOLD, name))
    s = pd.Solver(m, precision=prec, eps=1e-8 if prec == "f64" else 1e-6, max_iters=2_000_000)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    tol = 1e-6 if prec == "f64" else 1e-4
    assert m.objective(x) == pytest.approx(_ref(name), abs=tol * (1 + abs(_ref(name))))
    if name == "small.mps":
        assert m.row_duals(y)[1] == pytest.approx(1.0, abs=1e-3)

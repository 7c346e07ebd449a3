"""One GPU's share of a row / column partition of the Zipf LP: the rows of K
(all columns, n >> m) and the rows of K^T (all rows of K, many of them empty
in the block), each solved as an LP in its own right.  FP64 fixed steps
against the oracle, element by element, as for the whole LP."""
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


@pytest.fixture(scope="module")
def base():
    return lpgen.config2(9, m=16000, n=32000, kmax=3000)


# lay: whole rows, or both sweeps in column slices (rows of >= 16 S entries)
@pytest.mark.parametrize("lay", [{}, dict(col_slices=4, col_slices_t=2)], ids=["whole", "sliced"])
@pytest.mark.parametrize("kind,p", [("rows", 0), ("rows", 7), ("cols", 0), ("cols", 5)])
def test_shard_fixed_steps_f64(orc, pd, base, kind, p, lay):
    P = 8
    if kind == "rows":
        lp = lpgen.row_block(base, p * base.m // P, (p + 1) * base.m // P)
    else:
        lp = lpgen.col_block(base, p * base.n // P, (p + 1) * base.n // P)
        assert np.count_nonzero(np.diff(lp.rowptr) == 0) > 0  # empty rows are part of the case
    o = orc.Oracle(lp)
    rho, kap = o.ruiz(10)
    s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=1.0, primal_weight=1.0)
    eta, omega = 0.9 / s.info()["knorm"], 1.7
    s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=eta, primal_weight=omega, **lay)
    x0s = np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap)
    y0s = np.zeros(lp.m)
    done = 0
    for k in (1, 15):
        s.iterate(k)
        done += k
        xs, ys = o.steps(x0s, y0s, eta / omega, eta * omega, done, ruiz_iters=10)
        x, y = s.solution(which=pd.SOL_CURRENT)
        xo, yo = np.clip(kap * xs, lp.l, lp.u), rho * ys
        tol = 1e-12 if k == 1 else 1e-10
        np.testing.assert_allclose(x, xo, rtol=tol, atol=tol * (1 + np.abs(xo).max()))
        np.testing.assert_allclose(y, yo, rtol=tol, atol=tol * (1 + np.abs(yo).max()))


def test_shard_tuned_layout_sets_up_and_steps(pd, base):
    """The tuned layout of the full Zipf LP sets up and steps on both block
    shapes (the launch configuration the benchmark's partition leg times)."""
    import os

    from paper_2508_16806_amd import tuner

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    tune = tuner.load(os.path.join(root, "paper_2508_16806_amd", "tuning", "zipf_c2_f32.json"))
    for sub in (lpgen.row_block(base, 0, base.m // 8), lpgen.col_block(base, 0, base.n // 8)):
        s = pd.Solver(sub, precision="f32", **tune)
        k = s.time_kernels(reps=2)
        assert k["ms_primal"] > 0 and k["ms_dual"] > 0
        s.iterate(64)
        x, y = s.solution(which=pd.SOL_CURRENT)
        assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
        assert np.all(x >= sub.l - 1e-9) and np.all(x <= sub.u + 1e-9)

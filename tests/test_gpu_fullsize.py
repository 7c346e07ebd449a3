"""Parity at the benchmark's full size and launch configuration.

C1 (SCED-shaped, n = 418,048, m = 298,072, nnz = 15.25M) with the tuned bins
bench.py uses: every element of one FP32 step against the FP64 oracle (derived
FP32 bound), the Ruiz factors bitwise, and the oracle's relative KKT of the
GPU's 1e-4 solve.  C2's Zipf row-length structure is exercised at 1/10 scale
(m = 100k, n = 200k) with a planted optimum.
"""
import os

import numpy as np
import pytest

import lpgen
from test_gpu_parity import fp32_step_bounds

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_16806_amd as pd

    pd.lib()
    return pd


@pytest.fixture(scope="module")
def c1():
    return lpgen.config1()


@pytest.fixture(scope="module")
def tune():
    from paper_2508_16806_amd import tuner

    return tuner.load(os.path.join(ROOT, "paper_2508_16806_amd", "tuning", "sced_c1_f32.json"))


def test_c1_ruiz_bitwise(orc, pd, c1, tune):
    s = pd.Solver(c1, precision="f32", **tune)
    rho, kap = s.scaling()
    rho_o, kap_o = orc.Oracle(c1).ruiz(10)
    np.testing.assert_array_equal(rho, rho_o)
    np.testing.assert_array_equal(kap, kap_o)


def test_c1_one_step_every_element(orc, pd, c1, tune):
    lp = c1
    o = orc.Oracle(lp)
    rho, kap = o.ruiz(10)
    eta = 0.01
    s = pd.Solver(lp, precision="f32", step_size=eta, primal_weight=1.0, **tune)
    rng = np.random.default_rng(7)
    lo, hi = lp.l / kap, lp.u / kap
    xs = np.clip(rng.uniform(-1, 1, lp.n) * np.minimum(np.abs(hi), 10), lo, hi)
    xs = xs.astype(np.float32).astype(np.float64)
    xs = np.clip(xs, lo.astype(np.float32).astype(np.float64), hi.astype(np.float32).astype(np.float64))
    ys = rng.standard_normal(lp.m).astype(np.float32).astype(np.float64)
    ys[lp.row_type == 0] = np.abs(ys[lp.row_type == 0])
    s.set_state(kap * xs, rho * ys)
    x0, y0 = s.solution(which=pd.SOL_CURRENT)
    xs, ys = x0 / kap, y0 / rho  # what the GPU actually holds (FP32)
    s.iterate(1)
    x, y = s.solution(which=pd.SOL_CURRENT)
    xo, yo = o.steps(xs, ys, eta, eta, 1, ruiz_iters=10)
    Ks = abs(lp.scipy().multiply(rho[:, None]).multiply(kap[None, :])).tocsr()
    # the bound derived in test_gpu_parity.fp32_step_bounds
    bx, by = fp32_step_bounds(Ks, kap * lp.c, rho * lp.rhs, xs, ys, xo, yo, eta, eta)
    ex = np.abs(x / kap - xo) / bx
    ey = np.abs(y / rho - yo) / by
    assert ex.max() <= 1.0, (ex.max(), int(ex.argmax()))
    assert ey.max() <= 1.0, (ey.max(), int(ey.argmax()))


def test_c1_solve_1e4_oracle_kkt(orc, pd, c1, tune):
    s = pd.Solver(c1, precision="f32", eps=1e-4, **tune)
    r = s.solve()[0]
    assert r["status_name"] == "OPTIMAL", r
    x, y = s.solution()
    chk = orc.Oracle(c1).kkt(x, y)
    assert chk["rel_kkt"] <= 1e-4, chk
    # the GPU's own FP64 re-check of the returned point agrees with the oracle
    assert s.kkt(x, y)["rel_kkt"] == pytest.approx(chk["rel_kkt"], rel=1e-6)


def test_c2_tenth_scale(orc, pd):
    lp = lpgen.config2(2, m=100_000, n=200_000)
    s = pd.Solver(lp, precision="f32", eps=1e-5, max_iters=300000)
    r = s.solve()[0]
    x, y = s.solution()
    chk = orc.Oracle(lp).kkt(x, y)
    gap = abs(chk["pobj"] - lp.f_star) / (1 + abs(lp.f_star))
    print("C2/10", r["status_name"], r["iters"], r["restarts"], chk["rel_kkt"], gap)
    assert chk["rel_kkt"] <= 1e-4
    assert gap <= 1e-5


def test_c2_tenth_sliced_steps_f64(orc, pd):
    """C2 at 1/10 scale (100k x 200k, Zipf(1.5) rows) with the dual sweep in 4
    column slices and the primal sweep in 2: FP64 fixed steps against the
    oracle, element by element, after 1 step (1e-12) and 50 (1e-9)."""
    lp = lpgen.config2(2, m=100_000, n=200_000)
    o = orc.Oracle(lp)
    rho, kap = o.ruiz(10)
    lay = dict(col_slices=4, col_slices_t=2)
    s = pd.Solver(lp, precision="f64", step_size=1.0, primal_weight=1.0, **lay)
    eta, omega = 0.9 / s.info()["knorm"], 1.3
    s.close()
    s = pd.Solver(lp, precision="f64", step_size=eta, primal_weight=omega, **lay)
    x0 = np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap)
    done = 0
    for k, tol in ((1, 1e-12), (49, 1e-9)):
        s.iterate(k)
        done += k
        xs, ys = o.steps(x0, np.zeros(lp.m), eta / omega, eta * omega, done, ruiz_iters=10)
        x, y = s.solution(which=pd.SOL_CURRENT)
        xo, yo = np.clip(kap * xs, lp.l, lp.u), rho * ys
        np.testing.assert_allclose(x, xo, rtol=tol, atol=tol * (1 + np.abs(xo).max()))
        np.testing.assert_allclose(y, yo, rtol=tol, atol=tol * (1 + np.abs(yo).max()))


def test_c2_full_solve_1e4_oracle_kkt(orc, pd):
    """C2 at its configured size (m = 1M rows, n = 2M, Zipf(1.5) row lengths,
    ~54M nonzeros), FP32 with its tuned layout: a cold-start solve to the
    paper's 1e-4, with the oracle's KKT error of the returned point at most
    1e-4 and the objective gap to the planted optimum reported (reading 18:
    a 1e-4 KKT error does not bound it to 1e-5)."""
    from paper_2508_16806_amd import tuner

    lp = lpgen.config2()
    tune = tuner.load(os.path.join(ROOT, "paper_2508_16806_amd", "tuning", "zipf_c2_f32.json"))
    s = pd.Solver(lp, precision="f32", eps=1e-4, max_iters=200_000, time_limit=150.0, **tune)
    r = s.solve()[0]
    x, y = s.solution()
    s.close()
    chk = orc.Oracle(lp).kkt(x, y)
    gap = abs(chk["pobj"] - lp.f_star) / (1 + abs(lp.f_star))
    print(f"[c2-full] {r['status_name']} iters {r['iters']} restarts {r['restarts']} seconds {r['seconds']:.1f} "
          f"oracle rel_kkt {chk['rel_kkt']:.3e} gap to planted {gap:.3e}", flush=True)
    assert r["status_name"] == "OPTIMAL", r
    assert chk["rel_kkt"] <= 1e-4 * 1.01, chk

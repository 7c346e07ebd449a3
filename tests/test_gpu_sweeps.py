"""Wide sweeps over seeded structures (each a single test that lists every
failing case): 200 random structures (FP64 steps and KKT against the oracle,
FP64 solves to 1e-7 at the planted objective, FP32 solves at 1e-4; FP32 with
adaptive steps and detection; FP64 with each), 240 infeasible or unbounded
solves with detection, 120 fishnet casts followed by solves, and 40 adjoints
against the oracle's reverse mode."""
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


def _gap(lp, p):
    return abs(p - lp.f_star) / (1 + abs(lp.f_star))


def test_sweep_random_structures(orc, pd):
    fails = []
    for seed in range(32, 232):
        lp = lpgen.random_case(seed)
        o = orc.Oracle(lp)
        s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=1.0, primal_weight=1.0)
        eta, omega = 0.9 / s.info()["knorm"], 0.8
        s = pd.Solver(lp, precision="f64", ruiz_iters=10, step_size=eta, primal_weight=omega)
        rho, kap = o.ruiz(10)
        s.iterate(20)
        xs, ys = o.steps(np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap), np.zeros(lp.m), eta / omega,
                         eta * omega, 20, ruiz_iters=10)
        x, y = s.solution(which=pd.SOL_CURRENT)
        xo, yo = np.clip(kap * xs, lp.l, lp.u), rho * ys
        if np.abs(x - xo).max() > 1e-9 * (1 + np.abs(xo).max()) or \
                (lp.m and np.abs(y - yo).max() > 1e-9 * (1 + np.abs(yo).max())):
            fails.append((seed, "steps"))
        for prec, eps, opt in (("f64", 1e-7, {}), ("f32", 1e-4, {}),
                               ("f32", 1e-4, dict(adaptive_step=1, detect_infeas=1)),
                               ("f64", 1e-7, dict(detect_infeas=1)), ("f64", 1e-7, dict(adaptive_step=1))):
            r = pd.Solver(lp, precision=prec, eps=eps, max_iters=400000, **opt)
            rr = r.solve()[0]
            k = o.kkt(*r.solution())
            bad = rr["status_name"] != "OPTIMAL" or k["rel_kkt"] > 1.05 * eps
            if prec == "f64" and not opt:
                bad = bad or _gap(lp, k["pobj"]) > 1e-5
            if bad:
                fails.append((seed, lp.name, prec, sorted(opt), rr["status_name"], k["rel_kkt"]))
    assert not fails, fails


def test_sweep_infeasible_and_unbounded(pd):
    fails = []
    for seed in range(40):
        rng = np.random.default_rng(7000 + seed)
        m = int(rng.integers(20, 150))
        n = int(rng.integers(m, 3 * m))
        d = float(rng.uniform(0.03, 0.15))
        for lp, want in ((lpgen.primal_infeasible(m, n, d, seed, kind="bound"), "PRIMAL_INFEASIBLE"),
                         (lpgen.primal_infeasible(m, n, d, seed, kind="pair"), "PRIMAL_INFEASIBLE"),
                         (lpgen.dual_infeasible(m, n, d, seed), "DUAL_INFEASIBLE")):
            for prec in ("f64", "f32"):
                r = pd.Solver(lp, precision=prec, eps=1e-6, detect_infeas=1, max_iters=200000).solve()[0]
                if r["status_name"] != want:
                    fails.append((seed, want, prec, r["status_name"]))
    assert not fails, fails


def test_sweep_fishnet(orc, pd):
    fails = []
    for seed in range(300, 360):
        lp = lpgen.random_case(seed)
        for prec, P, eps in (("f64", 8, 1e-6), ("f32", 32, 1e-4)):
            s = pd.Solver(lp, precision=prec, eps=eps, fishnet_points=P, max_iters=400000)
            s.fishnet(P, 32, seed=seed)
            r = s.solve()[0]
            k = orc.Oracle(lp).kkt(*s.solution())
            bad = r["status_name"] != "OPTIMAL" or k["rel_kkt"] > 1.05 * eps or \
                (prec == "f64" and _gap(lp, k["pobj"]) > 1e-5)
            if bad:
                fails.append((seed, prec, r["status_name"], k["rel_kkt"]))
    assert not fails, fails


def test_sweep_adjoint(orc, pd):
    from test_gpu_adjoint import _setup

    fails = []
    for seed in range(400, 440):
        lp = lpgen.random_case(seed)
        K, C = 40, 12
        o, s, tau, sigma, x0, y0, gx, gy = _setup(pd, orc, lp, "f64", K=K, C=C, seed=seed)
        s.set_state(x0, y0)
        s.iterate(K, record=True)
        g = s.backward(gx, gy)
        go = o.unrolled_vjp(10, tau, sigma, lp.c, lp.rhs, lp.l, lp.u, x0, y0, K, gx, gy)
        for name, key in (("c", "c"), ("rhs", "q"), ("l", "l"), ("u", "u"), ("x0", "x0"), ("y0", "y0")):
            a, b = g[name], go[key]
            if b.size and np.linalg.norm(a - b) > 1e-9 * np.linalg.norm(b) + 1e-12:
                fails.append((seed, name, np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)))
    assert not fails, fails

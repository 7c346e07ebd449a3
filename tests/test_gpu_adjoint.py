"""GPU adjoint of unrolled fixed-step PDHG vs the oracle's reverse mode.

The oracle's reverse mode (orc_unrolled_vjp) is itself pinned by central
finite differences in tests/test_oracle.py.  Both sides compute the Ruiz
factors independently (bitwise equal, see test_gpu_parity) and use the same
explicit step size eta and primal weight omega, so they differentiate the same
map.  FP64 mode differs from the oracle only in summation order (tolerance
1e-9 relative to the gradient's scale); FP32 mode stores the matrix and the
replayed iterates in FP32 (unit roundoff 6e-8) with FP64 adjoint vectors, and
after K = 60 steps of a non-expansive map the gradient agrees to 1e-4
relative in norm unless a clip decision flips, which the test's strictly
interior start avoids.
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


def _setup(pd, orc, lp, prec, K=60, C=16, seed=0):
    o = orc.Oracle(lp)
    kn, _ = o.power_norm(10, max_iters=5000, tol=1e-10)
    eta, omega = 0.8 / kn, 1.7
    s = pd.Solver(lp, precision=prec, step_size=eta, primal_weight=omega, unroll_capacity=K,
                  unroll_checkpoint=C)
    rng = np.random.default_rng(seed)
    l = np.where(np.isfinite(lp.l), lp.l, -5.0)
    u = np.where(np.isfinite(lp.u), lp.u, l + 10.0)
    x0 = l + rng.uniform(0.1, 0.9, lp.n) * (u - l)
    y0 = rng.standard_normal(lp.m) * 0.5
    y0[lp.row_type == 0] = np.abs(y0[lp.row_type == 0]) + 0.05
    gx = rng.standard_normal(lp.n)
    gy = rng.standard_normal(lp.m)
    return o, s, eta / omega, eta * omega, x0, y0, gx, gy


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("K,C", [(60, 16), (32, 32), (7, 50)])
def test_backward_matches_oracle_vjp(orc, pd, prec, K, C):
    lp = lpgen.planted(150, 400, 0.03, 11, ge_frac=0.5)
    o, s, tau, sigma, x0, y0, gx, gy = _setup(pd, orc, lp, prec, K=K, C=C)
    s.set_state(x0, y0)
    s.iterate(K, record=True)
    xk, yk = s.solution(which=pd.SOL_CURRENT)
    xo, yo = o.unrolled(10, tau, sigma, lp.c, lp.rhs, lp.l, lp.u, x0, y0, K)
    g = s.backward(gx, gy)
    go = o.unrolled_vjp(10, tau, sigma, lp.c, lp.rhs, lp.l, lp.u, x0, y0, K, gx, gy)
    if prec == "f64":
        np.testing.assert_allclose(xk, xo, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(yk, yo, rtol=1e-10, atol=1e-10)
        tol = 1e-9
    else:
        tol = 1e-4
    for name, key in (("c", "c"), ("rhs", "q"), ("l", "l"), ("u", "u"), ("x0", "x0"), ("y0", "y0")):
        a, b = g[name], go[key]
        scale = np.linalg.norm(b) + 1e-30
        assert np.linalg.norm(a - b) <= tol * scale + 1e-12, (name, np.linalg.norm(a - b) / scale)
    # the iterate is restored after the backward pass
    x2, y2 = s.solution(which=pd.SOL_CURRENT)
    np.testing.assert_array_equal(x2, xk)
    np.testing.assert_array_equal(y2, yk)


def test_backward_batched_equals_solo(orc, pd):
    lps = [lpgen.planted(80, 200, 0.05, 40 + i, ge_frac=0.4) for i in range(3)]
    K, C = 24, 10
    kw = dict(precision="f64", step_size=0.05, primal_weight=1.0, unroll_capacity=K, unroll_checkpoint=C)
    b = pd.Solver(lps, **kw)
    rng = np.random.default_rng(5)
    gxs = [rng.standard_normal(lp.n) for lp in lps]
    gys = [rng.standard_normal(lp.m) for lp in lps]
    b.iterate(K, record=True)
    gb = b.backward(np.concatenate(gxs), np.concatenate(gys))
    xo = yo = 0
    for i, lp in enumerate(lps):
        s = pd.Solver(lp, **kw)
        s.iterate(K, record=True)
        gs = s.backward(gxs[i], gys[i])
        for k in ("c", "l", "u", "x0"):
            np.testing.assert_array_equal(gb[k][xo:xo + lp.n], gs[k])
        for k in ("rhs", "y0"):
            np.testing.assert_array_equal(gb[k][yo:yo + lp.m], gs[k])
        xo += lp.n
        yo += lp.m


def test_backward_zero_steps_is_identity(pd):
    lp = lpgen.planted(50, 120, 0.05, 3)
    s = pd.Solver(lp, precision="f64", unroll_capacity=10, unroll_checkpoint=4)
    s.iterate(0, record=True)
    gx, gy = np.arange(lp.n, dtype=float), np.arange(lp.m, dtype=float)
    g = s.backward(gx, gy)
    np.testing.assert_allclose(g["x0"], gx)
    np.testing.assert_allclose(g["y0"], gy)
    assert not g["c"].any() and not g["rhs"].any()


def test_backward_without_record_errors(pd):
    lp = lpgen.planted(50, 120, 0.05, 3)
    s = pd.Solver(lp, precision="f64")
    with pytest.raises(pd.PDHGError):
        s.iterate(5, record=True)
    s2 = pd.Solver(lp, precision="f64", unroll_capacity=4)
    with pytest.raises(pd.PDHGError):
        s2.backward(np.zeros(lp.n), np.zeros(lp.m))
    with pytest.raises(pd.PDHGError):
        s2.iterate(5, record=True)


def test_set_data_changes_solution(orc, pd):
    lp = lpgen.planted(120, 300, 0.03, 9, ge_frac=0.3)
    s = pd.Solver(lp, precision="f64", eps=1e-7)
    s.solve()
    lp2 = lpgen.planted(120, 300, 0.03, 9, ge_frac=0.3)
    rng = np.random.default_rng(2)
    lp2.c = lp.c + 0.1 * rng.standard_normal(lp.n)
    s.set_data(c=lp2.c)
    s.set_state(np.zeros(lp.n), np.zeros(lp.m))
    r = s.solve()[0]
    x, y = s.solution()
    chk = orc.Oracle(lp2).kkt(x, y)
    assert r["status"] == 0 and chk["rel_kkt"] <= 1.01e-7
    assert s.kkt(x, y)["rel_kkt"] == pytest.approx(chk["rel_kkt"], rel=1e-6)


def test_autograd_function(orc, pd):
    import torch

    from paper_2508_16806_amd.autograd import PDHGUnroll

    lp = lpgen.planted(100, 250, 0.04, 12, ge_frac=0.5)
    K = 30
    o, s, tau, sigma, x0, y0, gx, gy = _setup(pd, orc, lp, "f64", K=K, C=8, seed=3)
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    c, q, l, u, xs, ys = T(lp.c), T(lp.rhs), T(lp.l), T(lp.u), T(x0), T(y0)
    xk, yk = PDHGUnroll.apply(s, K, c, q, l, u, xs, ys)
    loss = (xk * torch.from_numpy(gx)).sum() + (yk * torch.from_numpy(gy)).sum()
    loss.backward()
    go = o.unrolled_vjp(10, tau, sigma, lp.c, lp.rhs, lp.l, lp.u, x0, y0, K, gx, gy)
    np.testing.assert_allclose(c.grad.numpy(), go["c"], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(q.grad.numpy(), go["q"], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(xs.grad.numpy(), go["x0"], rtol=1e-8, atol=1e-10)


def test_backward_refuses_a_tape_replaced_by_set_data(pd):
    """pdhg_set_data drops the recorded tape: backward raises PDHG_ERR_STATE
    instead of replaying old checkpoints against the new data."""
    lp = lpgen.planted(60, 150, 0.05, 8, ge_frac=0.3)
    s = pd.Solver(lp, precision="f64", unroll_capacity=12, unroll_checkpoint=4)
    g0 = s.info()["record_generation"]
    s.iterate(12, record=True)
    assert s.info()["record_valid"] == 1 and s.info()["record_generation"] == g0 + 1
    s.backward(np.ones(lp.n), np.zeros(lp.m))
    s.set_data(c=lp.c * 1.5)
    assert s.info()["record_valid"] == 0 and s.info()["record_generation"] == g0 + 2
    with pytest.raises(pd.PDHGError) as e:
        s.backward(np.ones(lp.n), np.zeros(lp.m))
    assert e.value.code == -7
    # a new recording restores it
    s.iterate(5, record=True)
    s.backward(np.ones(lp.n), np.zeros(lp.m))


def test_autograd_refuses_a_replaced_tape(orc, pd):
    """Two forward calls on one handle, then the first one's backward: raises
    (the handle keeps only the second tape); the second's backward is right."""
    import torch

    from paper_2508_16806_amd.autograd import PDHGUnroll

    lp = lpgen.planted(80, 200, 0.04, 14, ge_frac=0.5)
    K = 20
    o, s, tau, sigma, x0, y0, gx, gy = _setup(pd, orc, lp, "f64", K=K, C=8, seed=4)
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    c1 = T(lp.c)
    xk1, _ = PDHGUnroll.apply(s, K, c1, T(lp.rhs), T(lp.l), T(lp.u), T(x0), T(y0))
    c2 = T(lp.c * 1.1)
    xk2, _ = PDHGUnroll.apply(s, K, c2, T(lp.rhs), T(lp.l), T(lp.u), T(x0), T(y0))
    with pytest.raises(pd.PDHGError) as e:
        (xk1 * torch.from_numpy(gx)).sum().backward()
    assert e.value.code == -7
    (xk2 * torch.from_numpy(gx)).sum().backward()
    go = o.unrolled_vjp(10, tau, sigma, lp.c * 1.1, lp.rhs, lp.l, lp.u, x0, y0, K, gx, np.zeros(lp.m))
    np.testing.assert_allclose(c2.grad.numpy(), go["c"], rtol=1e-8, atol=1e-10)

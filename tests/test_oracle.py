"""Pins for the FP64 CPU oracle against what the paper and the mathematics fix.

Each test ties one oracle function to something other than itself: a library
routine (scipy.sparse, numpy.linalg, HiGHS through scipy.optimize.linprog),
brute-force vertex enumeration, a planted optimal pair (Section 2.2 duality),
hand-derived fixtures under tests/golden/, or inequalities proved in
Appendix D (boundedness and the ergodic gap bound).
"""
import ctypes
import json
import os

import numpy as np
import pytest

import lpgen
from vertex_enum import vertex_optimum

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return abs(a - b) / (1.0 + abs(b))


# ---------------------------------------------------------------------------
# sparse products
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spmv_matches_scipy(orc, seed):
    lp = lpgen.planted(300, 700, 0.03, seed, ge_frac=0.4)
    o = orc.Oracle(lp)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    A = lp.scipy()
    np.testing.assert_allclose(o.spmv(x), A @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(o.spmv_t(y), A.T @ y, rtol=1e-13, atol=1e-13)


def test_spmv_empty_rows_and_columns(orc):
    K = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 2.0], [0.0, 0.0, 0.0]])
    lp = lpgen.from_dense(K, [1, 0, 1], [0, 1, 0], [1, 1, 1], [0, 0, 0], [1, 1, 1])
    o = orc.Oracle(lp)
    np.testing.assert_array_equal(o.spmv(np.array([1.0, 5.0, 3.0])), [0.0, 7.0, 0.0])
    np.testing.assert_array_equal(o.spmv_t(np.array([1.0, 2.0, 3.0])), [2.0, 0.0, 4.0])


# ---------------------------------------------------------------------------
# KKT error (Section 2.3.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: lpgen.config0(0), lambda: lpgen.config0(1, unique=True),
    lambda: lpgen.planted(400, 900, 0.02, 5, ge_frac=0.5),
    lambda: lpgen.tiny(3, n=8, m=4, free_frac=0.5),
    lambda: lpgen.config2(7, m=2000, n=4000, kmax=300),
])
def test_kkt_zero_at_planted_optimum(orc, maker):
    """The left-hand sides of the termination conditions vanish at an optimum."""
    lp = maker()
    k = orc.Oracle(lp).kkt(lp.x_star, lp.y_star)
    assert k["rel_kkt"] < 1e-12, k
    assert _rel(k["pobj"], lp.f_star) < 1e-12


def test_kkt_handsolved_golden(orc):
    g = json.load(open(os.path.join(GOLD, "lp_handsolved.json")))
    lp = lpgen.from_dense(np.array(g["K"]), g["row_type"], g["rhs"], g["c"], g["l"], g["u"])
    k = orc.Oracle(lp).kkt(np.array(g["x_star"]), np.array(g["y_star"]))
    assert k["rel_kkt"] == 0.0
    assert k["pobj"] == g["f_star"] and k["dobj"] == g["f_star"]


def test_kkt_primal_residual_closed_form(orc):
    """x* + d e_j on an all-equality LP: ||Ax - b|| = |d| ||A[:, j]||."""
    lp = lpgen.config0(2)
    o = orc.Oracle(lp)
    A = lp.dense()
    for j in (3, 77, 401):
        d = 0.37
        x = lp.x_star.copy()
        x[j] += d
        k = o.kkt(x, lp.y_star)
        assert k["pres"] == pytest.approx(abs(d) * np.linalg.norm(A[:, j]), rel=1e-12)
        assert k["dres"] == pytest.approx(0.0, abs=1e-12)
        assert k["pobj"] - lp.f_star == pytest.approx(d * lp.c[j], rel=1e-9, abs=1e-9)


def test_kkt_inequality_residual_is_one_sided(orc):
    """[h - Gx]^+ counts only violated ">=" rows (Section 2.3.2, term2)."""
    K = np.array([[1.0, 1.0]])
    lp = lpgen.from_dense(K, [0], [2.0], [1.0, 1.0], [0, 0], [10, 10])
    o = orc.Oracle(lp)
    assert o.kkt(np.array([3.0, 3.0]), np.array([0.0]))["pres"] == 0.0
    assert o.kkt(np.array([0.5, 0.5]), np.array([0.0]))["pres"] == pytest.approx(1.0)


def test_kkt_dual_residual_cones(orc):
    """lambda = proj_Lambda(c - K'y) with Lambda_i set by which bounds are finite."""
    K = np.zeros((1, 4))
    K[0, 0] = 1.0
    inf = np.inf
    # variables: free, upper-only, lower-only, boxed; c chosen so c - K'y = (2, 3, -5, 7)
    lp = lpgen.from_dense(K, [1], [0.0], [2.0, 3.0, -5.0, 7.0], [-inf, -inf, 0.0, -1.0],
                          [inf, 1.0, inf, 1.0])
    k = orc.Oracle(lp).kkt(np.zeros(4), np.zeros(1))
    # free: lambda=0 -> residual 2; upper-only: lambda=min(3,0)=0 -> 3;
    # lower-only: lambda=max(-5,0)=0 -> 5; boxed: lambda=7 -> 0
    assert k["dres"] == pytest.approx(np.sqrt(4 + 9 + 25))
    # dual objective: boxed var with lambda = 7 > 0 contributes l * 7 = -7 (0*inf never formed)
    assert k["dobj"] == pytest.approx(-7.0)
    assert np.isfinite(k["rel_kkt"])


# ---------------------------------------------------------------------------
# Ruiz scaling (Algorithm 3)
# ---------------------------------------------------------------------------

def test_ruiz_golden_2x2(orc):
    g = json.load(open(os.path.join(GOLD, "ruiz_2x2.json")))
    K = np.array(g["K"])
    lp = lpgen.from_dense(K, [1, 1], [0, 0], [1, 1], [0, 0], [1, 1])
    o = orc.Oracle(lp)
    rho, kap = o.ruiz(1)
    np.testing.assert_array_equal(rho, g["rho_after_1"])
    np.testing.assert_array_equal(kap, g["kappa_after_1"])
    np.testing.assert_array_equal(rho[:, None] * K * kap[None, :], g["K_scaled"])
    rho, kap = o.ruiz(5)
    np.testing.assert_array_equal(rho, g["rho_after_5"])
    np.testing.assert_array_equal(kap, g["kappa_after_5"])


def test_ruiz_equilibrates_inf_norms(orc):
    """Row and column infinity norms of diag(rho) K diag(kappa) tend to 1."""
    lp = lpgen.sced(50, 20, 6, 10, seed=3)
    o = orc.Oracle(lp)
    rho, kap = o.ruiz(40)
    Ks = (lp.scipy().multiply(rho[:, None]).multiply(kap[None, :])).tocsr()
    rn = abs(Ks).max(axis=1).toarray().ravel()
    cn = abs(Ks).max(axis=0).toarray().ravel()
    assert np.max(np.abs(rn - 1)) < 1e-3 and np.max(np.abs(cn - 1)) < 1e-3
    # one pass: every row's scaled inf-norm is sqrt of what it was (column factors <= 1 aside)
    rho1, kap1 = o.ruiz(1)
    A = lp.scipy()
    np.testing.assert_allclose(rho1, 1.0 / np.sqrt(abs(A).max(axis=1).toarray().ravel()))
    np.testing.assert_allclose(kap1, 1.0 / np.sqrt(abs(A).max(axis=0).toarray().ravel()))


def test_ruiz_zero_rows_keep_factor_one(orc):
    K = np.array([[0.0, 0.0], [3.0, 0.0]])
    lp = lpgen.from_dense(K, [1, 1], [0, 1], [1, 1], [0, 0], [1, 1])
    rho, kap = orc.Oracle(lp).ruiz(3)
    assert rho[0] == 1.0 and kap[1] == 1.0


# ---------------------------------------------------------------------------
# power iteration (Algorithm 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 4])
def test_power_norm_matches_svd(orc, seed):
    lp = lpgen.planted(150, 260, 0.05, seed, ge_frac=0.3)
    v, it = orc.Oracle(lp).power_norm(0, max_iters=5000, tol=1e-10)
    assert v == pytest.approx(np.linalg.norm(lp.dense(), 2), rel=1e-6)


def test_power_norm_diagonal_exact(orc):
    K = np.diag([3.0, 1.0, 0.5])
    lp = lpgen.from_dense(K, [1, 1, 1], [0, 0, 0], [1, 1, 1], [0, 0, 0], [1, 1, 1])
    v, it = orc.Oracle(lp).power_norm(0, tol=1e-12)
    assert v == pytest.approx(3.0, rel=1e-10)


def test_power_norm_of_scaled_matrix(orc):
    lp = lpgen.sced(30, 12, 4, 6, seed=2)
    o = orc.Oracle(lp)
    rho, kap = o.ruiz(10)
    Ks = rho[:, None] * lp.dense() * kap[None, :]
    v, _ = o.power_norm(10, max_iters=20000, tol=1e-12)
    assert v == pytest.approx(np.linalg.norm(Ks, 2), rel=1e-6)


# ---------------------------------------------------------------------------
# PDHG steps (Algorithm 1, appendix form) and the Appendix D bounds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [lambda: lpgen.config0(3),
                                   lambda: lpgen.planted(120, 300, 0.04, 9, ge_frac=0.5),
                                   lambda: lpgen.tiny(11, n=7, m=3)])
def test_planted_optimum_is_fixed_point(orc, maker):
    """A saddle point is a fixed point of the PDHG map (Appendix D, final step)."""
    lp = maker()
    o = orc.Oracle(lp)
    x, y = o.steps(lp.x_star, lp.y_star, 0.05, 0.07, 5)
    np.testing.assert_allclose(x, lp.x_star, atol=1e-12)
    np.testing.assert_allclose(y, lp.y_star, atol=1e-12)


def test_step_prox_closed_form(orc):
    """From y = 0 on K = I: x+ = clip(x - tau c, l, u), y+ = q - 2x+ + x scaled by sigma (App. C)."""
    n = 4
    lp = lpgen.from_dense(np.eye(n), [0, 0, 1, 1], [0.5, -1.0, 2.0, 0.1], [1.0, -2.0, 0.5, 3.0],
                          [0, -1, -1, 0], [1, 1, 1, 2])
    o = orc.Oracle(lp)
    x0 = np.array([0.5, 0.5, 0.5, 0.5])
    tau, sigma = 0.3, 0.2
    x, y = o.steps(x0, np.zeros(n), tau, sigma, 1)
    np.testing.assert_allclose(x, [0.2, 1.0, 0.35, 0.0])
    w = sigma * (np.array([0.5, -1.0, 2.0, 0.1]) - (2 * x - x0))
    np.testing.assert_allclose(y, [max(w[0], 0), max(w[1], 0), w[2], w[3]])


@pytest.mark.parametrize("seed", [0, 1])
def test_convergence_bounds_appendix_d(orc, seed):
    """Boundedness and the O(1/N) ergodic gap bound proved in Appendix D.

    With (xh, yh) a saddle point and tau sigma ||K||^2 < 1, for every N:
      (1 - tau sigma ||K||^2) ||yh - y^{N-1}||^2/(2 sigma) + ||xh - x^N||^2/(2 tau)
          <= ||yh - y^0||^2/(2 sigma) + ||xh - x^0||^2/(2 tau)
    and, with x_N = mean(x^1..x^N), y_N = mean(y^0..y^{N-1}) and
    L(x, y) = c'x - y'Kx + q'y:
      L(x_N, yh) - L(xh, y_N) <= (1/N) (||yh - y^0||^2/(2 sigma) + ||xh - x^0||^2/(2 tau)).
    """
    lp = lpgen.planted(60, 150, 0.08, seed, ge_frac=0.5)
    o = orc.Oracle(lp)
    K = lp.dense()
    kn = np.linalg.norm(K, 2)
    tau, sigma = 0.9 / kn / 1.7, 0.9 * 1.7 / kn
    xh, yh = lp.x_star, lp.y_star
    x, y = np.clip(np.zeros(lp.n), lp.l, lp.u), np.zeros(lp.m)
    x0, y0 = x.copy(), y.copy()
    rhs = np.sum((yh - y0) ** 2) / (2 * sigma) + np.sum((xh - x0) ** 2) / (2 * tau)
    xs, ys = np.zeros(lp.n), np.zeros(lp.m)
    q = lp.rhs

    def L(xx, yy):
        return lp.c @ xx - yy @ (K @ xx) + q @ yy

    for N in range(1, 301):
        y_prev = y.copy()
        ys += y_prev
        x, y = o.steps(x, y, tau, sigma, 1)
        xs += x
        lhs = (1 - tau * sigma * kn ** 2) * np.sum((yh - y_prev) ** 2) / (2 * sigma) \
            + np.sum((xh - x) ** 2) / (2 * tau)
        assert lhs <= rhs * (1 + 1e-12) + 1e-12
        gap = L(xs / N, yh) - L(xh, ys / N)
        assert gap <= rhs / N * (1 + 1e-10) + 1e-10


def test_wrong_sign_fails_fixed_point():
    """Guard for the pins above: the paper's Algorithm 1 signs (c + K'y) move off the optimum."""
    lp = lpgen.config0(3)
    A = lp.dense()
    tau = 0.05
    x = np.clip(lp.x_star - tau * (lp.c + A.T @ lp.y_star), lp.l, lp.u)
    assert np.max(np.abs(x - lp.x_star)) > 1e-3


# ---------------------------------------------------------------------------
# restarted solve (Sections 2.3-2.4)
# ---------------------------------------------------------------------------

def test_solve_handsolved_golden(orc):
    g = json.load(open(os.path.join(GOLD, "lp_handsolved.json")))
    lp = lpgen.from_dense(np.array(g["K"]), g["row_type"], g["rhs"], g["c"], g["l"], g["u"])
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-9))
    assert r.status == 0
    np.testing.assert_allclose(r.x, g["x_star"], atol=1e-6)
    np.testing.assert_allclose(r.y, g["y_star"], atol=1e-6)


@pytest.mark.parametrize("seed", range(6))
def test_solve_tiny_matches_vertex_enumeration(orc, seed):
    lp = lpgen.tiny(100 + seed, n=6, m=3, free_frac=0.3 if seed % 2 else 0.0)
    f_bf, _ = vertex_optimum(lp.dense(), lp.row_type, lp.rhs, lp.c, lp.l, lp.u)
    assert _rel(f_bf, lp.f_star) < 1e-9  # the planted value is the brute-force optimum
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-9))
    assert r.status == 0
    assert _rel(r.kkt["pobj"], f_bf) < 1e-7


@pytest.mark.parametrize("unique", [False, True])
def test_solve_c0_restarted_matches_planted_and_highs(orc, unique):
    from scipy.optimize import linprog

    lp = lpgen.config0(0, unique=unique)
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6))
    assert r.status == 0 and r.kkt["rel_kkt"] <= 1e-6
    assert _rel(r.kkt["pobj"], lp.f_star) < 1e-5
    h = linprog(lp.c, A_eq=lp.dense(), b_eq=lp.rhs, bounds=list(zip(lp.l, lp.u)), method="highs")
    assert _rel(h.fun, lp.f_star) < 1e-9
    if unique:
        # unique optimum, but the optimal basis has condition number ~1e5, so at
        # rel-KKT 1e-6 the primal iterate is only within a few percent of x*
        assert np.linalg.norm(r.x - lp.x_star) / np.linalg.norm(lp.x_star) < 0.05


def test_solve_c0_plain(orc):
    lp = lpgen.config0(0)
    r = orc.Oracle(lp).solve(orc.SolveOpts.plain(eps=1e-6, max_iters=400000))
    assert r.status == 0 and r.restarts == 0 and not r.from_avg
    assert _rel(r.kkt["pobj"], lp.f_star) < 1e-5
    assert r.omega == r.omega0


def test_solve_mixed_rows_matches_highs(orc):
    from scipy.optimize import linprog

    lp = lpgen.planted(150, 400, 0.03, 21, ge_frac=0.5)
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-7))
    assert r.status == 0
    ge, eq = lp.row_type == 0, lp.row_type == 1
    A = lp.dense()
    h = linprog(lp.c, A_ub=-A[ge], b_ub=-lp.rhs[ge], A_eq=A[eq], b_eq=lp.rhs[eq],
                bounds=list(zip(lp.l, lp.u)), method="highs")
    assert _rel(h.fun, lp.f_star) < 1e-9
    assert _rel(r.kkt["pobj"], h.fun) < 1e-6


@pytest.mark.slow
def test_solve_small_sced_matches_highs(orc):
    from scipy.optimize import linprog

    lp = lpgen.sced(40, 16, 8, 12, seed=5)
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6, max_iters=400000))
    assert r.status == 0
    ge, eq = lp.row_type == 0, lp.row_type == 1
    A = lp.scipy()
    h = linprog(lp.c, A_ub=-A[ge], b_ub=-lp.rhs[ge], A_eq=A[eq], b_eq=lp.rhs[eq],
                bounds=list(zip(lp.l, [None if not np.isfinite(v) else v for v in lp.u])),
                method="highs")
    assert h.status == 0
    assert _rel(r.kkt["pobj"], h.fun) < 1e-5


def _kkt_w(pres, dres, gap, w):
    """KKT_omega of Section 2.4.2 from a point's scaled-LP terms."""
    return np.sqrt(w * w * pres * pres + dres * dres / (w * w) + gap * gap)


def _assert_restart_rule(tr, omega0, kkt0_start, bs=0.2, bn=0.8, ba=0.36, eps_zero=1e-6):
    """Every check of a trace follows Section 2.4.2 and Algorithm 4.

    The epoch reference, the previous candidate, the epoch length and the
    primal weight are tracked here from the trace itself (not read from the
    solver's state), so a solver that keeps any of them wrongly disagrees with
    its own records.  Returns how often each criterion decided a restart.
    """
    omega, kkt0, prev, last_restart = omega0, kkt0_start, np.inf, 0
    fired = {"sufficient": 0, "necessary": 0, "artificial": 0, "none": 0}
    for i, t in enumerate(tr):
        assert t["omega_before"] == omega
        assert t["kkt0"] == pytest.approx(kkt0, rel=1e-14)
        assert t["kkt_prev"] == prev
        assert t["t_inner"] == t["iter"] - last_restart
        kc = t["kkt_cand"]
        assert kc == pytest.approx(_kkt_w(t["cand_pres"], t["cand_dres"], t["cand_gap"], omega), rel=1e-13)
        if i == len(tr) - 1:
            break  # the terminating check makes no restart decision
        suff = kc <= bs * kkt0
        nec = kc <= bn * kkt0 and kc > prev
        art = t["t_inner"] > ba * t["iter"]
        assert t["restarted"] == int(suff or nec or art), (i, t, suff, nec, art)
        if not t["restarted"]:
            fired["none"] += 1
            assert t["omega"] == omega and t["kkt0_next"] == kkt0
            prev = kc
            continue
        for name, f in (("sufficient", suff), ("necessary", nec), ("artificial", art)):
            fired[name] += f
        dx, dy = t["delta_x"], t["delta_y"]
        if dx > eps_zero and dy > eps_zero:
            want = np.exp(0.5 * np.log(dy / dx) + 0.5 * np.log(omega))
            assert t["omega"] == pytest.approx(want, rel=1e-14)
        else:
            assert t["omega"] == omega
        omega = t["omega"]
        # the new epoch's reference: the candidate's KKT_omega at the NEW omega (reading R10)
        kkt0 = _kkt_w(t["cand_pres"], t["cand_dres"], t["cand_gap"], omega)
        assert t["kkt0_next"] == pytest.approx(kkt0, rel=1e-13)
        prev, last_restart = np.inf, t["iter"]
    return fired


def _start_kkt_w(o, opts, omega0):
    from oracle import KKT as _KKTStruct

    """KKT_omega of the starting point (proj_X(0), 0) on the scaled LP."""
    s = o.scaled(opts.ruiz_iters)
    x = np.clip(np.zeros(o.n), o.l / s.kap, o.u / s.kap)
    k = _KKTStruct()
    o.lib.orc_kkt(s.h, x, np.zeros(o.m), ctypes.byref(k))
    return _kkt_w(k.pres, k.dres, k.gap, omega0)


RESTART_CASES = {"mixed": lambda: lpgen.planted(200, 500, 0.02, 8, ge_frac=0.3),
                 "c0u": lambda: lpgen.config0(3, unique=True),
                 "sced": lambda: lpgen.sced(20, 8, 6, 6, seed=2)}


def check_restart_properties(orc, case, lib=None):
    """Solves RESTART_CASES[case] to 1e-7 and checks every check of its trace
    with _assert_restart_rule (``lib``: an oracle library built elsewhere)."""
    lp = RESTART_CASES[case]()
    o = orc.Oracle(lp, lib=lib)
    opts = orc.SolveOpts(eps=1e-7, max_iters=200000)
    r = o.solve(opts)
    assert r.status == 0 and r.restarts > 0
    fired = _assert_restart_rule(r.trace, r.omega0, _start_kkt_w(o, opts, r.omega0))
    assert r.trace[0]["restarted"] == 1  # first check: t_inner = k_total > 0.36 k_total
    assert sum(t["restarted"] for t in r.trace) == r.restarts
    return fired


def check_golden_1x1(orc, lib=None):
    """The oracle's trace on the 1 x 1 LP of tests/golden/restart_1x1.py
    against the stored hand derivation; returns the restart kinds seen."""
    g = json.load(open(os.path.join(GOLD, "restart_trace_1x1.json")))
    lp = lpgen.from_dense(np.array(g["lp"]["K"]), g["lp"]["row_type"], g["lp"]["q"], g["lp"]["c"],
                          np.array(g["lp"]["l"]), np.array([np.inf]))
    o = orc.Oracle(lp, lib=lib)
    opts = orc.SolveOpts(eps=g["opts"]["eps"], check_every=g["opts"]["check_every"],
                         ruiz_iters=g["opts"]["ruiz_iters"])
    r = o.solve(opts)
    assert r.eta == g["opts"]["eta"] and r.omega0 == g["opts"]["omega0"]
    assert r.status == 0
    want = g["checks"]
    assert len(r.trace) == len(want)
    kinds = set()
    for t, w in zip(r.trace, want):
        assert t["iter"] == w["iter"] and t["t_inner"] == w["t_inner"]
        assert t["restarted"] == w["restarted"] and t["cand_avg"] == w["cand_avg"], (t, w)
        for k in ("kkt_cand", "kkt0", "omega_before", "omega", "kkt0_next", "rel_kkt_cur", "rel_kkt_avg",
                  "delta_x", "delta_y"):
            assert t[k] == pytest.approx(w[k], rel=1e-9, abs=1e-300), (k, t, w)
        wp = np.inf if w["kkt_prev"] == "inf" else w["kkt_prev"]
        assert t["kkt_prev"] == pytest.approx(wp, rel=1e-9)
        if w["restarted"] and len(w["criteria"]) == 1:
            kinds.add(w["criteria"][0])
    assert r.iters == want[-1]["iter"] and r.restarts == sum(w["restarted"] for w in want)
    # the start (0, 0) has pres = 4, dres = 0, gap = 0: KKT_omega0 = 0.75 * 4 = 3
    _assert_restart_rule(r.trace, r.omega0, 3.0)
    return kinds


@pytest.mark.parametrize("case", sorted(RESTART_CASES))
def test_solve_restart_trace_properties(orc, case):
    """At every check the restart decision is exactly (sufficient decay) or
    (necessary decay and no progress) or (long inner loop) with 0.2 / 0.8 /
    0.36 (Section 2.4.2); omega moves only at restarts, by Algorithm 4; the
    new epoch's reference is the candidate's metric at the new omega."""
    fired = check_restart_properties(orc, case)
    # the trace exercises more than the artificial rule and has checks without a restart
    assert fired["sufficient"] + fired["necessary"] > 0 and fired["none"] > 0, fired


def test_restart_trace_1x1_golden(orc):
    """The oracle's check-by-check trace on a 1 x 1 LP equals the trace derived
    by hand from Section 2.4.2 and Algorithm 4 (tests/golden/restart_1x1.py,
    60-digit arithmetic): the same restart decisions and candidates at every
    check, every kind of restart present, and the KKT_omega values, the
    reference values and omega to 1e-9."""
    assert check_golden_1x1(orc) == {"sufficient", "necessary", "artificial"}


def test_solve_zero_rows_closed_form(orc):
    """m = 0: x_i = l_i if c_i > 0, u_i if c_i < 0 (dual function derivation, App. B)."""
    n = 6
    c = np.array([1.0, -2.0, 0.5, -0.1, 3.0, -1.0])
    lp = lpgen.from_dense(np.zeros((0, n)), [], [], c, np.full(n, -1.0), np.full(n, 2.0))
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-10))
    np.testing.assert_allclose(r.x, np.where(c > 0, -1.0, 2.0), atol=1e-9)


def test_solve_identity_equalities(orc):
    """K = I with "=" rows: x = b when l <= b <= u."""
    n = 5
    b = np.array([0.5, -0.2, 1.0, 0.0, 0.9])
    lp = lpgen.from_dense(np.eye(n), [1] * n, b, np.array([1.0, -1, 2, 0.5, -3]),
                          np.full(n, -1.0), np.full(n, 1.0))
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-10))
    np.testing.assert_allclose(r.x, b, atol=1e-8)


# ---------------------------------------------------------------------------
# differentiation oracle
# ---------------------------------------------------------------------------

def _vjp_case(orc, seed=0, K=25):
    lp = lpgen.planted(30, 70, 0.1, seed, ge_frac=0.5)
    o = orc.Oracle(lp)
    rng = np.random.default_rng(seed)
    # strictly inside the box: a start on a bound with a zero reduced cost sits on
    # a kink of the clip, where central differences average two one-sided slopes
    x0 = lp.l + rng.uniform(0.1, 0.9, size=lp.n) * (lp.u - lp.l)
    y0 = rng.standard_normal(lp.m) * 0.3
    kn, _ = o.power_norm(3)
    tau, sigma = 0.8 / kn, 0.8 / kn
    return lp, o, x0, y0, tau, sigma, K


@pytest.mark.parametrize("seed", [0, 1])
def test_unrolled_vjp_matches_central_fd(orc, seed):
    lp, o, x0, y0, tau, sigma, K = _vjp_case(orc, seed)
    rng = np.random.default_rng(100 + seed)
    gx = rng.standard_normal(lp.n)
    gy = rng.standard_normal(lp.m)

    def loss(c, q, l, u, xx, yy):
        xk, yk = o.unrolled(3, tau, sigma, c, q, l, u, xx, yy, K)
        return gx @ xk + gy @ yk

    g = o.unrolled_vjp(3, tau, sigma, lp.c, lp.rhs, lp.l, lp.u, x0, y0, K, gx, gy)
    args = dict(c=lp.c, q=lp.rhs, l=lp.l, u=lp.u, x0=x0, y0=y0)
    names = ["c", "q", "l", "u", "x0", "y0"]
    h = 1e-6
    for name in names:
        for d in range(3):
            v = rng.standard_normal(args[name].shape[0])
            ap = {k: a.copy() for k, a in args.items()}
            am = {k: a.copy() for k, a in args.items()}
            ap[name] = ap[name] + h * v
            am[name] = am[name] - h * v
            f0 = loss(*[args[k] for k in names])
            fp = loss(*[ap[k] for k in names])
            fm = loss(*[am[k] for k in names])
            an = g[name] @ v
            central, fwd, bwd = (fp - fm) / (2 * h), (fp - f0) / h, (f0 - fm) / h
            close = lambda a, b: abs(a - b) <= 1e-5 * abs(b) + 1e-7
            if close(fwd, bwd):
                assert close(an, central), (name, an, central)
            else:
                # the piecewise-linear map has a kink at the base point (an iterate
                # exactly on a bound); the adjoint is then one of the one-sided slopes
                assert close(an, fwd) or close(an, bwd), (name, an, fwd, bwd)


def test_unrolled_zero_steps_is_identity(orc):
    lp, o, x0, y0, tau, sigma, _ = _vjp_case(orc, 0)
    xk, yk = o.unrolled(3, tau, sigma, lp.c, lp.rhs, lp.l, lp.u, x0, y0, 0)
    np.testing.assert_allclose(xk, x0, rtol=1e-15)
    np.testing.assert_allclose(yk, y0, rtol=1e-15)


# ---------------------------------------------------------------------------
# adaptive step size (Section 2.4.4, Algorithm 5)
# ---------------------------------------------------------------------------

def test_adaptive_attempt_golden_1x1(orc):
    """Hand-worked attempts: a rejection, an acceptance and the zero-interaction case."""
    with open(os.path.join(GOLD, "adaptive_1x1.json")) as f:
        g = json.load(f)
    for cs in g["cases"]:
        lo = -np.inf if cs["l"] is None else cs["l"]
        hi = np.inf if cs["u"] is None else cs["u"]
        lp = lpgen.from_dense(np.array([[1.0]]), [cs["row_type"]], [cs["q"]], [cs["c"]], [lo], [hi])
        acc, xn, yn, eb, en = orc.Oracle(lp).adaptive_attempt([0.0], [0.0], cs["omega"], cs["eta"], cs["k"])
        assert acc == cs["accepted"], cs["name"]
        if cs["etabar"] == "inf":
            assert eb == np.inf
        else:
            assert eb == pytest.approx(cs["etabar"], rel=1e-14), cs["name"]
        assert en == pytest.approx(cs["eta_next"], rel=1e-14), cs["name"]
        assert xn[0] == pytest.approx(cs["x"], rel=1e-14, abs=1e-300), cs["name"]
        assert yn[0] == pytest.approx(cs["y"], rel=1e-14, abs=1e-300), cs["name"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adaptive_etabar_at_least_inverse_norm(orc, seed):
    """2|dy' K dx| <= ||K||_2 (w ||dx||^2 + ||dy||^2 / w) (Cauchy-Schwarz and
    AM-GM), so etabar >= 1/||K||_2 and every step up to 1/||K||_2 is accepted;
    the candidate is one fixed PDHG step with tau = eta/w, sigma = eta w."""
    lp = lpgen.planted(40, 90, 0.08, 30 + seed, ge_frac=0.5)
    o = orc.Oracle(lp)
    kn = np.linalg.norm(lp.scipy().toarray(), 2)
    rng = np.random.default_rng(seed)
    lo = np.where(np.isfinite(lp.l), lp.l, -3.0)
    hi = np.where(np.isfinite(lp.u), lp.u, lo + 6.0)
    for trial in range(6):
        x = lo + rng.uniform(0, 1, lp.n) * (hi - lo)
        y = rng.standard_normal(lp.m)
        y[lp.row_type == 0] = np.abs(y[lp.row_type == 0])
        w = [0.3, 1.0, 4.0][trial % 3]
        for f in (0.5, 0.999, 3.0, 30.0):
            eta = f / kn
            acc, xn, yn, eb, en = o.adaptive_attempt(x, y, w, eta, trial + 1)
            assert eb >= (1.0 / kn) * (1.0 - 1e-12)
            assert acc == (eta <= eb)
            if f < 1.0:
                assert acc
            xo, yo = o.steps(x, y, eta / w, eta * w, 1)
            np.testing.assert_allclose(xn, xo, rtol=1e-14, atol=1e-14)
            np.testing.assert_allclose(yn, yo, rtol=1e-14, atol=1e-14)
            assert 0.0 < en <= (1.0 + (trial + 2) ** -0.6) * eta * (1 + 1e-15)


@pytest.mark.parametrize("maker", [lambda: lpgen.config0(0), lambda: lpgen.config0(1, unique=True),
                                   lambda: lpgen.planted(150, 400, 0.03, 8, ge_frac=0.5)])
def test_adaptive_solve_matches_planted(orc, maker):
    lp = maker()
    o = orc.Oracle(lp)
    r = o.solve(orc.SolveOpts(eps=1e-6, adaptive_step=True))
    assert r.status == 0
    chk = o.kkt(r.x, r.y)
    assert chk["rel_kkt"] <= 1e-6 * 1.0001
    assert _rel(chk["pobj"], lp.f_star) <= 1e-5
    assert 0 < r.accepted <= r.iters
    assert r.eta_next > 0.0


def test_adaptive_solve_matches_highs(orc):
    from scipy.optimize import linprog

    lp = lpgen.planted(120, 260, 0.05, 21, ge_frac=0.6)
    A = lp.scipy().toarray()
    ge, eq = lp.row_type == 0, lp.row_type == 1
    ref = linprog(lp.c, A_ub=-A[ge], b_ub=-lp.rhs[ge], A_eq=A[eq], b_eq=lp.rhs[eq],
                  bounds=list(zip(lp.l, lp.u)), method="highs")
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-7, adaptive_step=True))
    assert r.status == 0
    assert _rel(r.kkt["pobj"], ref.fun) <= 1e-6


def test_adaptive_first_check_weighted_average(orc):
    """Replays the first check period attempt by attempt with the pinned single
    attempt and forms the step-weighted average sum(eta_i z_i) / sum(eta_i)
    (Section 2.4.2) in numpy: the solve's first check must report its KKT."""
    lp = lpgen.planted(60, 150, 0.05, 1, ge_frac=0.5)
    o = orc.Oracle(lp)
    r = o.solve(orc.SolveOpts(eps=1e-12, adaptive_step=True, max_iters=64))
    rho, kap = o.ruiz(10)
    x = np.clip(np.zeros(lp.n), lp.l / kap, lp.u / kap)
    y = np.zeros(lp.m)
    eta, w = r.eta, r.omega0
    sx, sy, ws, acc_n = np.zeros(lp.n), np.zeros(lp.m), 0.0, 0
    ux, uy = np.zeros(lp.n), np.zeros(lp.m)
    for k in range(1, 65):
        acc, xn, yn, eb, en = o.adaptive_attempt(x, y, w, eta, k, ruiz_iters=10)
        if acc:
            x, y = xn, yn
            sx += eta * x
            sy += eta * y
            ws += eta
            ux += x
            uy += y
            acc_n += 1
        eta = en
    t0 = r.trace[0]
    assert t0["accepted"] == acc_n
    assert t0["eta_next"] == pytest.approx(eta, rel=1e-12)
    avg = o.kkt(kap * sx / ws, rho * sy / ws)
    cur = o.kkt(kap * x, rho * y)
    assert t0["rel_kkt_avg"] == pytest.approx(avg["rel_kkt"], rel=1e-10)
    assert t0["rel_kkt_cur"] == pytest.approx(cur["rel_kkt"], rel=1e-10)
    # the plain mean of the same iterates is measurably different (the weights matter)
    plain = o.kkt(kap * ux / acc_n, rho * uy / acc_n)
    assert abs(plain["rel_kkt"] - avg["rel_kkt"]) > 1e3 * abs(t0["rel_kkt_avg"] - avg["rel_kkt"])


# ---------------------------------------------------------------------------
# infeasibility detection (Section 2.4.5, Algorithm 6)
# ---------------------------------------------------------------------------

def _fl(v):
    return np.array([float(t) for t in v], dtype=np.float64)


def test_infeas_golden_cases(orc):
    with open(os.path.join(GOLD, "infeas_cases.json")) as f:
        g = json.load(f)
    for cs in g["cases"]:
        lp = lpgen.from_dense(np.array(cs["K"]), cs["row_type"], cs["rhs"], cs["c"], _fl(cs["l"]), _fl(cs["u"]))
        out = orc.Oracle(lp).infeas_test(_fl(cs["x"]), _fl(cs["y"]), _fl(cs["xp"]), _fl(cs["yp"]), g["tol"])
        assert out["verdict"] == cs["verdict"], (cs["name"], out)
        for k in ("psi", "res_norm", "c_dx", "ineq_min", "v_viol"):
            if k in cs:
                want = float(cs[k])
                if np.isinf(want):
                    assert out[k] == want, (cs["name"], k)
                else:
                    assert out[k] == pytest.approx(want, rel=1e-9, abs=1e-15), (cs["name"], k, out[k])


def _highs_status(lp):
    from scipy.optimize import linprog

    A = lp.scipy().toarray()
    ge, eq = lp.row_type == 0, lp.row_type == 1
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b) for a, b in zip(lp.l, lp.u)]
    r = linprog(lp.c, A_ub=-A[ge] if ge.any() else None, b_ub=-lp.rhs[ge] if ge.any() else None,
                A_eq=A[eq] if eq.any() else None, b_eq=lp.rhs[eq] if eq.any() else None, bounds=bounds,
                method="highs")
    return r.status  # 0 optimal, 2 infeasible, 3 unbounded


@pytest.mark.parametrize("maker,want,highs", [
    (lambda: lpgen.primal_infeasible(60, 150, 0.05, 1, "bound"), 4, 2),
    (lambda: lpgen.primal_infeasible(60, 150, 0.05, 2, "pair"), 4, 2),
    (lambda: lpgen.primal_infeasible(300, 700, 0.02, 4, "pair"), 4, 2),
    (lambda: lpgen.dual_infeasible(60, 150, 0.05, 3), 5, 3),
    (lambda: lpgen.dual_infeasible(300, 700, 0.02, 5), 5, 3),
])
@pytest.mark.parametrize("adaptive", [False, True])
def test_infeas_detected_matches_highs(orc, maker, want, highs, adaptive):
    lp = maker()
    assert _highs_status(lp) == highs
    r = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6, detect_infeas=True, adaptive_step=adaptive,
                                           max_iters=100_000))
    assert r.status == want, (r.status, r.iters)
    without = orc.Oracle(lp).solve(orc.SolveOpts(eps=1e-6, adaptive_step=adaptive, max_iters=r.iters + 640))
    assert without.status == 1  # no optimum exists: only the iteration limit stops it


@pytest.mark.parametrize("maker", [lambda: lpgen.config0(1, unique=True),
                                   lambda: lpgen.planted(300, 700, 0.02, 5, ge_frac=0.5),
                                   lambda: lpgen.sced(40, 16, 8, 12, seed=5),
                                   lambda: lpgen.tiny(3, n=8, m=4, free_frac=0.5),
                                   lambda: lpgen.planted(100, 250, 0.05, 9, ge_frac=0.8)])
@pytest.mark.parametrize("adaptive", [False, True])
def test_infeas_no_false_positive(orc, maker, adaptive):
    """On feasible bounded LPs detection never fires: the solve takes the same
    path as without it."""
    lp = maker()
    o = orc.Oracle(lp)
    a = o.solve(orc.SolveOpts(eps=1e-8, detect_infeas=True, adaptive_step=adaptive, max_iters=60_000))
    b = o.solve(orc.SolveOpts(eps=1e-8, adaptive_step=adaptive, max_iters=60_000))
    assert a.status == b.status and a.status in (0, 1)
    assert a.iters == b.iters
    np.testing.assert_array_equal(a.x, b.x)


# ---------------------------------------------------------------------------
# fishnet casting (Section 2.5, Algorithm 7)
# ---------------------------------------------------------------------------

def _fish_setup(orc, lp, ruiz=10):
    o = orc.Oracle(lp)
    r = o.solve(orc.SolveOpts(max_iters=1, eps=1e-12, ruiz_iters=ruiz))
    rho, kap = o.ruiz(ruiz)
    return o, r.eta, r.omega0, r.knorm, rho, kap


def _replay(o, lp, eta, w, kn, rho, kap, P, k, G, wraw, ruiz=10):
    """Algorithm 7 replayed from pinned pieces: the scaled product through
    orc_spmv, k fixed steps through orc_steps, the gap through orc_kkt."""
    X = [(kn / np.sqrt(lp.n)) * G[q] for q in range(P)]
    Y = [rho * o.spmv(kap * x) for x in X]
    j, rnd, pos, keeps = P, 0, 0, []
    while j > 1:
        gaps = []
        for q in range(j):
            X[q], Y[q] = o.steps(X[q], Y[q], eta / w, eta * w, k, ruiz_iters=ruiz)
            gaps.append(o.kkt(kap * X[q], rho * Y[q])["gap"])
        order = sorted(range(j), key=lambda q: (gaps[q], q))
        half = j // 2
        keeps.append(order[:half])
        X, Y = [X[q] for q in order[:half]], [Y[q] for q in order[:half]]
        if rnd % 2 == 1 and j > 2:
            for a in range(half):
                ws = np.abs(wraw[pos:pos + half])
                pos += half
                ws = ws / ws.sum()
                X.append(sum(ws[s] * X[s] for s in range(half)))
                Y.append(sum(ws[s] * Y[s] for s in range(half)))
        j = len(X)
        rnd += 1
    return kap * X[0], rho * Y[0], keeps


@pytest.mark.parametrize("P,k", [(2, 20), (4, 16), (8, 10), (16, 6)])
def test_fishnet_replay_from_pinned_pieces(orc, P, k):
    lp = lpgen.planted(40, 100, 0.06, 17, ge_frac=0.5)
    o, eta, w, kn, rho, kap = _fish_setup(orc, lp)
    G, wraw = lpgen.fishnet_draws(lp.n, P, seed=5)
    x, y, gaps, keep = o.fishnet(10, eta, w, kn, P, k, G, wraw)
    xr, yr, keeps = _replay(o, lp, eta, w, kn, rho, kap, P, k, G, wraw)
    p = int(np.log2(P))
    assert len(keep) == (1 if P == 2 else 2 * p - 2)
    for r, kr in enumerate(keeps):
        assert list(keep[r][:len(kr)]) == kr
    np.testing.assert_allclose(x, xr, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(y, yr, rtol=1e-10, atol=1e-12)


def test_fishnet_one_hot_weights_copy_survivors(orc):
    """Raw weights that are one-hot make each new point a copy of a survivor,
    so the next round's gaps come in equal pairs."""
    lp = lpgen.planted(40, 100, 0.06, 18, ge_frac=0.3)
    o, eta, w, kn, rho, kap = _fish_setup(orc, lp)
    P = 8
    G, _ = lpgen.fishnet_draws(lp.n, P, seed=6)
    wraw = np.zeros(P * P)
    # round 0 keeps 4 of 8; round 1 keeps 2 of 4 and appends 2 new points,
    # point a one-hot on survivor a
    wraw[0] = 1.0
    wraw[3] = -1.0  # the sign of a draw does not matter
    x, y, gaps, keep = o.fishnet(10, eta, w, kn, P, 8, G, wraw)
    g2 = gaps[2][:4]
    np.testing.assert_array_equal(g2[:2], g2[2:4])
    # all-zero draws give equal weights: the replay with equal weights agrees
    x2, y2, _, _ = o.fishnet(10, eta, w, kn, P, 8, G, np.zeros(P * P))
    x3, y3, _, _ = o.fishnet(10, eta, w, kn, P, 8, G, np.ones(P * P))
    np.testing.assert_allclose(x2, x3, rtol=1e-13, atol=1e-15)


def test_fishnet_warm_start_solves(orc):
    lp = lpgen.config0(2)
    o, eta, w, kn, rho, kap = _fish_setup(orc, lp)
    G, wraw = lpgen.fishnet_draws(lp.n, 32, seed=7)
    x0, y0, gaps, keep = o.fishnet(10, eta, w, kn, 32, 64, G, wraw)
    r = o.solve(orc.SolveOpts(eps=1e-6), x0=x0, y0=y0)
    assert r.status == 0
    assert _rel(r.kkt["pobj"], lp.f_star) <= 1e-5
    # culling keeps the smaller gaps
    for rr in range(len(keep)):
        kept = [q for q in keep[rr] if q >= 0]
        n_live = int(np.count_nonzero(gaps[rr] != 0.0)) or len(kept) * 2
        dropped = [q for q in range(n_live) if q not in kept]
        if dropped:
            assert max(gaps[rr][kept]) <= min(gaps[rr][dropped])


def test_solve_from_start_point(orc):
    """A start point is projected: starting at the planted optimum stops at the
    first check."""
    lp = lpgen.config0(0)
    o = orc.Oracle(lp)
    r = o.solve(orc.SolveOpts(eps=1e-6), x0=lp.x_star, y0=lp.y_star)
    assert r.status == 0 and r.iters == 0

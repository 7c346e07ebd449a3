"""FP64 CPU oracle for restarted PDHG (Python side of ``pdhg_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library and its
Python binding never import, call or fall back to it, and the two share no
code: the only common input is the problem data built by ``lpgen``.

The C library is plain double-precision loops in the order the paper states
the method (see the header of ``pdhg_oracle.c`` for the section each function
follows).  This wrapper only marshals arrays and performs one bookkeeping step
of its own: the stable reordering of rows so that the ">=" rows come first
(the stacked K = [G; A] of Section 2.2); vectors indexed by rows are taken and
returned in the caller's row order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdhg_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (plain IEEE double; x86-64 without FMA).

    ``src`` / ``out`` default to this package's source and library; the tests
    that plant a mistake in a copy of the source build that copy elsewhere."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off", src, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class KKT(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("pres", "dres", "pobj", "dobj", "gap", "rel_pres", "rel_dres", "rel_gap", "rel_kkt")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Opts(C.Structure):
    _fields_ = [("ruiz_iters", C.c_int), ("use_restarts", C.c_int), ("use_pw_update", C.c_int),
                ("check_every", C.c_int), ("max_iters", C.c_longlong), ("eps", C.c_double),
                ("step_size", C.c_double), ("step_frac", C.c_double), ("primal_weight", C.c_double),
                ("power_max_iters", C.c_int), ("power_tol", C.c_double), ("beta_suff", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double), ("eps_zero", C.c_double),
                ("adaptive_step", C.c_int), ("detect_infeas", C.c_int), ("infeas_tol", C.c_double)]


class InfeasOut(C.Structure):
    _fields_ = [("eq_norm", C.c_double), ("ineq_min", C.c_double), ("c_dx", C.c_double),
                ("v_viol", C.c_double), ("res_norm", C.c_double), ("dy_min", C.c_double),
                ("psi", C.c_double), ("verdict", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("from_avg", C.c_int), ("iters", C.c_longlong),
                ("restarts", C.c_int), ("power_iters", C.c_int), ("knorm", C.c_double),
                ("eta", C.c_double), ("omega0", C.c_double), ("omega", C.c_double),
                ("tau", C.c_double), ("sigma", C.c_double), ("kkt", KKT), ("trace_len", C.c_int),
                ("accepted", C.c_longlong), ("eta_next", C.c_double)]


class TraceRec(C.Structure):
    _fields_ = [("iter", C.c_longlong), ("restarted", C.c_int), ("cand_avg", C.c_int),
                ("kkt_cand", C.c_double), ("omega", C.c_double), ("rel_kkt_cur", C.c_double),
                ("rel_kkt_avg", C.c_double), ("eta_next", C.c_double), ("accepted", C.c_longlong),
                ("t_inner", C.c_longlong), ("kkt0", C.c_double), ("kkt_prev", C.c_double),
                ("omega_before", C.c_double), ("delta_x", C.c_double), ("delta_y", C.c_double),
                ("kkt0_next", C.c_double), ("cand_pres", C.c_double), ("cand_dres", C.c_double),
                ("cand_gap", C.c_double)]


_lib = None


def _load(path: Optional[str] = None):
    """The oracle library with its signatures declared (``path``: a library
    built from a copy of the source, loaded beside this package's own)."""
    global _lib
    if path is not None or _lib is None:
        if path is None and not os.path.exists(_LIB):
            build()
        L = C.CDLL(path or _LIB)
        P = C.c_void_p
        D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        L.orc_prob_create.restype = P
        L.orc_prob_create.argtypes = [C.c_int64, C.c_int64, C.c_int64, I64, I32, D, D, D, D, D]
        L.orc_prob_free.argtypes = [P]
        L.orc_spmv.argtypes = [P, D, D]
        L.orc_spmv_t.argtypes = [P, D, D]
        L.orc_kkt.argtypes = [P, D, D, C.POINTER(KKT)]
        L.orc_ruiz.argtypes = [P, C.c_int, D, D]
        L.orc_prob_scaled.restype = P
        L.orc_prob_scaled.argtypes = [P, D, D]
        L.orc_power_norm.restype = C.c_double
        L.orc_power_norm.argtypes = [P, C.c_int, C.c_double, C.POINTER(C.c_int)]
        L.orc_steps.argtypes = [P, C.c_double, C.c_double, D, D, C.c_longlong]
        L.orc_solve_from.restype = C.c_int
        L.orc_solve_from.argtypes = [P, C.POINTER(Opts), C.c_void_p, C.c_void_p, D, D, C.POINTER(Result),
                                     C.c_void_p, C.c_int]
        L.orc_fishnet.restype = C.c_int
        L.orc_fishnet.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_int, C.c_longlong, D, D, D, D,
                                  C.c_void_p, C.c_void_p]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [P, C.POINTER(Opts), D, D, C.POINTER(Result), C.c_void_p, C.c_int]
        L.orc_infeas_test.restype = C.c_int
        L.orc_infeas_test.argtypes = [P, D, D, D, D, C.c_double, C.POINTER(InfeasOut)]
        L.orc_adaptive_attempt.restype = C.c_int
        L.orc_adaptive_attempt.argtypes = [P, C.c_double, C.c_double, C.c_longlong, D, D, D, D,
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_unrolled.argtypes = [P, D, D, C.c_double, C.c_double, D, D, D, D, D, D,
                                   C.c_longlong, D, D]
        L.orc_unrolled_vjp.argtypes = [P, D, D, C.c_double, C.c_double, D, D, D, D, D, D,
                                       C.c_longlong, D, D, D, D, D, D, D, D]
        if path is not None:
            return L
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class SolveOpts:
    """Options of the restarted solve; defaults are the paper's constants.

    eps 1e-4 (Section 2.3.2), step 0.9/||K||_2 (Sections 4.1-4.2), restart
    constants 0.2 / 0.8 / 0.36 (Section 2.4.2), eps_zero 1e-6 (Section 2.4.3).
    Choices the paper leaves open: 10 Ruiz passes, a check every 64 iterations,
    power iteration to 1e-6 relative change or 1000 passes.  adaptive_step
    turns on the backtracking step size of Algorithm 5 (Section 2.4.4); the
    first attempt tries the fixed step.  detect_infeas turns on the
    infeasibility tests of Algorithm 6 (Section 2.4.5) at every check, on the
    difference of the last step, with tolerance infeas_tol (1e-4, Section 4).
    """

    ruiz_iters: int = 10
    use_restarts: bool = True
    use_pw_update: bool = True
    check_every: int = 64
    max_iters: int = 1_000_000
    eps: float = 1e-4
    step_size: float = 0.0
    step_frac: float = 0.9
    primal_weight: float = 0.0
    power_max_iters: int = 1000
    power_tol: float = 1e-6
    beta_suff: float = 0.2
    beta_nec: float = 0.8
    beta_art: float = 0.36
    eps_zero: float = 1e-6
    adaptive_step: bool = False
    detect_infeas: bool = False
    infeas_tol: float = 1e-4

    @staticmethod
    def plain(**kw) -> "SolveOpts":
        """Plain PDHG: no scaling, no restarts, no primal-weight updates."""
        o = SolveOpts(ruiz_iters=0, use_restarts=False, use_pw_update=False)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def c(self) -> Opts:
        return Opts(self.ruiz_iters, int(self.use_restarts), int(self.use_pw_update),
                    self.check_every, self.max_iters, self.eps, self.step_size, self.step_frac,
                    self.primal_weight, self.power_max_iters, self.power_tol, self.beta_suff,
                    self.beta_nec, self.beta_art, self.eps_zero, int(self.adaptive_step),
                    int(self.detect_infeas), self.infeas_tol)


@dataclass
class SolveResult:
    status: int
    x: np.ndarray
    y: np.ndarray
    iters: int
    restarts: int
    from_avg: bool
    knorm: float
    eta: float
    omega0: float
    omega: float
    kkt: dict
    power_iters: int
    trace: list = field(default_factory=list)
    accepted: int = 0
    eta_next: float = 0.0


class Oracle:
    """An LP loaded into the oracle (rows reordered to [G; A] internally)."""

    def __init__(self, lp, lib=None):
        self.lib = lib if lib is not None else _load()
        self.lp = lp
        rt = np.asarray(lp.row_type)
        ge = np.nonzero(rt == 0)[0]
        eq = np.nonzero(rt != 0)[0]
        self.perm = np.concatenate([ge, eq]).astype(np.int64)  # internal row i = user row perm[i]
        self.m1 = int(ge.shape[0])
        self.n, self.m = int(lp.n), int(lp.m)
        lens = np.diff(lp.rowptr)[self.perm]
        rp = np.zeros(self.m + 1, dtype=np.int64)
        np.cumsum(lens, out=rp[1:])
        idx = _gather_rows(lp.rowptr, self.perm)
        self._rp = rp
        self._ci = np.ascontiguousarray(np.asarray(lp.col)[idx], dtype=np.int32)
        self._v = _f64(np.asarray(lp.val)[idx])
        self.q = _f64(np.asarray(lp.rhs)[self.perm])
        self.c, self.l, self.u = _f64(lp.c), _f64(lp.l), _f64(lp.u)
        self.h = self.lib.orc_prob_create(self.n, self.m, self.m1, self._rp, self._ci, self._v,
                                          self.c, self.q, self.l, self.u)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_prob_free(h)
            self.h = None

    # row-order helpers ------------------------------------------------------
    def to_internal_rows(self, y):
        return _f64(np.asarray(y)[self.perm])

    def to_user_rows(self, yi):
        out = np.empty(self.m)
        out[self.perm] = yi
        return out

    # primitives -------------------------------------------------------------
    def spmv(self, x):
        """K x in user row order."""
        out = np.empty(self.m)
        self.lib.orc_spmv(self.h, _f64(x), out)
        return self.to_user_rows(out)

    def spmv_t(self, y):
        """K^T y for y in user row order."""
        out = np.empty(self.n)
        self.lib.orc_spmv_t(self.h, self.to_internal_rows(y), out)
        return out

    def kkt(self, x, y) -> dict:
        """Relative KKT error terms (Section 2.3.2) of (x, y), y in user row order."""
        k = KKT()
        self.lib.orc_kkt(self.h, _f64(x), self.to_internal_rows(y), C.byref(k))
        return k.as_dict()

    def ruiz(self, iters: int):
        """Ruiz factors (rho in user row order, kappa) after ``iters`` passes."""
        rho = np.empty(self.m)
        kap = np.empty(self.n)
        self.lib.orc_ruiz(self.h, iters, rho, kap)
        return self.to_user_rows(rho), kap

    def scaled(self, iters: int) -> "_Scaled":
        return _Scaled(self, iters)

    def power_norm(self, ruiz_iters: int = 0, max_iters: int = 1000, tol: float = 1e-6):
        s = self.scaled(ruiz_iters)
        it = C.c_int(0)
        v = self.lib.orc_power_norm(s.h, max_iters, tol, C.byref(it))
        return v, it.value

    def steps(self, x, y, tau, sigma, k, ruiz_iters: int = 0):
        """k fixed PDHG steps on the scaled problem; (x, y) in scaled variables, y user order."""
        s = self.scaled(ruiz_iters)
        xi = _f64(np.array(x, copy=True))
        yi = self.to_internal_rows(y)
        self.lib.orc_steps(s.h, tau, sigma, xi, yi, k)
        return xi, self.to_user_rows(yi)

    def solve(self, opts: Optional[SolveOpts] = None, trace_cap: int = 4096, x0=None, y0=None) -> SolveResult:
        """Restarted solve; (x0, y0) (original variables, y in user row order)
        replace the default start proj_X(0), 0."""
        opts = opts or SolveOpts()
        x = np.empty(self.n)
        y = np.empty(self.m)
        r = Result()
        tr = (TraceRec * trace_cap)()
        xs = None if x0 is None else _f64(x0)
        ys = None if y0 is None else self.to_internal_rows(y0)
        self.lib.orc_solve_from(self.h, C.byref(opts.c()), None if xs is None else xs.ctypes.data,
                                None if ys is None else ys.ctypes.data, x, y, C.byref(r),
                                C.cast(tr, C.c_void_p), trace_cap)
        trace = [{k: getattr(t, k) for k, _ in TraceRec._fields_} for t in tr[:r.trace_len]]
        return SolveResult(r.status, x, self.to_user_rows(y), r.iters, r.restarts, bool(r.from_avg),
                           r.knorm, r.eta, r.omega0, r.omega, r.kkt.as_dict(), r.power_iters, trace,
                           r.accepted, r.eta_next)

    def fishnet(self, ruiz_iters, eta, omega, knorm, P, k, G, wraw):
        """Algorithm 7 on the scaled problem (Ruiz passes ruiz_iters) with fixed
        steps eta, omega, radius knorm, P = 2^p points, k steps per round, the
        standard normal draws G (P x n, point-major) and wraw (repopulation
        draws).  Returns the last point in original variables (y in user row
        order), each round's gaps (rounds x P) and kept indices (rounds x P,
        -1 past the kept half)."""
        s = self.scaled(ruiz_iters)
        x, y = np.empty(self.n), np.empty(self.m)
        maxr = 2 * 7
        gaps = np.zeros((maxr, P))
        keep = np.zeros((maxr, P), dtype=np.int32)
        G = _f64(np.asarray(G).reshape(-1))
        w = _f64(np.asarray(wraw).reshape(-1)) if len(wraw) else np.zeros(1)
        rounds = self.lib.orc_fishnet(s.h, eta, omega, knorm, P, k, G, w, x, y, gaps.ctypes.data,
                                      keep.ctypes.data)
        if rounds < 0:
            raise ValueError("P must be a power of two in 2..64")
        return s.kap * x, self.to_user_rows(s.rho_i * y), gaps[:rounds], keep[:rounds]

    def infeas_test(self, x, y, xp, yp, tol: float = 1e-4) -> dict:
        """Algorithm 6's tests on the original LP for dx = x - xp, dy = y - yp
        (original variables, y in user row order); verdict 0 none, 1 primal
        infeasible, 2 dual infeasible."""
        out = InfeasOut()
        self.lib.orc_infeas_test(self.h, _f64(x), self.to_internal_rows(y), _f64(xp), self.to_internal_rows(yp),
                                 tol, C.byref(out))
        return out.as_dict()

    def adaptive_attempt(self, x, y, omega, eta, k, ruiz_iters: int = 0):
        """One attempt of Algorithm 5 on the scaled problem from (x, y) (scaled
        variables, y in user row order) with step eta, primal weight omega and
        attempt count k (k >= 1).  Returns (accepted, x', y', etabar, eta')."""
        s = self.scaled(ruiz_iters)
        xn, yn = np.empty(self.n), np.empty(self.m)
        eb, en = C.c_double(0.0), C.c_double(0.0)
        acc = self.lib.orc_adaptive_attempt(s.h, omega, eta, k, _f64(x), self.to_internal_rows(y), xn, yn,
                                            C.byref(eb), C.byref(en))
        return bool(acc), xn, self.to_user_rows(yn), eb.value, en.value

    def unrolled(self, ruiz_iters, tau, sigma, c, q, l, u, x0, y0, K):
        """K fixed PDHG steps with inputs and outputs in original variables (q, y user order)."""
        s = self.scaled(ruiz_iters)
        xk = np.empty(self.n)
        yk = np.empty(self.m)
        self.lib.orc_unrolled(s.h, s.rho_i, s.kap, tau, sigma, _f64(c), self.to_internal_rows(q),
                              _f64(l), _f64(u), _f64(x0), self.to_internal_rows(y0), K, xk, yk)
        return xk, self.to_user_rows(yk)

    def unrolled_vjp(self, ruiz_iters, tau, sigma, c, q, l, u, x0, y0, K, gx, gy):
        """Reverse-mode derivative of ``unrolled``: dict of dL/d{c,q,l,u,x0,y0}."""
        s = self.scaled(ruiz_iters)
        n, m = self.n, self.m
        gc, gl, gu, gx0 = (np.empty(n) for _ in range(4))
        gq, gy0 = np.empty(m), np.empty(m)
        self.lib.orc_unrolled_vjp(s.h, s.rho_i, s.kap, tau, sigma, _f64(c), self.to_internal_rows(q),
                                  _f64(l), _f64(u), _f64(x0), self.to_internal_rows(y0), K, _f64(gx),
                                  self.to_internal_rows(gy), gc, gq, gl, gu, gx0, gy0)
        return dict(c=gc, q=self.to_user_rows(gq), l=gl, u=gu, x0=gx0, y0=self.to_user_rows(gy0))


class _Scaled:
    """Scaled problem K~ = diag(rho) K diag(kappa) owned by the oracle."""

    def __init__(self, o: Oracle, iters: int):
        self.lib = o.lib
        self.rho_i = np.empty(o.m)
        self.kap = np.empty(o.n)
        o.lib.orc_ruiz(o.h, iters, self.rho_i, self.kap)
        self.h = o.lib.orc_prob_scaled(o.h, self.rho_i, self.kap)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_prob_free(h)
            self.h = None


def _gather_rows(rowptr, perm):
    """Entry indices of rows ``perm`` concatenated (vectorised)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    if perm.shape[0] == 0:
        return np.zeros(0, dtype=np.int64)
    lens = rowptr[perm + 1] - rowptr[perm]
    starts = rowptr[perm]
    tot = int(lens.sum())
    out = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return out + np.arange(tot, dtype=np.int64)

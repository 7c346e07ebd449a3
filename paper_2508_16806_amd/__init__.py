"""MI355X-native restarted PDHG for linear programs (Python binding of libpdhg).

Solves  min c'x  s.t.  Gx >= h,  Ax = b,  l <= x <= u  (Section 2.2 of
arXiv 2508.16806) with restarted Primal-Dual Hybrid Gradient.  Every step of
the method runs in the hand-written gfx950 kernels of ``libpdhg.so``; this
module only marshals arguments through the C-ABI declared in
``include/pdhg.h`` (same call names), with PyTorch supplying the device
workspace and the stream.  There is no CPU fallback: a missing library or a
missing GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

__all__ = ["Solver", "autotune", "autotune_workspace_bytes", "read_mps", "write_mps", "MPSModel", "Opts", "lib", "LIB_PATH", "PDHGError", "STATUS", "SOL_RESULT", "SOL_CURRENT",
           "SOL_AVERAGE"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpdhg.so")

MEM_HOST, MEM_DEVICE = 0, 1
PREC_F64, PREC_F32 = 0, 1
SOL_RESULT, SOL_CURRENT, SOL_AVERAGE = 0, 1, 2
STATUS = {0: "OPTIMAL", 1: "ITERATION_LIMIT", 2: "TIME_LIMIT", 3: "NUMERICAL_ERROR", 4: "PRIMAL_INFEASIBLE",
          5: "DUAL_INFEASIBLE"}
ERR_NOMEM = -5
PDHG_ERR_STATE = -7
ERRORS = {-1: "INVALID_ARG", -2: "SHAPE", -3: "BOUNDS", -4: "NONFINITE", -5: "NOMEM", -6: "HIP",
          -7: "STATE"}


class PDHGError(RuntimeError):
    """A negative status of the C-ABI (code) with the library's message."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"PDHG_ERR_{ERRORS.get(code, code)}: {msg}")
        self.code = code


class LPDesc(C.Structure):
    """pdhg_lp: one LP in CSR form (pointers in memory space `mem`)."""

    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("c", C.c_void_p), ("rhs", C.c_void_p),
                ("l", C.c_void_p), ("u", C.c_void_p), ("row_type", C.c_void_p), ("mem", C.c_int32)]


class Opts(C.Structure):
    """pdhg_opts (field meanings in include/pdhg.h)."""

    _fields_ = [("precision", C.c_int32), ("ruiz_iters", C.c_int32), ("use_restarts", C.c_int32),
                ("use_pw_update", C.c_int32), ("check_every", C.c_int32),
                ("power_max_iters", C.c_int32), ("max_iters", C.c_int64), ("eps", C.c_double),
                ("time_limit", C.c_double), ("step_size", C.c_double), ("step_frac", C.c_double),
                ("primal_weight", C.c_double), ("power_tol", C.c_double), ("beta_suff", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double), ("eps_zero", C.c_double),
                ("unroll_capacity", C.c_int32), ("unroll_checkpoint", C.c_int32),
                ("use_graph", C.c_int32), ("xcd_remap", C.c_int32), ("bin_len_dual", C.c_int32 * 8),
                ("bin_len_primal", C.c_int32 * 8), ("bin_rows_dual", C.c_int32 * 8),
                ("bin_rows_primal", C.c_int32 * 8), ("max_grid", C.c_int32), ("adaptive_step", C.c_int32),
                ("detect_infeas", C.c_int32), ("infeas_tol", C.c_double), ("fishnet_points", C.c_int32),
                ("batch_resident_bytes", C.c_int64), ("trace_capacity", C.c_int32), ("col_slices", C.c_int32),
                ("col_slices_t", C.c_int32)]


class TraceRec(C.Structure):
    """pdhg_trace_rec: one check of pdhg_solve."""

    _fields_ = [("iter", C.c_int64), ("restarted", C.c_int32), ("cand_avg", C.c_int32), ("kkt_cand", C.c_double),
                ("omega", C.c_double), ("rel_kkt_cur", C.c_double), ("rel_kkt_avg", C.c_double),
                ("eta_next", C.c_double), ("accepted", C.c_int64), ("t_inner", C.c_int64),
                ("kkt0", C.c_double), ("kkt_prev", C.c_double), ("omega_before", C.c_double),
                ("delta_x", C.c_double), ("delta_y", C.c_double), ("kkt0_next", C.c_double),
                ("cand_pres", C.c_double), ("cand_dres", C.c_double), ("cand_gap", C.c_double)]


class KKTOut(C.Structure):
    """pdhg_kkt_out: relative KKT terms on the original LP."""

    _fields_ = [(k, C.c_double) for k in
                ("pres", "dres", "pobj", "dobj", "gap", "rel_pres", "rel_dres", "rel_gap", "rel_kkt")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Result(C.Structure):
    """pdhg_result: status and counters of one instance's solve."""

    _fields_ = [("status", C.c_int32), ("from_avg", C.c_int32), ("iters", C.c_int64),
                ("restarts", C.c_int32), ("power_iters", C.c_int32), ("knorm", C.c_double),
                ("eta", C.c_double), ("omega0", C.c_double), ("omega", C.c_double),
                ("tau", C.c_double), ("sigma", C.c_double), ("kkt", KKTOut), ("seconds", C.c_double),
                ("accepted", C.c_int64), ("eta_next", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "kkt"}
        d["kkt"] = self.kkt.as_dict()
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class KernelTimes(C.Structure):
    """pdhg_kernel_times: average device ms per launch of each phase."""

    _fields_ = [("ms_primal", C.c_double), ("ms_dual", C.c_double), ("ms_check", C.c_double),
                ("ms_control", C.c_double), ("ms_restart", C.c_double), ("reps", C.c_int32),
                ("ms_primal_ad", C.c_double), ("ms_dual_ad", C.c_double), ("ms_step_ad", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    """pdhg_info: sizes, step parameters, layout and setup phases."""

    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("m_ineq", C.c_int64), ("nnz", C.c_int64),
                ("knorm", C.c_double), ("eta", C.c_double), ("omega", C.c_double), ("tau", C.c_double),
                ("sigma", C.c_double), ("setup_seconds", C.c_double), ("precision", C.c_int32),
                ("batch", C.c_int32), ("workspace_bytes", C.c_int64), ("nseg_primal", C.c_int32),
                ("nseg_dual", C.c_int32), ("nblk_primal", C.c_int64), ("nblk_dual", C.c_int64),
                ("setup_plan_seconds", C.c_double), ("setup_host_seconds", C.c_double),
                ("setup_copy_seconds", C.c_double), ("setup_device_seconds", C.c_double),
                ("setup_power_seconds", C.c_double), ("power_iters_max", C.c_int32),
                ("record_valid", C.c_int32), ("record_generation", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["pdhg_default_opts", "pdhg_workspace_bytes", "pdhg_setup", "pdhg_iterate", "pdhg_solve",
           "pdhg_get_solution", "pdhg_set_state", "pdhg_kkt", "pdhg_backward", "pdhg_get_scaling",
           "pdhg_get_info", "pdhg_time_kernels", "pdhg_set_opts", "pdhg_set_data",
           "pdhg_destroy", "pdhg_last_error", "pdhg_fishnet", "pdhg_fishnet_rounds", "pdhg_autotune",
           "pdhg_get_trace", "pdhg_last_error_code", "pdhg_setup_noalloc"]

_lib = None


def lib():
    """The loaded libpdhg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, S = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
        L.pdhg_default_opts.argtypes = [C.POINTER(Opts)]
        L.pdhg_workspace_bytes.restype = C.c_size_t
        L.pdhg_workspace_bytes.argtypes = [P, I32, C.POINTER(Opts)]
        L.pdhg_setup.argtypes = [P, I32, C.POINTER(Opts), P, C.c_size_t, S, C.POINTER(P)]
        L.pdhg_setup_noalloc.argtypes = [P, I32, C.POINTER(Opts), S, C.POINTER(P)]
        L.pdhg_iterate.argtypes = [P, I64, I32, S]
        L.pdhg_solve.argtypes = [P, P, S]
        L.pdhg_get_solution.argtypes = [P, I32, I32, P, P, P, I32, S]
        L.pdhg_set_state.argtypes = [P, I32, P, P, I32, S]
        L.pdhg_kkt.argtypes = [P, I32, P, P, I32, C.POINTER(KKTOut), S]
        L.pdhg_backward.argtypes = [P, P, P, P, P, P, P, P, P, I32, S]
        L.pdhg_get_scaling.argtypes = [P, I32, P, P, I32, S]
        L.pdhg_get_info.argtypes = [P, C.POINTER(Info)]
        L.pdhg_set_opts.argtypes = [P, C.POINTER(Opts)]
        L.pdhg_set_data.argtypes = [P, P, P, P, P, I32, S]
        L.pdhg_time_kernels.argtypes = [P, I32, C.POINTER(KernelTimes), S]
        L.pdhg_fishnet.argtypes = [P, I32, I32, P, P, I64, I32, P, P, S]
        L.pdhg_fishnet_rounds.argtypes = [I32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.pdhg_autotune.argtypes = [P, I32, C.POINTER(Opts), P, C.c_size_t, C.POINTER(C.c_size_t), I32, S,
                                    C.POINTER(Opts), C.c_char_p]
        L.pdhg_get_trace.argtypes = [P, I32, P, I32, C.POINTER(C.c_int64), S]
        L.pdhg_destroy.argtypes = [P]
        L.pdhg_last_error.restype = C.c_char_p
        L.pdhg_last_error_code.restype = C.c_int32
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise PDHGError(rc, lib().pdhg_last_error().decode())


def default_opts(**kw) -> Opts:
    """pdhg_default_opts with the given fields replaced (precision may be "f32" / "f64")."""
    o = Opts()
    lib().pdhg_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"f32": PREC_F32, "f64": PREC_F64}[v]
        if k in ("bin_len_dual", "bin_len_primal", "bin_rows_dual", "bin_rows_primal"):
            setattr(o, k, (C.c_int32 * 8)(*v))
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def _is_torch_cuda(a) -> bool:
    return hasattr(a, "is_cuda") and a.is_cuda


def _stream(stream=None):
    import torch

    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class _Desc:
    """Keeps the arrays of one LP alive and builds its pdhg_lp descriptor."""

    def __init__(self, lp):
        dev = _is_torch_cuda(lp.val)
        if dev:
            import torch

            conv = {"rowptr": torch.int64, "col": torch.int32, "val": torch.float64, "rhs": torch.float64,
                    "c": torch.float64, "l": torch.float64, "u": torch.float64, "row_type": torch.uint8}
            self.a = {k: getattr(lp, k).to(dtype=t).contiguous() for k, t in conv.items()
                      if getattr(lp, k, None) is not None}
        else:
            conv = {"rowptr": np.int64, "col": np.int32, "val": np.float64, "rhs": np.float64,
                    "c": np.float64, "l": np.float64, "u": np.float64, "row_type": np.uint8}
            self.a = {k: np.ascontiguousarray(getattr(lp, k), dtype=t) for k, t in conv.items()
                      if getattr(lp, k, None) is not None}
        a = self.a
        self.desc = LPDesc(int(lp.n), int(lp.m), int(a["rowptr"][-1]), _ptr(a["rowptr"]), _ptr(a["col"]),
                           _ptr(a["val"]), _ptr(a["c"]), _ptr(a["rhs"]), _ptr(a["l"]), _ptr(a["u"]),
                           _ptr(a.get("row_type")), MEM_DEVICE if dev else MEM_HOST)


def autotune_workspace_bytes(lps, opts: Optional[Opts] = None, **kw) -> int:
    """Workspace pdhg_autotune needs for these LPs (host-side planning only)."""
    L = lib()
    if not isinstance(lps, (list, tuple)):
        lps = [lps]
    o = opts if opts is not None else default_opts(**kw)
    descs = [_Desc(lp) for lp in lps]
    arr = (LPDesc * len(lps))(*[d.desc for d in descs])
    need = C.c_size_t(0)
    best = Opts()
    rc = L.pdhg_autotune(C.cast(arr, C.c_void_p), len(lps), C.byref(o), None, 0, C.byref(need), 1, None,
                         C.byref(best), None)
    if rc != ERR_NOMEM:
        raise PDHGError(rc, L.pdhg_last_error().decode())
    return int(need.value)


def autotune(lps, reps: int = 20, out_json: Optional[str] = None, device: str = "cuda", stream=None,
             opts: Optional[Opts] = None, **kw):
    """Runs the library's launch-layout autotuner (pdhg_autotune) on ``lps``.

    Returns (best options, the tuner's JSON record as a dict).  Options other
    than the bins, rows per lane group, XCD remap and grid cap come from
    ``opts`` / ``kw``.
    """
    import json
    import tempfile

    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("libpdhg needs an AMD GPU; torch.cuda.is_available() is False")
    L = lib()
    if not isinstance(lps, (list, tuple)):
        lps = [lps]
    o = opts if opts is not None else default_opts(**kw)
    need = autotune_workspace_bytes(lps, o)
    descs = [_Desc(lp) for lp in lps]
    arr = (LPDesc * len(lps))(*[d.desc for d in descs])
    dev = torch.device(device)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    best = Opts()
    got = C.c_size_t(0)
    with tempfile.TemporaryDirectory() as td:
        path = out_json or os.path.join(td, "tune.json")
        with torch.cuda.device(dev):
            _check(L.pdhg_autotune(C.cast(arr, C.c_void_p), len(lps), C.byref(o), ws.data_ptr(), need,
                                   C.byref(got), int(reps), _stream(stream), C.byref(best), path.encode()))
        with open(path) as f:
            rec = json.load(f)
    del ws, descs
    return best, rec


class Solver:
    """One handle over ``batch`` LPs resident in a torch-allocated workspace.

    ``lps`` is one LP or a sequence of LPs; an LP is any object with fields
    n, m, rowptr, col, val, row_type, rhs, c, l, u (NumPy arrays, or CUDA torch
    tensors for device-resident input).  ``noalloc=True`` sets up through
    pdhg_setup_noalloc instead: no workspace tensor, the library's fixed
    per-device array (one such handle per device at a time).
    """

    def __init__(self, lps, device: str = "cuda", opts: Optional[Opts] = None, stream=None,
                 noalloc: bool = False, **kw):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libpdhg needs an AMD GPU; torch.cuda.is_available() is False")
        L = lib()
        if not isinstance(lps, (list, tuple)):
            lps = [lps]
        self.batch = len(lps)
        self.opts = opts if opts is not None else default_opts(**kw)
        descs = [_Desc(lp) for lp in lps]
        arr = (LPDesc * self.batch)(*[d.desc for d in descs])
        self.sizes = [(int(lp.n), int(lp.m)) for lp in lps]
        self.device = torch.device(device)
        h = C.c_void_p()
        if noalloc:
            self.ws = None
            with torch.cuda.device(self.device):
                _check(L.pdhg_setup_noalloc(C.cast(arr, C.c_void_p), self.batch, C.byref(self.opts),
                                            _stream(stream), C.byref(h)))
            self.h = h
            del descs
            return
        nbytes = L.pdhg_workspace_bytes(C.cast(arr, C.c_void_p), self.batch, C.byref(self.opts))
        if nbytes == 0:
            raise PDHGError(L.pdhg_last_error_code(), L.pdhg_last_error().decode())
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(L.pdhg_setup(C.cast(arr, C.c_void_p), self.batch, C.byref(self.opts), self.ws.data_ptr(),
                                int(nbytes), _stream(stream), C.byref(h)))
        self.h = h
        del descs

    def close(self):
        """pdhg_destroy (the workspace tensor is freed with the object)."""
        if getattr(self, "h", None) and self.h.value:
            lib().pdhg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ calls
    def set_opts(self, **kw):
        """Change run-time options (eps, max_iters, time_limit, restarts, ...)."""
        for k, v in kw.items():
            if not hasattr(self.opts, k):
                raise TypeError(f"unknown option {k}")
            setattr(self.opts, k, v)
        _check(lib().pdhg_set_opts(self.h, C.byref(self.opts)))

    def solve(self, stream=None) -> list:
        """pdhg_solve: one result dict per instance."""
        res = (Result * self.batch)()
        _check(lib().pdhg_solve(self.h, C.cast(res, C.c_void_p), _stream(stream)))
        return [r.as_dict() for r in res]

    def iterate(self, k: int, record: bool = False, stream=None):
        """pdhg_iterate: k fixed steps (recorded for backward when record)."""
        _check(lib().pdhg_iterate(self.h, int(k), int(bool(record)), _stream(stream)))

    def solution(self, inst: int = 0, which: int = SOL_RESULT, lam: bool = False, stream=None):
        """(x, y, lambda) in original variables as float64 NumPy arrays."""
        n, m = self.sizes[inst]
        x = np.empty(n)
        y = np.empty(m)
        la = np.empty(n) if lam else None
        _check(lib().pdhg_get_solution(self.h, inst, which, x.ctypes.data, y.ctypes.data,
                                       la.ctypes.data if lam else None, MEM_HOST, _stream(stream)))
        return (x, y, la) if lam else (x, y)

    def set_state(self, x, y, inst: int = 0, stream=None):
        """pdhg_set_state: the iterate of instance inst, original variables."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        _check(lib().pdhg_set_state(self.h, inst, x.ctypes.data, y.ctypes.data, MEM_HOST, _stream(stream)))

    def set_data(self, c=None, rhs=None, l=None, u=None, stream=None):
        """New cost / right-hand side / bounds (concatenated over the batch)."""
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (c, rhs, l, u)]
        ptrs = [None if a is None else a.ctypes.data for a in arrs]
        _check(lib().pdhg_set_data(self.h, *ptrs, MEM_HOST, _stream(stream)))

    def kkt(self, x, y, inst: int = 0, stream=None) -> dict:
        """pdhg_kkt: FP64 relative KKT terms of a caller point (host arrays or CUDA tensors)."""
        if _is_torch_cuda(x):
            xp, yp, mem = x.data_ptr(), y.data_ptr(), MEM_DEVICE
        else:
            x = np.ascontiguousarray(x, dtype=np.float64)
            y = np.ascontiguousarray(y, dtype=np.float64)
            xp, yp, mem = x.ctypes.data, y.ctypes.data, MEM_HOST
        out = KKTOut()
        _check(lib().pdhg_kkt(self.h, inst, xp, yp, mem, C.byref(out), _stream(stream)))
        return out.as_dict()

    def backward(self, gx, gy, stream=None) -> dict:
        """Adjoint of the last recorded ``iterate`` (whole batch, concatenated)."""
        nt = sum(n for n, _ in self.sizes)
        mt = sum(m for _, m in self.sizes)
        gx = np.ascontiguousarray(gx, dtype=np.float64)
        gy = np.ascontiguousarray(gy, dtype=np.float64)
        out = {k: np.empty(nt) for k in ("c", "l", "u", "x0")}
        out["rhs"] = np.empty(mt)
        out["y0"] = np.empty(mt)
        _check(lib().pdhg_backward(self.h, gx.ctypes.data, gy.ctypes.data, out["c"].ctypes.data,
                                   out["rhs"].ctypes.data, out["l"].ctypes.data, out["u"].ctypes.data,
                                   out["x0"].ctypes.data, out["y0"].ctypes.data, MEM_HOST, _stream(stream)))
        return out

    def scaling(self, inst: int = 0, stream=None):
        """Ruiz factors (rho in caller row order, kappa)."""
        n, m = self.sizes[inst]
        rho, kap = np.empty(m), np.empty(n)
        _check(lib().pdhg_get_scaling(self.h, inst, rho.ctypes.data, kap.ctypes.data, MEM_HOST,
                                      _stream(stream)))
        return rho, kap

    def fishnet(self, npoints: int = 32, k: int = 64, G=None, wraw=None, seed: int = 0, stream=None) -> dict:
        """Fishnet casting (Algorithm 7) on a one-LP handle; the surviving point
        becomes the current iterate.  G (npoints x n) and wraw are standard
        normal draws; when omitted they are drawn from numpy's PCG64 with
        `seed`.  Returns {"rounds", "gaps" (rounds x npoints), "keep"}."""
        r, nd = C.c_int32(0), C.c_int64(0)
        _check(lib().pdhg_fishnet_rounds(int(npoints), C.byref(r), C.byref(nd)))
        n = self.sizes[0][0]
        if G is None or wraw is None:
            rng = np.random.default_rng(seed)
            G = rng.standard_normal((npoints, n)) if G is None else G
            wraw = rng.standard_normal(npoints * npoints) if wraw is None else wraw
        G = np.ascontiguousarray(G, dtype=np.float64).reshape(-1)
        wraw = np.ascontiguousarray(wraw, dtype=np.float64).reshape(-1)
        if G.size != npoints * n:
            raise ValueError(f"G must hold {npoints} x {n} draws")
        gaps = np.zeros((r.value, npoints))
        keep = np.zeros((r.value, npoints), dtype=np.int32)
        _check(lib().pdhg_fishnet(self.h, int(npoints), int(k), G.ctypes.data, wraw.ctypes.data, wraw.size,
                                  MEM_HOST, gaps.ctypes.data, keep.ctypes.data, _stream(stream)))
        return {"rounds": r.value, "gaps": gaps, "keep": keep}

    def time_kernels(self, reps: int = 20, stream=None) -> dict:
        """Average per-launch device time of each phase kernel (ms), from HIP events; the
        sweeps are timed alternately, as the iteration runs them (1 <= reps <= 10000)."""
        t = KernelTimes()
        _check(lib().pdhg_time_kernels(self.h, int(reps), C.byref(t), _stream(stream)))
        return t.as_dict()

    def trace(self, inst: int = 0, stream=None):
        """(check records of the last solve, oldest first, as dicts; total checks)."""
        cap = int(self.opts.trace_capacity)
        recs = (TraceRec * max(cap, 1))()
        total = C.c_int64(0)
        _check(lib().pdhg_get_trace(self.h, inst, C.cast(recs, C.c_void_p), cap, C.byref(total), _stream(stream)))
        n = min(cap, total.value)
        return [{k: getattr(r, k) for k, _ in TraceRec._fields_} for r in recs[:n]], int(total.value)

    def info(self) -> dict:
        """pdhg_get_info as a dict."""
        i = Info()
        _check(lib().pdhg_get_info(self.h, C.byref(i)))
        return i.as_dict()


from .mps import MPSModel, parse_mps, read_mps, write_mps  # noqa: E402

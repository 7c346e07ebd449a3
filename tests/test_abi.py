"""CPU-side checks of the C-ABI library: it loads, exports every function the
public header declares, and rejects invalid LPs before any GPU work (the
validation in pdhg_workspace_bytes runs on the host only)."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import lpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pd():
    import paper_2508_16806_amd as pd
    from paper_2508_16806_amd import build as hb

    if hb.stale():
        hb.build()
    return pd


def _declared():
    src = open(os.path.join(ROOT, "include", "pdhg.h")).read()
    return sorted(set(re.findall(r"\b(pdhg_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(pd):
    L = pd.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pd.EXPORTS)


def test_struct_layouts_match_header(pd):
    """ctypes mirrors of the C structs have the sizes the library was built with."""
    L = pd.lib()
    o = pd.default_opts()
    assert o.precision == 1 and o.ruiz_iters == 10 and o.check_every == 64
    assert o.eps == 1e-4 and o.step_frac == 0.9 and o.beta_art == 0.36
    assert o.adaptive_step == 0 and o.max_grid == 8192
    # the option struct ends with the detection fields; the result and timer structs
    # end with the adaptive-step fields
    assert pd.Opts.fishnet_points.offset == pd.Opts.infeas_tol.offset + 8
    assert o.fishnet_points == 0
    assert pd.Opts.batch_resident_bytes.offset == pd.Opts.fishnet_points.offset + 8
    assert o.batch_resident_bytes == 192_000_000
    assert pd.Opts.trace_capacity.offset == pd.Opts.batch_resident_bytes.offset + 8 and o.trace_capacity == 0
    assert pd.Opts.col_slices.offset == pd.Opts.trace_capacity.offset + 4 and o.col_slices == 0
    assert pd.Opts.col_slices_t.offset == pd.Opts.col_slices.offset + 4 and o.col_slices_t == 0
    assert C.sizeof(pd.Opts) == (pd.Opts.col_slices_t.offset + 4 + 7) // 8 * 8  # padded to 8-byte alignment
    assert C.sizeof(pd.TraceRec) == 144
    assert o.detect_infeas == 0 and o.infeas_tol == 1e-4
    assert pd.Result.eta_next.offset + 8 == C.sizeof(pd.Result)
    assert pd.KernelTimes.ms_step_ad.offset + 8 == C.sizeof(pd.KernelTimes)
    assert L.pdhg_last_error() is not None


_LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "pdhg.h"
#define S(T) printf(#T " size %zu\n", sizeof(T));
#define F(T, f) printf(#T " %s %zu\n", #f, offsetof(T, f));
int main(void) {
    S(pdhg_opts) S(pdhg_result) S(pdhg_trace_rec) S(pdhg_info) S(pdhg_kernel_times) S(pdhg_kkt_out) S(pdhg_lp)
    F(pdhg_trace_rec, t_inner) F(pdhg_trace_rec, kkt0) F(pdhg_trace_rec, cand_gap)
    F(pdhg_info, power_iters_max) F(pdhg_info, record_valid) F(pdhg_info, record_generation)
    F(pdhg_opts, trace_capacity) F(pdhg_opts, col_slices) F(pdhg_opts, col_slices_t)
    F(pdhg_result, eta_next)
    printf("noalloc %llu\n", (unsigned long long)PDHG_NOALLOC_MAX_BYTES);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_mirrors_match_the_c_header(pd, tmp_path):
    """Sizes and field offsets of the binding's ctypes structs equal what a C
    compiler makes of include/pdhg.h."""
    src = tmp_path / "layout.c"
    src.write_text(_LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        parts = line.split()
        got[" ".join(parts[:-1])] = int(parts[-1])
    mirrors = {"pdhg_opts": pd.Opts, "pdhg_result": pd.Result, "pdhg_trace_rec": pd.TraceRec,
               "pdhg_info": pd.Info, "pdhg_kernel_times": pd.KernelTimes, "pdhg_kkt_out": pd.KKTOut,
               "pdhg_lp": pd.LPDesc}
    for name, cls in mirrors.items():
        assert got[f"{name} size"] == C.sizeof(cls), name
    for key, off in got.items():
        parts = key.split()
        if len(parts) == 2 and parts[1] != "size" and parts[0] in mirrors:
            assert getattr(mirrors[parts[0]], parts[1]).offset == off, key
    assert got["noalloc"] == 64 << 20


def _nbytes(pd, lp, **kw):
    d = pd._Desc(lp)
    arr = (pd.LPDesc * 1)(d.desc)
    return pd.lib().pdhg_workspace_bytes(C.cast(arr, C.c_void_p), 1, C.byref(pd.default_opts(**kw)))


def test_workspace_bytes_positive_and_monotone(pd):
    small = _nbytes(pd, lpgen.config0(0))
    big = _nbytes(pd, lpgen.planted(400, 1000, 0.02, 1))
    assert 0 < small < big
    assert _nbytes(pd, lpgen.config0(0), precision="f64") > 0
    with_unroll = _nbytes(pd, lpgen.config0(0), unroll_capacity=100, unroll_checkpoint=10)
    assert with_unroll > small


def _err(pd):
    return pd.lib().pdhg_last_error().decode()


def test_rejects_bad_shapes(pd):
    lp = lpgen.config0(0)
    bad = lpgen.LP(**{**lp.__dict__})
    bad.col = lp.col.copy()
    bad.col[5] = lp.n + 3
    assert _nbytes(pd, bad) == 0 and "out of range" in _err(pd)
    bad = lpgen.LP(**{**lp.__dict__})
    bad.rowptr = lp.rowptr.copy()
    bad.rowptr[10], bad.rowptr[11] = bad.rowptr[11] + 1, bad.rowptr[10]
    assert _nbytes(pd, bad) == 0 and "monotone" in _err(pd)


def test_rejects_bounds_and_nonfinite(pd):
    lp = lpgen.config0(0)
    bad = lpgen.LP(**{**lp.__dict__})
    bad.l = lp.l.copy()
    bad.l[3] = lp.u[3] + 1.0
    assert _nbytes(pd, bad) == 0 and "bounds" in _err(pd)
    bad = lpgen.LP(**{**lp.__dict__})
    bad.c = lp.c.copy()
    bad.c[7] = np.nan
    assert _nbytes(pd, bad) == 0 and "not finite" in _err(pd)
    bad = lpgen.LP(**{**lp.__dict__})
    bad.val = lp.val.copy()
    bad.val[0] = np.inf
    assert _nbytes(pd, bad) == 0 and "not finite" in _err(pd)
    bad = lpgen.LP(**{**lp.__dict__})
    bad.rhs = lp.rhs.copy()
    bad.rhs[1] = -np.inf
    assert _nbytes(pd, bad) == 0 and "not finite" in _err(pd)
    bad = lpgen.LP(**{**lp.__dict__})
    bad.l = lp.l.copy()
    bad.l[0] = np.inf
    bad.u = lp.u.copy()
    bad.u[0] = np.inf
    assert _nbytes(pd, bad) == 0 and "bounds" in _err(pd)


def test_last_error_code(pd):
    """A sizing call that fails leaves its status code beside the message."""
    lp = lpgen.config0(0)
    bad = lpgen.config0(0)
    bad.val = bad.val.copy()
    bad.val[0] = np.nan
    assert _nbytes(pd, bad) == 0 and pd.lib().pdhg_last_error_code() == -4
    bad = lpgen.config0(0)
    bad.l = bad.l.copy()
    bad.l[0] = bad.u[0] + 1
    assert _nbytes(pd, bad) == 0 and pd.lib().pdhg_last_error_code() == -3
    assert _nbytes(pd, lp, check_every=0) == 0 and pd.lib().pdhg_last_error_code() == -1


def test_rejects_bad_options(pd):
    lp = lpgen.config0(0)
    assert _nbytes(pd, lp, check_every=0) == 0 and "check_every" in _err(pd)
    assert _nbytes(pd, lp, eps=0.0) == 0
    assert _nbytes(pd, lp, precision=7) == 0
    assert _nbytes(pd, lp, adaptive_step=2) == 0 and "adaptive_step" in _err(pd)
    assert _nbytes(pd, lp, adaptive_step=1) == _nbytes(pd, lp)
    assert _nbytes(pd, lp, detect_infeas=2) == 0 and "detect_infeas" in _err(pd)
    assert _nbytes(pd, lp, detect_infeas=1, infeas_tol=0.0) == 0 and "infeas_tol" in _err(pd)
    assert _nbytes(pd, lp, detect_infeas=1) == _nbytes(pd, lp)
    assert _nbytes(pd, lp, fishnet_points=3) == 0 and "fishnet_points" in _err(pd)
    assert _nbytes(pd, lp, fishnet_points=128) == 0
    assert _nbytes(pd, lp, fishnet_points=32) > _nbytes(pd, lp)
    assert _nbytes(pd, lp, batch_resident_bytes=-1) == 0 and "batch_resident_bytes" in _err(pd)
    assert _nbytes(pd, lp, bin_rows_dual=[3, 1, 1, 1, 1, 1, 1, 1]) == 0 and "bin_rows" in _err(pd)
    assert _nbytes(pd, lp, bin_rows_primal=[1, 1, 1, 1, 1, 2, 1, 1]) == 0
    assert _nbytes(pd, lp, bin_rows_primal=[4, 4, 2, 2, 1, 0, 0, 0]) > 0
    assert _nbytes(pd, lp, bin_len_dual=[-1, 8, 16, 32, 64, 128, 512, 0]) == 0 and "bin_len" in _err(pd)
    assert _nbytes(pd, lp, col_slices=17) == 0 and "col_slices" in _err(pd)
    assert _nbytes(pd, lp, col_slices=-1) == 0
    assert _nbytes(pd, lp, col_slices_t=17) == 0 and "col_slices" in _err(pd)
    assert _nbytes(pd, lp, col_slices_t=-1) == 0
    # slice starts (m x (S - 1) int32) and the partial products (m FP64); n
    # of each for the primal sweep
    assert _nbytes(pd, lp, col_slices=4) >= _nbytes(pd, lp) + lp.m * (3 * 4 + 8)
    assert _nbytes(pd, lp, col_slices_t=4) >= _nbytes(pd, lp) + lp.n * (3 * 4 + 8)
    assert _nbytes(pd, lp, trace_capacity=-1) == 0 and "trace_capacity" in _err(pd)
    assert _nbytes(pd, lp, trace_capacity=(1 << 20) + 1) == 0
    # the ring: one pdhg_trace_rec (144 bytes) per record and instance (within the carve's
    # 256-byte alignment)
    grow = _nbytes(pd, lp, trace_capacity=1000) - _nbytes(pd, lp)
    assert 144 * 1000 <= grow <= 144 * 1000 + 512


def test_fishnet_rounds_and_draws(pd):
    L = pd.lib()
    r, n = C.c_int32(0), C.c_int64(0)
    # 2^p points: 2p - 2 rounds (one for two points); the repopulating rounds
    # keep 2^(p-2), ..., 2 points and draw (kept)^2 weights each
    for P, rounds, draws in ((2, 1, 0), (4, 2, 0), (8, 4, 4), (16, 6, 20), (32, 8, 84), (64, 10, 340)):
        assert L.pdhg_fishnet_rounds(P, C.byref(r), C.byref(n)) == 0
        assert (r.value, n.value) == (rounds, draws), P
    assert L.pdhg_fishnet_rounds(6, C.byref(r), C.byref(n)) != 0


def test_infinite_bounds_accepted(pd):
    lp = lpgen.tiny(3, n=8, m=4, free_frac=0.5)
    assert np.isinf(lp.l).any()
    assert _nbytes(pd, lp) > 0


def test_autotune_workspace_covers_every_candidate(pd):
    """pdhg_autotune without a workspace fails with NOMEM and reports a size
    that holds every combination of limits, rows per group, launch shape and
    column slices its search can set up."""
    from paper_2508_16806_amd.tuner import limits

    for lp in (lpgen.config0(0), lpgen.config2(m=3000, n=6000)):
        need = pd.autotune_workspace_bytes(lp)
        assert need > 0 and need % 256 == 0
        cands = [limits(f, w) for f in (2, 4, 8, 16) for w in (512, 2048) if w >= 64 * f]
        worst = 0
        for lp_lim in cands:
            for ld_lim in cands:
                for rows in (1, 2, 4):
                    rr = [rows] * 5 + [1, 1, 1]
                    for S in (0, 2, 4, 8):
                        b = _nbytes(pd, lp, bin_len_primal=lp_lim, bin_len_dual=ld_lim, bin_rows_primal=rr,
                                    bin_rows_dual=rr, col_slices=S, col_slices_t=S)
                        assert b > 0
                        worst = max(worst, b)
        assert need >= worst
        # and it is a bound, not a gross overestimate
        assert need <= worst * 1.05


def test_autotune_rejects_bad_arguments(pd):
    L = pd.lib()
    d = pd._Desc(lpgen.config0(0))
    arr = (pd.LPDesc * 1)(d.desc)
    o, best, need = pd.default_opts(), pd.Opts(), C.c_size_t(7)
    assert L.pdhg_autotune(C.cast(arr, C.c_void_p), 1, C.byref(o), None, 0, C.byref(need), 0, None,
                           C.byref(best), None) == -1  # reps < 1
    assert L.pdhg_autotune(C.cast(arr, C.c_void_p), 0, C.byref(o), None, 0, C.byref(need), 1, None,
                           C.byref(best), None) == -1  # batch < 1
    bad = pd.default_opts(check_every=0)
    assert L.pdhg_autotune(C.cast(arr, C.c_void_p), 1, C.byref(bad), None, 0, C.byref(need), 1, None,
                           C.byref(best), None) == -1
    assert L.pdhg_autotune(C.cast(arr, C.c_void_p), 1, C.byref(o), None, 0, C.byref(need), 1, None,
                           C.byref(best), None) == -5
    assert need.value > 0 and "workspace" in _err(pd)

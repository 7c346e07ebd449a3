"""Autotuner for the row-length bins of the two fused sweeps.

After the bins it tunes the rows handled by one lane group (1, 2 or 4 in
the bins of at most 16 lanes) and the launch shape: XCD-contiguous workgroup
numbering on or off and the cap on workgroups per sweep launch.

A bin sweeps each row with a fixed number of lanes (1, 2, 4, ..., 64 lanes of
a wavefront, or a whole 256-lane workgroup).  The tuner tries bin limits

    limit_k = f * 2^k  (k = 0..5),   limit_6 = w,   bin 7 = rows longer than w

for a grid of elements-per-lane f and whole-workgroup thresholds w, times the
primal and the dual sweep of each candidate on the GPU with the library's
event timers (pdhg_time_kernels), and keeps the fastest limits for each
operator separately.  The result is a small JSON tuning file that Solver and
bench.py load (``tuning=``).

    python -m paper_2508_16806_amd.autotune --workload sced --out tuning.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def limits(f: int, w: int):
    lim = [f * (1 << k) for k in range(6)] + [max(w, 64 * f), 0]
    return lim


def autotune(lp, precision: str = "f32", factors=(2, 4, 8, 16), wg_thresholds=(512, 2048),
             grid_caps=(4096, 8192, 16384, 65536), reps: int = 20, verbose: bool = True) -> dict:
    import paper_2508_16806_amd as pd

    trials = []
    for f in factors:
        for w in wg_thresholds:
            if w < 64 * f:
                continue
            lim = limits(f, w)
            s = pd.Solver(lp, precision=precision, bin_len_dual=lim, bin_len_primal=lim)
            s.time_kernels(reps=3)  # warm caches and clocks
            t = s.time_kernels(reps=reps)
            trials.append({"f": f, "w": w, "limits": lim, "ms_primal": t["ms_primal"], "ms_dual": t["ms_dual"]})
            if verbose:
                print(f"[autotune] f={f} w={w}: primal {t['ms_primal']*1e3:.1f} us, dual "
                      f"{t['ms_dual']*1e3:.1f} us", file=sys.stderr, flush=True)
            s.close()
    bp = min(trials, key=lambda r: r["ms_primal"])
    bd = min(trials, key=lambda r: r["ms_dual"])
    # rows per lane group in the bins of at most 16 lanes
    rtrials = []
    for rows in (1, 2, 4):
        rr = [rows] * 5 + [1, 1, 1]
        s = pd.Solver(lp, precision=precision, bin_len_dual=bd["limits"], bin_len_primal=bp["limits"],
                      bin_rows_dual=rr, bin_rows_primal=rr)
        s.time_kernels(reps=3)
        t = s.time_kernels(reps=reps)
        rtrials.append({"rows": rr, "ms_primal": t["ms_primal"], "ms_dual": t["ms_dual"]})
        if verbose:
            print(f"[autotune] rows/group={rows}: primal {t['ms_primal']*1e3:.1f} us, dual "
                  f"{t['ms_dual']*1e3:.1f} us", file=sys.stderr, flush=True)
        s.close()
    rp_ = min(rtrials, key=lambda r: r["ms_primal"])["rows"]
    rd_ = min(rtrials, key=lambda r: r["ms_dual"])["rows"]
    # launch shape: XCD-contiguous numbering on/off, sweep grid cap
    shapes = []
    for remap in (0, 1):
        for grid in grid_caps:
            s = pd.Solver(lp, precision=precision, bin_len_dual=bd["limits"], bin_len_primal=bp["limits"],
                          bin_rows_dual=rd_, bin_rows_primal=rp_, xcd_remap=remap, max_grid=grid)
            s.time_kernels(reps=3)
            t = s.time_kernels(reps=reps)
            tot = t["ms_primal"] + t["ms_dual"] + t["ms_check"] / 64.0
            shapes.append({"xcd_remap": remap, "max_grid": grid, "ms_primal": t["ms_primal"],
                           "ms_dual": t["ms_dual"], "ms_check": t["ms_check"], "ms_iter": tot})
            if verbose:
                print(f"[autotune] remap={remap} grid={grid}: primal {t['ms_primal']*1e3:.1f} us, dual "
                      f"{t['ms_dual']*1e3:.1f} us, check {t['ms_check']*1e3:.1f} us", file=sys.stderr, flush=True)
            s.close()
    bs = min(shapes, key=lambda r: r["ms_iter"])
    return {"n": int(lp.n), "m": int(lp.m), "nnz": int(lp.nnz), "precision": precision,
            "bin_len_primal": bp["limits"], "bin_len_dual": bd["limits"],
            "bin_rows_primal": rp_, "bin_rows_dual": rd_, "rows_trials": rtrials,
            "xcd_remap": bs["xcd_remap"], "max_grid": bs["max_grid"],
            "ms_primal": bs["ms_primal"], "ms_dual": bs["ms_dual"], "trials": trials, "shapes": shapes,
            "time": time.strftime("%Y-%m-%d %H:%M:%S")}


def load(path: str) -> dict:
    with open(path) as f:
        t = json.load(f)
    out = {"bin_len_primal": t["bin_len_primal"], "bin_len_dual": t["bin_len_dual"]}
    for k in ("xcd_remap", "max_grid", "bin_rows_primal", "bin_rows_dual"):
        if k in t:
            out[k] = t[k]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="sced", choices=["sced", "sced_small", "zipf", "zipf_small"])
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import lpgen

    lp = {"sced": lambda: lpgen.config1(), "sced_small": lambda: lpgen.sced(500, 200, 24, 125, seed=1),
          "zipf": lambda: lpgen.config2(), "zipf_small": lambda: lpgen.config2(m=100000, n=200000)}[
        args.workload]()
    res = autotune(lp, precision=args.precision)
    res["workload"] = args.workload
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: res[k] for k in ("bin_len_primal", "bin_len_dual", "bin_rows_primal", "bin_rows_dual",
                                          "xcd_remap", "max_grid", "ms_primal", "ms_dual")}))


if __name__ == "__main__":
    main()

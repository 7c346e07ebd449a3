"""Command line and tuning files of the launch-layout autotuner.

The search runs inside the library (``pdhg_autotune`` in ``include/pdhg.h``,
reached through ``paper_2508_16806_amd.autotune()``): it times the primal and
the dual sweep of candidate row-length bins

    limit_k = f * 2^k  (k = 0..5),   limit_6 = w,   bin 7 = rows longer than w

for f in {2, 4, 8, 16} and w in {512, 2048}, keeps the fastest limits for each
operator, then the rows handled by one lane group (1, 2 or 4 in the bins of at
most 16 lanes) and the launch shape (XCD-contiguous workgroup numbering on or
off, cap on workgroups per sweep launch), and last the column slices of the
two sweeps (none, or 2, 4 or 8 with every bin candidate for the dual sweep;
kept where they beat the unsliced sweep by 2%).  This module writes the result as a small JSON
tuning file that Solver and bench.py load (``tuning=``).

    python -m paper_2508_16806_amd.tuner --workload sced --out tuning.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def limits(f: int, w: int):
    """Bin limits of the candidate (f, w), as the library builds them."""
    return [f * (1 << k) for k in range(6)] + [max(w, 64 * f), 0]


def autotune(lp, precision: str = "f32", reps: int = 20, verbose: bool = True) -> dict:
    """Tunes the launch layout of ``lp`` (one LP or a batch) on the GPU."""
    import paper_2508_16806_amd as pd

    t0 = time.time()
    best, rec = pd.autotune(lp, reps=reps, precision=precision)
    lps = lp if isinstance(lp, (list, tuple)) else [lp]
    rec.update({"n": sum(int(p.n) for p in lps), "m": sum(int(p.m) for p in lps),
                "nnz": sum(int(p.rowptr[-1]) for p in lps), "batch": len(lps), "precision": precision,
                "tune_seconds": time.time() - t0, "time": time.strftime("%Y-%m-%d %H:%M:%S")})
    if verbose:
        for t in rec["trials"]:
            print(f"[autotune] f={t['f']} w={t['w']}: primal {t['ms_primal']*1e3:.1f} us, dual "
                  f"{t['ms_dual']*1e3:.1f} us", file=sys.stderr, flush=True)
        for t in rec["rows_trials"]:
            print(f"[autotune] rows/group={t['rows']}: primal {t['ms_primal']*1e3:.1f} us, dual "
                  f"{t['ms_dual']*1e3:.1f} us", file=sys.stderr, flush=True)
        for t in rec["shapes"]:
            print(f"[autotune] remap={t['xcd_remap']} grid={t['max_grid']}: primal {t['ms_primal']*1e3:.1f} us, "
                  f"dual {t['ms_dual']*1e3:.1f} us, check {t['ms_check']*1e3:.1f} us", file=sys.stderr, flush=True)
        for t in rec.get("slice_trials", []):
            print(f"[autotune] col_slices={t['col_slices']} f={t['f']} w={t['w']}: primal "
                  f"{t['ms_primal']*1e3:.1f} us, dual {t['ms_dual']*1e3:.1f} us", file=sys.stderr, flush=True)
    return rec


def load(path: str) -> dict:
    with open(path) as f:
        t = json.load(f)
    out = {"bin_len_primal": t["bin_len_primal"], "bin_len_dual": t["bin_len_dual"]}
    for k in ("xcd_remap", "max_grid", "bin_rows_primal", "bin_rows_dual", "col_slices", "col_slices_t"):
        if k in t:
            out[k] = t[k]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="sced",
                    choices=["sced", "sced_small", "sced_tenth64", "zipf", "zipf_small", "planted16"])
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import lpgen

    # planted16: the first 16 planted LPs of the batched workload (m ~ U{1000..50000}, n = 2.5m,
    # density U(0.1%, 1%)), tuned as one batch
    # sced_tenth64: the differentiation workload's batch of 64 SCED-shaped LPs at 1/10 size
    lp = {"sced": lambda: lpgen.config1(), "sced_small": lambda: lpgen.sced(500, 200, 24, 125, seed=1),
          "sced_tenth64": lambda: [lpgen.config4_instance(i) for i in range(64)],
          "zipf": lambda: lpgen.config2(), "zipf_small": lambda: lpgen.config2(m=100000, n=200000),
          "planted16": lambda: [lpgen.config3_instance(i) for i in range(16)]}[args.workload]()
    res = autotune(lp, precision=args.precision, reps=args.reps)
    res["workload"] = args.workload
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: res[k] for k in ("bin_len_primal", "bin_len_dual", "bin_rows_primal", "bin_rows_dual",
                                          "xcd_remap", "max_grid", "col_slices", "col_slices_t", "ms_primal",
                                          "ms_dual")}))


if __name__ == "__main__":
    main()

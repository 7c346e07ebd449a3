"""Benchmark of the PDHG hot path on one MI355X.

Workload: the SCED-shaped synthetic LP (5000 generators, 2000 buses, 24
periods, 125 lines: n = 418,048 variables, m = 298,072 rows, ~15.25M
nonzeros), FP32 iterates and matrix with FP64 accumulation, FP64 KKT check,
restart test and primal-weight update.  Inputs are seeded and synthetic and
are resident in HBM before any timed region.

One step = one chunk of the restarted method: 64 PDHG iterations (fused K~^T y
sweep + primal update and K~ xbar sweep + dual update, with the epoch
averages), the FP64 KKT check of the iterate and of the average, the
per-instance restart / primal-weight / termination decision, and the restart
copy -- one launch of the captured hipGraph.  value = PDHG iterations per
second over the K timed steps.

Also reported: per-kernel device times (HIP events, live), the roofline of the
dominant sweep from its algorithmic bytes, the time to a relative KKT error of
1e-4 from a cold start, and the FP64 CPU oracle timed on the host on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time to 1e-4 rel KKT; PDHG iter/s; HBM GB/s vs peak; batched vs 1-by-1 LPs/s"
KERNEL_SOURCES = ["paper_2508_16806_amd/csrc/kernels.hip", "paper_2508_16806_amd/csrc/sweep.h",
                  "paper_2508_16806_amd/csrc/pdhg_internal.h"]
TRAFFIC_FILE = "profiles/c1_sced_hbm_traffic.json"


def kernel_src_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_FILE)) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_src_sha") != kernel_src_hash() or kernel not in t.get("per_launch_bytes", {}):
        return None
    return t["per_launch_bytes"][kernel]
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def sweep_bytes(info, es=4):
    """Algorithmic HBM bytes of one launch of each fused sweep.

    primal (rows of K~^T): values + columns (es + 4) per nonzero, int64 row
    pointers (8 per row), one read of the gathered y (es per dual entry), and
    per variable: x read+write, xbar write, xavg read+write, c~, l~, u~ reads.
    dual (rows of K~): values + columns per nonzero, row pointers, one read of
    the gathered xbar, and per row: y read+write, yavg read+write, q~ read.
    """
    n, m, nnz = info["n"], info["m"], info["nnz"]
    primal = nnz * (es + 4) + 8 * (n + 1) + es * m + es * 8 * n
    dual = nnz * (es + 4) + 8 * (m + 1) + es * n + es * 5 * m
    return primal, dual


def sweep_bytes_ad(info, es=4):
    """Algorithmic HBM bytes of one launch of each adaptive-step sweep.

    primal: as the fixed sweep without the xbar write (x read, x' write,
    xavg read+write, c~, l~, u~: 7 per variable).  dual: values + columns,
    row pointers, one read of the gathered x', and per row y read, y' write,
    yavg read+write, q~ read, plus the FP64 K~x read and K~x' write.
    """
    n, m, nnz = info["n"], info["m"], info["nnz"]
    primal = nnz * (es + 4) + 8 * (n + 1) + es * m + es * 7 * n
    dual = nnz * (es + 4) + 8 * (m + 1) + es * n + es * 5 * m + 16 * m
    return primal, dual


def _oracle_rate(lp, budget_s):
    """FP64 CPU oracle iterations/s on this host: two restarted solves that
    differ only in their iteration limit; the rate is the difference of
    iterations over the difference of wall time, so setup cancels.  The
    extra iteration count is sized from a 3-step probe to take ~budget_s."""
    import numpy as np

    import oracle

    o = oracle.Oracle(lp)
    sc = o.scaled(10)
    x, y = np.zeros(lp.n), np.zeros(lp.m)
    t = time.perf_counter()
    o.lib.orc_steps(sc.h, 1e-3, 1e-3, x, y, 3)
    t_step = (time.perf_counter() - t) / 3
    del sc
    k = 64 * max(1, int(round(budget_s / (64 * t_step))))
    opts = oracle.SolveOpts(eps=1e-12, power_max_iters=20, max_iters=64)
    t0 = time.perf_counter()
    r1 = o.solve(opts)
    t1 = time.perf_counter()
    opts.max_iters = 64 + k
    r2 = o.solve(opts)
    t2 = time.perf_counter()
    rate = (r2.iters - r1.iters) / max((t2 - t1) - (t1 - t0), 1e-9)
    return rate, r1.iters, r2.iters


def _omp_threads():
    """Threads an OpenMP parallel region of this process uses."""
    import ctypes

    try:
        return int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_CORE = r"""
import json, sys
sys.path.insert(0, {root!r})
import bench, lpgen
lp = lpgen.sced(500, 200, 24, 125, seed=1) if {small} else lpgen.config1()
rate, i1, i2 = bench._oracle_rate(lp, {budget})
print(json.dumps({{"rate": rate, "i1": i1, "i2": i2}}))
"""


def _oracle_time_to_tol(lp, eps=1e-4):
    import oracle

    o = oracle.Oracle(lp)
    t = time.perf_counter()
    r = o.solve(oracle.SolveOpts(eps=eps, max_iters=400_000))
    return {"seconds": time.perf_counter() - t, "status": {0: "OPTIMAL", 1: "ITERATION_LIMIT"}.get(r.status, r.status),
            "iters": r.iters, "restarts": r.restarts, "rel_kkt": r.kkt["rel_kkt"]}


def oracle_leg(lp, points=None, small=False, budget_s=15.0, ttt_c1=True):
    """The benchmark's CPU leg: the FP64 oracle as it stands, on this host.

    cpu_baseline: its iteration rate on the same LP with every OpenMP thread
    of the process and, in a child process, on one thread; its time to a
    relative KKT error of 1e-4 from a cold start on C0 (and on C1 unless
    ttt_c1 is off), with the host's CPU model.  checks: the oracle's relative
    KKT error of each GPU point in ``points`` (name -> (x, y)) on the original
    LP, and its objective -- the checker side of the FP32 error report."""
    import subprocess

    import lpgen
    import oracle

    oracle.build(force=False)
    rate, i1, i2 = _oracle_rate(lp, budget_s)
    cpu = {"value": rate, "unit": "PDHG iter/s", "cores": _omp_threads(), "kind": "oracle",
           "sample": f"restarted FP64 oracle solve of the same LP: rate from the difference of two solves capped "
                     f"at {i1} and {i2} iterations (power iteration capped at 20 passes in both; setup cancels)",
           "cpu_model": _cpu_model()}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = _ONE_CORE.format(root=ROOT, small=bool(small), budget=max(budget_s / 2, 5.0))
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        one = json.loads(out.stdout.strip().splitlines()[-1])
        cpu["value_1core"] = one["rate"]
        cpu["sample_1core"] = f"the same two solves capped at {one['i1']} and {one['i2']} iterations, one thread"
    except Exception as e:  # noqa: BLE001 -- the one-core figure is optional
        cpu["value_1core"] = None
        cpu["sample_1core"] = f"not measured: {type(e).__name__}"
    ttt = {"C0": _oracle_time_to_tol(lpgen.config0(0))}
    if ttt_c1 and not small:
        ttt["C1"] = _oracle_time_to_tol(lp)
        ttt["C4[0]"] = _oracle_time_to_tol(lpgen.config4_instance(0))
    cpu["time_to_1e-4"] = ttt
    return cpu, oracle_checks(lp, points or {})


def oracle_checks(lp, points):
    """Part of the CPU leg: the oracle's relative KKT error and objective of
    each GPU point (name -> (x, y)) on the original LP."""
    import oracle

    out = {}
    if points:
        o = oracle.Oracle(lp)
        for name, (x, y) in points.items():
            k = o.kkt(x, y)
            out[name] = {"rel_kkt": k["rel_kkt"], "pobj": k["pobj"]}
    return out


def _gen_one(a):
    import lpgen

    i, m_max = a
    return lpgen.config3_instance(i, m_range=(1000, m_max))


def _gen_batched(B, m_max, stride=1):
    """The batch's instances (ids 0, stride, 2 stride, ...), generated by a
    pool of worker processes (each instance has its own seed, so the result
    does not depend on the pool)."""
    import multiprocessing as mp

    workers = max(1, min(16, (os.cpu_count() or 1), B))
    out = []
    # spawned workers: they share no state with this process (no GPU context)
    with mp.get_context("spawn").Pool(workers) as pool:
        for i, lp in enumerate(pool.imap(_gen_one, [(i * stride, m_max) for i in range(B)], chunksize=1)):
            out.append(lp)
            if (i + 1) % 32 == 0:
                print(f"[bench] generated {i + 1}/{B}", file=sys.stderr, flush=True)
    return out


def bench_batched(args, emit=True):
    """256 planted LPs (C3 recipe, m ~ U{1000..m_max}): one batched solve vs the
    same LPs solved one at a time with the same library on the same GPU.
    Prints the JSON line (emit) and returns it."""
    import numpy as np
    import torch

    import lpgen
    import paper_2508_16806_amd as pd

    B = args.batch
    stride = getattr(args, "stride", 1)
    t = time.perf_counter()
    lps = _gen_batched(B, args.m_max, stride)
    gen_s = time.perf_counter() - t
    nnz = sum(lp.nnz for lp in lps)
    print(f"[bench] generated {B} LPs (m <= {args.m_max}, every {stride}. instance), nnz {nnz} in {gen_s:.1f}s",
          file=sys.stderr, flush=True)
    kw = dict(precision="f32", eps=1e-4, max_iters=200000, time_limit=170.0)
    t0 = time.perf_counter()
    sb = pd.Solver(lps, batch_resident_bytes=args.resident_bytes, **kw)
    setup_s = time.perf_counter() - t0
    si = sb.info()
    setup = {"seconds": setup_s, **{k: si["setup_" + k + "_seconds"] for k in ("plan", "host", "copy", "device", "power")},
             "power_iters_max": si["power_iters_max"]}
    print(f"[bench] batched setup {setup_s:.1f}s ({json.dumps({k: round(v, 2) for k, v in setup.items()})})",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = sb.solve()
    tb = time.perf_counter() - t0
    print(f"[bench] batched: {tb:.2f}s, iters max {max(r['iters'] for r in rb)}", file=sys.stderr, flush=True)
    sb.close()
    del sb
    solo = []
    for i, lp in enumerate(lps if not getattr(args, "no_solo", False) else []):
        s = pd.Solver(lp, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()[0]
        solo.append((time.perf_counter() - t0, r, lp.m, lp.nnz))
        s.close()
        if (i + 1) % 16 == 0:
            print(f"[bench] one by one: {i + 1}/{B} solved, {sum(x[0] for x in solo):.1f}s so far", file=sys.stderr,
                  flush=True)
    ts = sum(x[0] for x in solo)
    same = all(rb[i]["iters"] == solo[i][1]["iters"] for i in range(len(solo))) if solo else None
    gaps = [abs(r["kkt"]["pobj"] - lp.f_star) / (1 + abs(lp.f_star)) for r, lp in zip(rb, lps)]
    buckets = {}
    for (dt, r, m, z) in solo:
        k = f"m<{((m - 1) // 2500 + 1) * 2500}"
        b = buckets.setdefault(k, {"lps": 0, "solo_s": 0.0, "iters": 0})
        b["lps"] += 1
        b["solo_s"] += dt
        b["iters"] += r["iters"]
    out = {"metric": METRIC, "value": B / tb, "unit": "LPs/s (batched)", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": tb * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{B} planted LPs (instances 0, {stride}, .., {(B - 1) * stride} of the batched "
                                  f"recipe), m ~ U{{1000..{args.m_max}}}, n = 2.5m, density U(0.001, 0.01); "
                                  f"total nnz {nnz}; eps 1e-4",
                      "batch": B, "nnz_total": nnz, "resident_bytes": args.resident_bytes,
                      "bins": {k: kw[k] for k in ("bin_len_primal", "bin_len_dual", "bin_rows_primal",
                                                  "bin_rows_dual", "xcd_remap", "max_grid") if k in kw}
                      or "default"},
           "batched": {"seconds": tb, "lps_per_s": B / tb, "setup": setup,
                       "status": {k: sum(1 for r in rb if r["status_name"] == k) for k in set(r["status_name"] for r in rb)}},
           "one_by_one": {"seconds": ts, "lps_per_s": B / ts, "buckets": buckets} if solo else None,
           "speedup": ts / tb if solo else None, "iterations_identical": same,
           "max_rel_obj_gap_vs_planted": max(gaps)}
    if emit:
        print(json.dumps(out), flush=True)
    return out


def bench_adjoint(args):
    """64 SCED-shaped LPs at 1/10 of C1: warm start from a batched solve at 1e-4,
    then K = 500 recorded fixed-step iterations (checkpoint every 50) and the
    adjoint of L = sum_i c_i' x_K,i."""
    import numpy as np
    import torch

    import lpgen
    import paper_2508_16806_amd as pd

    B, K, C = args.batch, 500, 50
    t = time.perf_counter()
    lps = [lpgen.config4_instance(i) for i in range(B)]
    print(f"[bench] generated {B} SCED/10 LPs in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    from paper_2508_16806_amd import tuner

    # the layout tuned on this batch (tuner --workload sced_tenth64)
    tune = tuner.load(os.path.join(ROOT, "paper_2508_16806_amd", "tuning", "sced_tenth64_f32.json"))
    s = pd.Solver(lps, precision="f32", eps=1e-4, max_iters=200000, unroll_capacity=K, unroll_checkpoint=C, **tune)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = s.solve()
    tsolve = time.perf_counter() - t0
    xs, ys = [], []
    for i in range(B):
        x, y = s.solution(inst=i)
        xs.append(x)
        ys.append(y)
    for i in range(B):
        s.set_state(xs[i], ys[i], inst=i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(K, record=True)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    c = np.concatenate([lp.c for lp in lps])
    t0 = time.perf_counter()
    g = s.backward(c, np.zeros(sum(lp.m for lp in lps)))
    tbw = time.perf_counter() - t0
    # envelope comparison (reported, not gated): d(c'x_K)/dc = x_K + (dx_K/dc)' c  vs  x*
    xk = np.concatenate([s.solution(inst=i, which=pd.SOL_CURRENT)[0] for i in range(B)])
    xstar = np.concatenate(xs)
    total = xk + g["c"]
    env = float(np.linalg.norm(total - xstar) / np.linalg.norm(xstar))
    nnz = sum(lp.nnz for lp in lps)
    out = {"metric": METRIC, "value": B * K / tf, "unit": "LP-steps/s (recorded forward)", "n_gpus": 1,
           "steps": K, "warmup": 0, "ms_per_step": tf * 1e3 / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{B} SCED-shaped LPs at 1/10 of C1 (n={lps[0].n}, m={lps[0].m}), "
                                  f"K={K} unrolled steps, checkpoint every {C}", "nnz_total": nnz, "bins": tune},
           "solve_seconds": tsolve, "solve_iters_max": max(r["iters"] for r in rs),
           "forward_seconds": tf, "backward_seconds": tbw, "backward_over_forward": tbw / tf,
           "envelope_rel_diff_dobj_dc_vs_xstar": env}
    print(json.dumps(out), flush=True)


def bench_c2(args, emit=True, shard_leg=True):
    """C2: the large random LP (m = 1M, n = 2M, Zipf(1.5) row lengths, ~54M
    nonzeros) with its tuned layout: chunked iterations/s, per-kernel times
    and roofline, the time to 1e-4 (objective gap to the planted optimum),
    and (shard_leg) the sweeps of one GPU's share under an 8-way row / column
    partition (rows m/8 of K with the full gathered xbar; rows n/8 of K^T with
    the full gathered y), each block timed.  Returns (record, lp, point):
    point is the time-to-tolerance solve's (x, y) for the oracle leg."""
    import numpy as np
    import torch

    import lpgen
    import paper_2508_16806_amd as pd
    from paper_2508_16806_amd import tuner

    t = time.perf_counter()
    zs = getattr(args, "zipf_s", 1.5)
    lp = lpgen.config2(s=zs)
    print(f"[bench] generated {lp.name}: n={lp.n} m={lp.m} nnz={lp.nnz} in {time.perf_counter() - t:.1f}s",
          file=sys.stderr, flush=True)
    # the tuning file was searched on the Zipf(1.5) LP; another exponent is
    # tuned here (one autotuner search)
    if zs == 1.5:
        tune = tuner.load(os.path.join(ROOT, "paper_2508_16806_amd", "tuning", "zipf_c2_f32.json"))
    else:
        best, rec = pd.autotune(lp, reps=10, precision="f32")
        tune = {k: rec[k] for k in ("bin_len_primal", "bin_len_dual", "bin_rows_primal", "bin_rows_dual",
                                    "xcd_remap", "max_grid", "col_slices", "col_slices_t")}
        print(f"[bench] tuned: {json.dumps(tune)}", file=sys.stderr, flush=True)
    CE = 64
    s = pd.Solver(lp, precision="f32", eps=1e-12, max_iters=CE * max(args.warmup, 1), **tune)
    info = s.info()
    print(f"[bench] C2 setup {info['setup_seconds']:.2f}s knorm={info['knorm']:.6g}", file=sys.stderr, flush=True)
    if args.warmup > 0:
        s.solve()
    s.set_opts(max_iters=CE * args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve()[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r["iters"] == CE * args.steps, r
    ips = r["iters"] / dt
    if getattr(args, "calib_copy", False):
        _calib_copy()
    kt = s.time_kernels(reps=20)
    pb, db = sweep_bytes(info, 4)
    pg, dg = pb / (kt["ms_primal"] * 1e-3) / 1e9, db / (kt["ms_dual"] * 1e-3) / 1e9
    dom = "dual" if kt["ms_dual"] >= kt["ms_primal"] else "primal"
    ach = dg if dom == "dual" else pg
    print(f"[bench] C2 {ips:.1f} iter/s; primal {kt['ms_primal']*1e3:.1f} us ({pg:.0f} GB/s), dual "
          f"{kt['ms_dual']*1e3:.1f} us ({dg:.0f} GB/s), check {kt['ms_check']*1e3:.1f} us", file=sys.stderr,
          flush=True)
    s.close()
    del s
    ttt, point, point_ad = None, None, None
    if not args.no_ttt:
        # a cold start on a fresh handle (a later solve of one handle starts
        # from its last primal weight); setup not timed
        s = pd.Solver(lp, precision="f32", eps=1e-4, max_iters=2_000_000, time_limit=120.0, **tune)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rt = s.solve()[0]
        tsec = time.perf_counter() - t0
        x, y = s.solution()
        point = (x, y)
        ttt = {"seconds": tsec, "status": rt["status_name"], "iters": rt["iters"], "restarts": rt["restarts"],
               "rel_kkt_gpu": rt["kkt"]["rel_kkt"], "rel_kkt_fp64_recheck": s.kkt(x, y)["rel_kkt"],
               "pobj": rt["kkt"]["pobj"],
               "rel_obj_gap_vs_planted": abs(rt["kkt"]["pobj"] - lp.f_star) / (1 + abs(lp.f_star)),
               "setup_seconds": info["setup_seconds"]}
        print(f"[bench] C2 time to 1e-4: {tsec:.2f}s {rt['status_name']} iters={rt['iters']}", file=sys.stderr,
              flush=True)
        s.close()
        del s
        # adaptive steps (Algorithm 5), the same cold start: the attempts'
        # dual sweep takes the tuned column slices too
        s = pd.Solver(lp, precision="f32", eps=1e-4, max_iters=2_000_000, time_limit=120.0, adaptive_step=1, **tune)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ra = s.solve()[0]
        tsa = time.perf_counter() - t0
        point_ad = s.solution()
        ka = s.time_kernels(reps=5)
        ttt["adaptive_step"] = {"seconds": tsa, "status": ra["status_name"], "iters": ra["iters"],
                                "accepted": ra["accepted"], "restarts": ra["restarts"],
                                "rel_kkt_gpu": ra["kkt"]["rel_kkt"],
                                "rel_obj_gap_vs_planted": abs(ra["kkt"]["pobj"] - lp.f_star) / (1 + abs(lp.f_star)),
                                "ms_primal_ad": ka["ms_primal_ad"], "ms_dual_ad": ka["ms_dual_ad"],
                                "ms_step_ad": ka["ms_step_ad"]}
        print(f"[bench] C2 adaptive steps: time to 1e-4: {tsa:.2f}s {ra['status_name']} attempts={ra['iters']}",
              file=sys.stderr, flush=True)
        s.close()
        del s
    shard = None
    if shard_leg:
        # one GPU's share of an 8-way partition, every block
        P = 8
        shard = {"parts": P, "dual_ms": [], "primal_ms": [], "dual_gbs": [], "primal_gbs": []}
        for p in range(P):
            r0, r1 = p * lp.m // P, (p + 1) * lp.m // P
            c0, c1 = p * lp.n // P, (p + 1) * lp.n // P
            for kind, sub in (("dual", lpgen.row_block(lp, r0, r1)), ("primal", lpgen.col_block(lp, c0, c1))):
                ss = pd.Solver(sub, precision="f32", **tune)
                si = ss.info()
                ss.time_kernels(reps=3)
                k = ss.time_kernels(reps=20)
                ms = k["ms_" + kind]
                b = sweep_bytes(si, 4)[0 if kind == "primal" else 1]
                shard[kind + "_ms"].append(ms)
                shard[kind + "_gbs"].append(b / (ms * 1e-3) / 1e9)
                ss.close()
                del ss, sub
            print(f"[bench] shard {p}/{P}: dual {shard['dual_ms'][-1]*1e3:.1f} us, primal "
                  f"{shard['primal_ms'][-1]*1e3:.1f} us", file=sys.stderr, flush=True)
        shard["iter_sweeps_ms_slowest"] = max(shard["dual_ms"]) + max(shard["primal_ms"])
        shard["full_sweeps_ms_over_parts"] = (kt["ms_dual"] + kt["ms_primal"]) / P
    out = {"metric": METRIC, "value": ips, "unit": "PDHG iter/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"large random LP {lp.name}: n={lp.n}, m={lp.m}, nnz={lp.nnz}, Zipf({zs}) row "
                                  f"lengths; FP32 iterates, FP64 accumulation and check; step = {CE} iterations "
                                  f"+ check", "n": lp.n, "m": lp.m, "nnz": lp.nnz, "iters_per_step": CE,
                      "bins": tune},
           "roofline": {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": ach / PEAK_HBM_GBS, "traffic": None, "kernel": f"k_{dom}",
                        "algorithmic_bytes": db if dom == "dual" else pb,
                        "ms_per_launch": kt["ms_dual" if dom == "dual" else "ms_primal"]},
           "kernels_ms": {k: v for k, v in kt.items() if k != "reps"}, "sweep_gbs": {"primal": pg, "dual": dg},
           "time_to_tol": ttt, "shard": shard, "cpu_baseline": None}
    if emit:
        print(json.dumps(out), flush=True)
    return out, lp, {"time_to_tol": point, "adaptive_step": point_ad}


def measured_copy_gbs(nbytes, reps=20):
    """Device-to-device copy bandwidth (bytes read + written per second, in
    GB/s), timed with HIP events on the current stream: two buffer pairs of
    `nbytes` each, copied alternately, as the iteration alternates its two
    sweeps (so the copies, like the sweeps, find in the Infinity Cache only
    what the other left).  The measured ceiling the sweeps are compared with."""
    import torch

    bufs = [(torch.empty(nbytes, dtype=torch.uint8, device="cuda"),
             torch.empty(nbytes, dtype=torch.uint8, device="cuda")) for _ in range(2)]
    for k in range(4):
        bufs[k & 1][1].copy_(bufs[k & 1][0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(2 * reps):
        bufs[k & 1][1].copy_(bufs[k & 1][0])
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / (2 * reps)
    del bufs
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _calib_copy():
    """Three plain 256 MiB device copies: the reference kernel against which
    the FETCH_SIZE / WRITE_SIZE counters are scaled under rocprofv3 --pmc."""
    import torch

    a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance solve")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-one-by-one legs of the default run (256 LPs with m <= 10,000; "
                         "64 LPs over m <= 50,000)")
    ap.add_argument("--no-c2", action="store_true", help="skip the large Zipf LP leg of the default run")
    ap.add_argument("--no-shard", action="store_true", help="--workload c2: skip the 8-way share leg")
    ap.add_argument("--zipf-s", type=float, default=1.5,
                    help="--workload c2: Zipf exponent of the row lengths (1.6956 gives ~20M nonzeros)")
    ap.add_argument("--small", action="store_true", help="reduced SCED size (for profiling tests)")
    ap.add_argument("--no-tuning", action="store_true", help="default bins instead of the tuned ones")
    ap.add_argument("--workload", default="c1", choices=["c1", "c2", "c3", "c4"],
                    help="c1: SCED-shaped LP (default); c2: large Zipf LP and one GPU's 1/8 share; "
                         "c3: batched vs one-by-one; c4: unrolled adjoint")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--m-max", type=int, default=50000)
    ap.add_argument("--no-solo", action="store_true",
                    help="--workload c3: the batched solve only (no one-by-one leg; for kernel traces)")
    ap.add_argument("--resident-bytes", type=int, default=192_000_000,
                    help="batched solve: admission budget of running instances' sweep bytes (0: all at once)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run plain 256 MiB device copies (counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the PDHG path is not sharded over "
              f"several GPUs; `--workload c2` times one GPU's 1/8 share of the large LP instead.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lpgen
    import paper_2508_16806_amd as pd

    if not torch.cuda.is_available():
        print("bench.py needs the GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "c3":
        args.batch = args.batch or 256
        return bench_batched(args)
    if args.workload == "c4":
        args.batch = args.batch or 64
        return bench_adjoint(args)
    if args.workload == "c2":
        bench_c2(args, shard_leg=not args.no_shard)
        return
    t = time.perf_counter()
    lp = lpgen.sced(500, 200, 24, 125, seed=1) if args.small else lpgen.config1()
    gen_s = time.perf_counter() - t
    print(f"[bench] generated {lp.name}: n={lp.n} m={lp.m} nnz={lp.nnz} in {gen_s:.1f}s", file=sys.stderr,
          flush=True)
    CE = 64
    tune = {}
    if not args.small and not args.no_tuning:
        from paper_2508_16806_amd import tuner

        tune = tuner.load(os.path.join(ROOT, "paper_2508_16806_amd", "tuning", "sced_c1_f32.json"))
    s = pd.Solver(lp, precision="f32", eps=1e-12, max_iters=CE * max(args.warmup, 1), **tune)
    info = s.info()
    print(f"[bench] setup {info['setup_seconds']:.2f}s knorm={info['knorm']:.6g} "
          f"blocks primal={info['nblk_primal']} dual={info['nblk_dual']}", file=sys.stderr, flush=True)
    # warmup: W steps
    if args.warmup > 0:
        s.solve()
    # timed: exactly K steps (the iteration limit caps the enqueued chunks)
    s.set_opts(max_iters=CE * args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve()[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r["iters"] == CE * args.steps, r
    ips = r["iters"] / dt
    print(f"[bench] {args.steps} steps of {CE} iterations in {dt*1e3:.1f} ms: {ips:.1f} iter/s",
          file=sys.stderr, flush=True)

    if args.calib_copy:
        _calib_copy()
    kt = s.time_kernels(reps=20)
    pb, db = sweep_bytes(info, 4)
    pg, dg = pb / (kt["ms_primal"] * 1e-3) / 1e9, db / (kt["ms_dual"] * 1e-3) / 1e9
    dom = "dual" if kt["ms_dual"] >= kt["ms_primal"] else "primal"
    ach = dg if dom == "dual" else pg
    # copies that read and write as many bytes as the two sweeps move, in turn
    # (not under --calib-copy: the counter calibration reads the copy kernels
    # of that run, which must be the 256 MiB ones alone)
    copy_gbs = None if args.calib_copy else measured_copy_gbs(int((db + pb) // 4))
    print(f"[bench] kernels (ms): {json.dumps({k: round(v, 4) for k, v in kt.items() if k != 'reps'})} "
          f"primal {pg:.0f} GB/s dual {dg:.0f} GB/s; device copies {copy_gbs or 0:.0f} GB/s",
          file=sys.stderr, flush=True)

    def cold_solves(runs, **extra):
        """`runs` cold-start solves to 1e-4, each on a fresh handle (a later
        solve of one handle starts from its last primal weight), setup not
        timed: the median run's result, handle and every run's seconds."""
        res = []
        for _ in range(runs):
            so = pd.Solver(lp, precision="f32", eps=1e-4, max_iters=2_000_000, time_limit=120.0, **tune, **extra)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ro = so.solve()[0]
            res.append((time.perf_counter() - t0, ro, so))
        order = sorted(range(runs), key=lambda i: res[i][0])
        med = res[order[runs // 2]]
        for i in range(runs):
            if res[i] is not med:
                res[i][2].close()
        return med, [r[0] for r in res]

    ttt = None
    points = {}  # returned points, checked by the oracle leg
    if not args.no_ttt:
        (tsec, rt, so), secs = cold_solves(5)
        x, y = so.solution()
        points["time_to_tol"] = (x, y)
        ttt = {"seconds": tsec, "runs_seconds": secs, "status": rt["status_name"], "iters": rt["iters"],
               "restarts": rt["restarts"], "rel_kkt_gpu": rt["kkt"]["rel_kkt"], "pobj": rt["kkt"]["pobj"],
               "setup_seconds": info["setup_seconds"]}
        # the library's own FP64 KKT of the returned point on the original LP
        ttt["rel_kkt_fp64_recheck"] = so.kkt(x, y)["rel_kkt"]
        so.close()
        print(f"[bench] time to 1e-4 (median of 5 cold starts): {tsec:.3f}s {rt['status_name']} "
              f"iters={rt['iters']} restarts={rt['restarts']}", file=sys.stderr, flush=True)

    # the other configurations' time to 1e-4 from a cold start on one LP each
    # (setup excluded), next to the oracle's in cpu_baseline.time_to_1e-4: C0
    # in FP64 (its configuration), one C4 LP (SCED/10) in FP32
    small_ttt = {}
    if not args.no_ttt:
        for name, slp, prec in (("C0", lpgen.config0(0), "f64"), ("C4[0]", lpgen.config4_instance(0), "f32")):
            so = pd.Solver(slp, precision=prec, eps=1e-4, max_iters=400_000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ro = so.solve()[0]
            small_ttt[name] = {"seconds": time.perf_counter() - t0, "status": ro["status_name"],
                               "iters": ro["iters"], "precision": prec, "rel_kkt_gpu": ro["kkt"]["rel_kkt"]}
            so.close()

    # adaptive step size (Algorithm 5): its sweeps' device time and the time
    # to the same tolerance from the same cold start
    pba, dba = sweep_bytes_ad(info, 4)
    adaptive = {"ms_primal_ad": kt["ms_primal_ad"], "ms_dual_ad": kt["ms_dual_ad"],
                "ms_step_ad": kt["ms_step_ad"],
                "gbs_primal_ad": pba / (kt["ms_primal_ad"] * 1e-3) / 1e9,
                "gbs_dual_ad": dba / (kt["ms_dual_ad"] * 1e-3) / 1e9}
    if not args.no_ttt:
        (tsa, ra, so), secs = cold_solves(5, adaptive_step=1)
        x, y = so.solution()
        points["adaptive_step"] = (x, y)
        adaptive["time_to_tol"] = {"seconds": tsa, "runs_seconds": secs, "status": ra["status_name"],
                                   "iters": ra["iters"], "accepted": ra["accepted"], "restarts": ra["restarts"],
                                   "rel_kkt_fp64_recheck": so.kkt(x, y)["rel_kkt"],
                                   "pobj": ra["kkt"]["pobj"]}
        so.close()
        print(f"[bench] adaptive steps: time to 1e-4 (median of 5): {tsa:.3f}s {ra['status_name']} "
              f"iters={ra['iters']} accepted={ra['accepted']} restarts={ra['restarts']}", file=sys.stderr,
              flush=True)

    # fishnet casting (Algorithm 7): 32 points, 64 steps per round, then the
    # restarted solve from the surviving point
    fish = None
    if not args.no_ttt:
        sf = pd.Solver(lp, precision="f32", eps=1e-4, max_iters=2_000_000, time_limit=120.0, fishnet_points=32,
                       **tune)
        sf.fishnet(32, 64, seed=0)  # first call: row orders and kernel loads
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fo = sf.fishnet(32, 64, seed=1)
        tfn = time.perf_counter() - t0
        t0 = time.perf_counter()
        rf = sf.solve()[0]
        tfs = time.perf_counter() - t0
        x, y = sf.solution()
        points["fishnet"] = (x, y)
        pts = 0
        j = 32
        for r in range(fo["rounds"]):  # live points per round
            pts += j * 64
            half = j // 2
            j = 2 * half if (r % 2 == 1 and j > 2) else half
        fish = {"points": 32, "k": 64, "rounds": fo["rounds"], "seconds_fishnet": tfn, "point_iters": pts,
                "point_iters_per_s": pts / tfn, "seconds_solve_after": tfs, "status": rf["status_name"],
                "iters_after": rf["iters"], "restarts_after": rf["restarts"],
                "rel_kkt_fp64_recheck": sf.kkt(x, y)["rel_kkt"], "pobj": rf["kkt"]["pobj"],
                "seconds_total": tfn + tfs}
        sf.close()
        del sf
        print(f"[bench] fishnet 32 x 64: {tfn:.3f}s ({pts / tfn:.0f} point-iter/s), then solve to 1e-4 in "
              f"{tfs:.3f}s {rf['status_name']} iters={rf['iters']}", file=sys.stderr, flush=True)

    # FP64 reference for the objective gaps of the FP32 points: an FP64 solve
    # to 1e-8, certified by the oracle leg below
    ref64 = None
    if not args.no_ttt and not args.no_cpu_baseline:
        s64 = pd.Solver(lp, precision="f64", eps=1e-8, max_iters=2_000_000, time_limit=120.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r64 = s64.solve()[0]
        t64 = time.perf_counter() - t0
        points["fp64_ref"] = s64.solution()
        ref64 = {"seconds": t64, "status": r64["status_name"], "iters": r64["iters"], "eps": 1e-8,
                 "pobj": r64["kkt"]["pobj"]}
        s64.close()
        del s64
        print(f"[bench] FP64 reference to 1e-8: {t64:.2f}s {r64['status_name']} iters={r64['iters']}",
              file=sys.stderr, flush=True)
    s.close()
    del s

    # the large Zipf LP (C2): its iteration rate, dominant sweep and time to 1e-4
    c2 = c2_lp = c2_point = None
    if not args.no_c2 and not args.small:
        c2a = argparse.Namespace(steps=20, warmup=1, no_ttt=args.no_ttt)
        c2o, c2_lp, c2_point = bench_c2(c2a, emit=False, shard_leg=False)
        c2 = {k: c2o[k] for k in ("value", "unit", "ms_per_step", "roofline", "kernels_ms", "sweep_gbs",
                                  "time_to_tol")}
        c2["workload"] = c2o["config"]["workload"]

    # batched vs one-by-one LPs/s: 256 planted LPs with m <= 10,000 (the
    # batched workload's small-m range), and 64 of its instances spread over
    # the full range m <= 50,000 (--workload c3 runs all 256 of them)
    batched = batched_full = None
    if not args.no_batched and not args.small:
        def _brief(bo):
            return {"workload": bo["config"]["workload"], "lps": bo["config"]["batch"],
                    "batched_lps_per_s": bo["batched"]["lps_per_s"],
                    "one_by_one_lps_per_s": bo["one_by_one"]["lps_per_s"], "speedup": bo["speedup"],
                    "iterations_identical": bo["iterations_identical"],
                    "max_rel_obj_gap_vs_planted": bo["max_rel_obj_gap_vs_planted"],
                    "batched_setup_seconds": bo["batched"]["setup"]["seconds"],
                    "buckets_one_by_one": bo["one_by_one"]["buckets"]}

        batched = _brief(bench_batched(argparse.Namespace(batch=256, m_max=10000, stride=1,
                                                          resident_bytes=args.resident_bytes), emit=False))
        print(f"[bench] batched vs one-by-one (256 LPs, m <= 10k): {batched['speedup']:.2f}x", file=sys.stderr,
              flush=True)
        batched_full = _brief(bench_batched(argparse.Namespace(batch=64, m_max=50000, stride=4,
                                                               resident_bytes=args.resident_bytes), emit=False))
        print(f"[bench] batched vs one-by-one (64 LPs over m <= 50k): {batched_full['speedup']:.2f}x",
              file=sys.stderr, flush=True)

    # the CPU leg: the oracle's rates and times, and its checks of the GPU points
    cpu = None
    if not args.no_cpu_baseline:
        cpu, checks = oracle_leg(lp, points, small=args.small)
        print(f"[bench] cpu baseline {cpu['value']:.2f} iter/s on {cpu['cores']} threads, "
              f"{cpu.get('value_1core') or 0:.2f} on one", file=sys.stderr, flush=True)
        if "fp64_ref" in checks:
            ref64["rel_kkt_oracle"] = checks["fp64_ref"]["rel_kkt"]
            ref64["certified"] = checks["fp64_ref"]["rel_kkt"] <= 1e-8 * 1.01
            fref = checks["fp64_ref"]["pobj"]
            for name, rec in (("time_to_tol", ttt), ("adaptive_step", adaptive.get("time_to_tol")),
                              ("fishnet", fish)):
                if rec is not None and name in checks:
                    rec["rel_kkt_oracle"] = checks[name]["rel_kkt"]
                    rec["rel_obj_gap_fp64_ref"] = abs(checks[name]["pobj"] - fref) / (1 + abs(fref))
        if c2_point is not None and c2_point["time_to_tol"] is not None:
            c2chk = oracle_checks(c2_lp, {k: v for k, v in c2_point.items() if v is not None})
            c2["time_to_tol"]["rel_kkt_oracle"] = c2chk["time_to_tol"]["rel_kkt"]
            if "adaptive_step" in c2chk:
                c2["time_to_tol"]["adaptive_step"]["rel_kkt_oracle"] = c2chk["adaptive_step"]["rel_kkt"]

    out = {
        "metric": METRIC,
        "value": ips,
        "unit": "PDHG iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"SCED-shaped LP {lp.name}: n={lp.n}, m={lp.m}, nnz={lp.nnz}; "
                               f"FP32 iterates, FP64 accumulation and check; step = {CE} iterations + check",
                   "n": lp.n, "m": lp.m, "nnz": lp.nnz, "iters_per_step": CE, "precision": "f32+f64acc",
                   "bins": tune or "default"},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic(f"k_{dom}"), "kernel": f"k_{dom}",
                     "algorithmic_bytes": db if dom == "dual" else pb,
                     "ms_per_launch": kt["ms_dual" if dom == "dual" else "ms_primal"],
                     # against device copies that move the two sweeps' bytes in turn
                     "measured_copy_gbs": copy_gbs, "frac_of_measured_copy": ach / copy_gbs if copy_gbs else None},
        "kernels_ms": {k: v for k, v in kt.items() if k != "reps"},
        "kernel_src_sha": kernel_src_hash(),
        "sweep_gbs": {"primal": pg, "dual": dg},
        "time_to_tol": ttt,
        "time_to_tol_small": small_ttt,
        "adaptive_step": adaptive,
        "fishnet": fish,
        "fp64_reference": ref64,
        "c2": c2,
        "batched": batched,
        "batched_full": batched_full,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the Join-Project hot path on one MI355X.

One step = the whole path for one query over inputs already resident in HBM:
jp_plan_create (mapping, CSR, partition by z) + jp_execute (SparseBMM and
DenseEC count kernels, per-row offsets) + jp_count (host read of the counts),
which is the paper's count-only mode.  The default workload is the skewed
single query: R and S with 1e7 distinct tuples each, x and z uniform in
[0, 1e6), y Zipf(1.0) over [0, 1e5).

Prints one JSON line with the metric, a roofline object for the dominant
kernel (times from HIP events on the stream the kernel runs on) and a CPU
baseline (the oracle timed on the host over a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# int32 vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one 32-bit op per lane per clock)
VALU_I32_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# dense INT8 matrix-core peak of MI355X (no structured sparsity)
MFMA_I8_PEAK_TOPS = 5000.0


# HBM traffic of the dominant count kernels, per launch: rocprofv3 FETCH_SIZE
# and WRITE_SIZE (KiB per dispatch, one counter per run) scaled by what the
# same counters read for one plain elementwise kernel that reads and writes
# 1 GiB (FETCH_SIZE reads 524308 KiB for it, WRITE_SIZE 1048576 KiB).  Each
# entry carries the sha256 of the sources the kernel was built from; when they
# differ from the tree being run the counters are stale and traffic is null.
FETCH_FACTOR = 1048576 / 524308.0
WRITE_FACTOR = 1.0
MEASURED_TRAFFIC = {
    # two count launches per step: rows without and with the pivot key (2 windows per workgroup, as tuned)
    "skewed": {"kernels": "k_dense_bits<false> x 2", "fetch_kib": 663647.8 + 275965.1, "write_kib": 80210.6 + 39764.1,
               "sources": {"dense_ec.hip": "9abaf47b14713dc235ed9bb4d25b280a95c0f2e143ff38b509303eb9123bc0ad",
                           "stages.h": "19c030a1670b519a14c35bf3e9f052e634aca0be7ac1bd4d72947b679aac04fc",
                           "common.h": "1e62888273711daaffd80f57584a98f295562b616c4d66eaa3fffa0c1186baa5"}},
    # the whole timed SparseBMM count region: per-entry segments and their scan,
    # row work, row lists, the light/medium/heavy count kernels
    "graph": {"kernels": "SparseBMM count pass (k_entry_seg ... k_sparse_heavy_count)",
              "fetch_kib": 2757289.5, "write_kib": 372779.5,
              "sources": {"sparse_bmm.hip": "0563945fb2abfe85c00b9423b0102642ee95735227e00dc29ac7eb30a2a15044",
                          "prim.hip": "357a597bf671428e992d90c55058e3ad4a1e381eb3669035c44e9d121fbb67c6",
                          "stages.h": "19c030a1670b519a14c35bf3e9f052e634aca0be7ac1bd4d72947b679aac04fc",
                          "common.h": "1e62888273711daaffd80f57584a98f295562b616c4d66eaa3fffa0c1186baa5"}},
    "dense": {"kernels": "k_dense_mfma", "fetch_kib": 809038.4, "write_kib": 12343.8,
              "sources": {"dense_mfma.hip": "c4103f00b68fb47500e9e25f66d0e6c7b0317e25200728f600fa7ef5ed3c3ed4",
                          "stages.h": "19c030a1670b519a14c35bf3e9f052e634aca0be7ac1bd4d72947b679aac04fc",
                          "common.h": "1e62888273711daaffd80f57584a98f295562b616c4d66eaa3fffa0c1186baa5"}},
}


def measured_traffic(workload: str):
    """HBM bytes per step of the dominant kernel(s) from the committed counter runs, or None if stale."""
    import hashlib

    m = MEASURED_TRAFFIC.get(workload)
    if m is None:
        return None
    csrc = os.path.join(ROOT, "paper_2206_04995_amd", "csrc")
    for f, h in m["sources"].items():
        with open(os.path.join(csrc, f), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != h:
                return None
    return (m["fetch_kib"] * FETCH_FACTOR + m["write_kib"] * WRITE_FACTOR) * 1024.0


def make_workload(name: str):
    import synth

    if name == "skewed":
        inst = synth.config2()
        desc = {"workload": "skewed single query", "tuples_per_side": 10_000_000, "x_z_domain": 1_000_000,
                "y_domain": 100_000, "y_zipf_s": 1.0, "distinct_tuples": True}
    elif name == "uniform":
        inst = synth.config1()
        desc = {"workload": "plain single query", "tuples_per_side": 100_000, "x_z_domain": 10_000,
                "y_domain": 5_000, "distinct_tuples": True}
    elif name == "dense":
        inst = synth.uniform_paper_default(n_tuples=10_000_000, n_domain=10_000)
        desc = {"workload": "dense uniform query", "tuples_per_side": 10_000_000, "x_y_z_domain": 10_000,
                "distinct_tuples": False}
    elif name == "graph":
        inst = synth.config3()
        desc = {"workload": "power-law graph self-join", "vertices": 2_000_000, "edges": 20_000_000,
                "out_degree": "Pareto(2.1)"}
    else:
        raise SystemExit(f"unknown workload {name}")
    return inst, desc


def cpu_baseline(inst, sample_mod: int):
    """The oracle as it stands, on the rows of every sample_mod-th x value (full S)."""
    import oracle

    oracle.build(force=False)
    sel = (inst.rx % sample_mod) == 0
    rx, ry = inst.rx[sel], inst.ry[sel]
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    pairs, _ = oracle.count(rx, ry, inst.sz, inst.sy, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"R rows with x % {sample_mod} == 0 ({int(sel.sum())} tuples), all of S; "
                      f"{pairs} distinct pairs in {dt:.2f} s"}


def batched(args):
    """Many independent instances: one batched plan (every stage one launch over
    all instances) against the plain loop of one plan per instance, same GPU,
    same inputs, identical per-instance counts required."""
    import torch
    import paper_2206_04995_amd as P
    import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    insts = [synth.config4_instance(i, hi=args.batch_hi) for i in range(args.instances)]
    cols = [tuple(torch.from_numpy(c).to(dev) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    n_tuples = sum(a.n_r + a.n_s for a in insts)
    print(f"[bench] {args.instances} instances, {n_tuples} tuples, generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    tuned = []
    if not args.no_tune:
        # one representative per shape signature among the first instances (both paths use the result)
        P.jp_tune_clear()
        seen = set()
        for c in cols[:args.tune_sample]:
            r = P.jp_tune(*c, stream=stream)
            if r["signature"] not in seen:
                seen.add(r["signature"])
                tuned.append({"tau": r["tau"], "model_tau": r["model_tau"], "signature": r["signature"]})
        print(f"[bench] tuned {len(seen)} shape signatures", file=sys.stderr, flush=True)

    def plain():
        out = []
        for c in cols:
            h = P.jp_plan_create(*c, stream=stream)
            try:
                P.jp_execute(h, stream)
                out.append(P.jp_count(h, stream)[0])
            finally:
                P.jp_plan_destroy(h)
        return np.array(out, dtype=np.int64)

    def batch():
        b = P.jp_batch_create(cols, stream=stream)
        try:
            P.jp_batch_execute(b, stream)
            return P.jp_batch_counts(b, len(cols), stream)
        finally:
            P.jp_batch_destroy(b)

    res = {}
    paths = (("batched", batch),) if args.batched_only else (("plain", plain), ("batched", batch))
    for name, fn in paths:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            counts = fn()
        torch.cuda.synchronize()
        res[name] = ((time.perf_counter() - t0) * 1000.0 / args.steps, counts)
        print(f"[bench] {name}: {res[name][0]:.2f} ms per pass", file=sys.stderr, flush=True)
    if "plain" in res and not np.array_equal(res["plain"][1], res["batched"][1]):
        raise SystemExit("batched and plain per-instance counts differ")
    plain_ms = res["plain"][0] if "plain" in res else None
    pairs = int(res["batched"][1].sum())
    ms = res["batched"][0]
    out = {
        "metric": "distinct (x,z) pairs/sec",
        "value": pairs / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator, inputs resident in HBM)",
        "config": {"workload": "batched instances", "instances": args.instances, "tuned_signatures": len(tuned),
                   "tuples_per_side": f"log-uniform [1e3, {args.batch_hi:.0e}]", "key_domain": "10% of tuples",
                   "y": "uniform (even) / Zipf 1.2 (odd)", "pairs": pairs, "tuples": n_tuples,
                   "plain_ms": plain_ms, "plain_pairs_per_s": None if plain_ms is None else pairs / (plain_ms * 1e-3),
                   "batched_over_plain": None if plain_ms is None else plain_ms / ms},
    }
    print(json.dumps(out), flush=True)


def served(args):
    """Poisson arrivals of a mix of queries: the continuous-batching server
    against the plain serial path (one query at a time, in arrival order) on the
    same trace, same device-resident tables; identical counts required."""
    import threading

    import torch
    import paper_2206_04995_amd as P
    import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    trace = synth.config5_trace(n_queries=args.queries, rate_per_s=1.0, p_large=args.p_large)
    n_small = sum(1 for _, k, _ in trace if k == 0)
    small = [synth.config4_instance(i, hi=args.batch_hi, batch_seed=1000) for i in range(n_small)]
    large = [synth.config2(seed_index=1 + j) for j in range(args.large_distinct)]

    def cols_of(a):
        return tuple(torch.from_numpy(c).to(dev) for c in (a.rx, a.ry, a.sz, a.sy))

    small_cols = [cols_of(a) for a in small]
    large_cols = [cols_of(a) for a in large]
    queries = [small_cols[s] if k == 0 else large_cols[(s - 1) % len(large_cols)] for _, k, s in trace]
    print(f"[bench] {len(queries)} queries ({len(queries) - n_small} large), tables built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()

    def one(c):
        h = P.jp_plan_create(*c, stream=stream)
        try:
            P.jp_execute(h, stream)
            return P.jp_count(h, stream)[0]
        finally:
            P.jp_plan_destroy(h)

    if not args.no_tune:  # thresholds for the shapes of the first queries and of the large tables
        P.jp_tune_clear()
        for c in small_cols[:args.tune_sample] + large_cols[:1]:
            P.jp_tune(*c, stream=stream)

    # calibration: service time of the serial path with every query present at once
    for c in queries[: min(8, len(queries))]:
        one(c)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    ref = [one(c) for c in queries]
    serial_busy = time.perf_counter() - tc
    rate = args.rate if args.rate > 0 else len(queries) / serial_busy
    arrivals = np.array([t for t, _, _ in trace]) / trace[-1][0] * (len(queries) / rate)

    def serial_run():
        lat = []
        start = time.perf_counter()
        for a, c in zip(arrivals, queries):
            now = time.perf_counter() - start
            if now < a:
                time.sleep(a - now)
            one(c)
            lat.append(time.perf_counter() - start - a)
        return time.perf_counter() - start, np.array(lat)

    def served_run():
        with P.Server(max_batch=args.max_batch) as srv:
            tickets = [None] * len(queries)
            start = time.perf_counter()

            def feed():
                for i, (a, c) in enumerate(zip(arrivals, queries)):
                    now = time.perf_counter() - start
                    if now < a:
                        time.sleep(a - now)
                    tickets[i] = srv.submit(*c)

            th = threading.Thread(target=feed)
            th.start()
            th.join()
            res = [srv.wait(t) for t in tickets]
            span = time.perf_counter() - start
            st = srv.stats()
        lat = np.array([(r["done_us"] - r["submit_us"]) * 1e-6 for r in res])
        return span, lat, [r["total"] for r in res], st

    s_span, s_lat = serial_run()
    v_span, v_lat, v_counts, st = served_run()
    if list(v_counts) != list(ref):
        raise SystemExit("served counts differ from the serial path")
    pairs = int(sum(ref))
    out = {
        "metric": "distinct (x,z) pairs/sec",
        "value": pairs / v_span,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": v_span * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator, tables resident in HBM)",
        "config": {"workload": "served query stream", "queries": len(queries), "large_queries": len(queries) - n_small,
                   "large_distinct_tables": len(large_cols), "arrival_rate_per_s": rate, "pairs": pairs,
                   "served": {"pairs_per_s": pairs / v_span, "p50_ms": float(np.percentile(v_lat, 50) * 1e3),
                              "p99_ms": float(np.percentile(v_lat, 99) * 1e3), "batches": st["batches"],
                              "peak_bytes": st["peak_bytes"]},
                   "serial": {"pairs_per_s": pairs / s_span, "p50_ms": float(np.percentile(s_lat, 50) * 1e3),
                              "p99_ms": float(np.percentile(s_lat, 99) * 1e3), "busy_s": serial_busy}},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="skewed",
                    choices=["skewed", "uniform", "dense", "graph", "batched", "served"])
    ap.add_argument("--queries", type=int, default=2000, help="served workload: queries in the trace")
    ap.add_argument("--p-large", type=float, default=0.01, help="served workload: share of 1e7-tuple queries")
    ap.add_argument("--large-distinct", type=int, default=2, help="served workload: distinct large tables")
    ap.add_argument("--rate", type=float, default=0.0, help="served workload: arrivals/s (0 = serial capacity)")
    ap.add_argument("--max-batch", type=int, default=256, help="served workload: server batch limit")
    ap.add_argument("--instances", type=int, default=4096, help="batched workload: number of instances")
    ap.add_argument("--batch-hi", type=float, default=1e6, help="batched workload: largest tuples per side")
    ap.add_argument("--cpu-sample-mod", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tau", type=int, default=None, help="fixed dense threshold (default: tuned cost model)")
    ap.add_argument("--no-tune", action="store_true", help="skip the threshold autotuner (untimed, before warmup)")
    ap.add_argument("--window-group", type=int, default=None,
                    help="DenseEC windows per workgroup (default: tuned or automatic; counter runs pin the tuned value)")
    ap.add_argument("--k-hot-max", type=int, default=None, help="cap on hot keys per instance (default: tuned or automatic)")
    ap.add_argument("--tune-sample", type=int, default=16, help="batched workload: instances the tuner times")
    ap.add_argument("--batched-only", action="store_true",
                    help="batched workload: skip the plain one-plan-per-instance loop (for kernel traces)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="first run one plain elementwise copy over this many MiB (a reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the path runs on a single GPU "
              f"(rows shard by x across GPUs with S broadcast, which this benchmark does not exercise)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        batched(args)
        return
    if args.workload == "served":
        served(args)
        return

    import torch
    import paper_2206_04995_amd as P

    inst, desc = make_workload(args.workload)
    print(f"[bench] workload {args.workload}: |R|={inst.n_r} |S|={inst.n_s}", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cols = [torch.from_numpy(c).to(dev) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    if args.copy_ref_mib > 0:
        # one kernel that reads and writes exactly copy_ref_mib MiB each
        src = torch.ones(args.copy_ref_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] copy reference: {args.copy_ref_mib} MiB read + written by one bitwise_not kernel",
              file=sys.stderr, flush=True)
    fixed = {}
    if args.window_group is not None:
        fixed["window_group"] = args.window_group
    if args.k_hot_max is not None:
        fixed["k_hot_max"] = args.k_hot_max
    if args.tau is None:
        opt = P.make_options(flags=P.JP_FLAG_TIMING, **fixed)
    else:
        opt = P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=args.tau, flags=P.JP_FLAG_TIMING, **fixed)
    stream = torch.cuda.current_stream()
    tune = None
    if not args.no_tune and args.tau is None:
        P.jp_tune_clear()
        tune = P.jp_tune(*cols, stream=stream)
        print(f"[bench] tuned tau {tune['tau']} (model {tune['model_tau']}): {tune['best_ms']:.2f} ms vs "
              f"{tune['model_ms']:.2f} ms", file=sys.stderr, flush=True)

    def step(want_work=False):
        h = P.jp_plan_create(*cols, opt=opt, stream=stream)
        try:
            P.jp_execute(h, stream)
            cnt = P.jp_count(h, stream)
            tm = P.jp_plan_timings(h, stream)
            st = P.jp_plan_stats(h)
            if want_work:
                tm.update(P.jp_plan_work(h, stream))
        finally:
            P.jp_plan_destroy(h)
        return cnt, tm, st

    work = None
    for i in range(args.warmup):
        cnt, tm, st = step(want_work=(i == 0))
        if i == 0:
            work = tm
        print(f"[bench] warmup {i}: pairs={cnt[0]} dense={cnt[1]} sparse={cnt[2]} tau={st['tau']} "
              f"z_dense={st['n_z_dense']} k_hot={st['k_hot']} exec={tm['execute_ms']:.2f} ms", file=sys.stderr,
              flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tms = []
    counts = set()
    for i in range(args.steps):
        cnt, tm, st = step()
        tms.append(tm)
        counts.add(cnt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if len(counts) != 1:
        raise SystemExit(f"counts differ between steps: {counts}")
    total, dense, sparse = counts.pop()
    ms = (t1 - t0) * 1000.0 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    sp_ms = float(np.mean([t["sparse_ms"] for t in tms]))
    de_ms = float(np.mean([t["dense_ms"] for t in tms]))
    ex_ms = float(np.mean([t["execute_ms"] for t in tms]))
    if work is None:  # no warmup step: take the counters from one extra, untimed step
        work = step(want_work=True)[1]
    t = work
    if de_ms >= sp_ms and t.get("dense_mfma_ops", 0) > 0:
        ops = t["dense_mfma_ops"]
        achieved = ops / (de_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "k_dense_mfma (DenseEC count, INT8 MFMA)", "achieved": achieved,
                "peak": MFMA_I8_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / MFMA_I8_PEAK_TOPS,
                "traffic": measured_traffic(args.workload), "kernel_ms": de_ms,
                "work": {"int8_ops": ops, "note": "2 * |X| * dense keys * |Z_dense|, padding excluded"}}
    elif de_ms >= sp_ms:
        ops = t["dense_hot_words"] + t["dense_row_words"] + t["dense_cold_entries"]
        achieved = ops / (de_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "k_dense_bits (DenseEC count)", "achieved": achieved,
                "peak": VALU_I32_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_I32_PEAK_TOPS,
                "traffic": measured_traffic(args.workload) if de_ms > 0 else None, "kernel_ms": de_ms,
                "work": {"int32_ops": ops, "hot_word_ors": t["dense_hot_words"],
                         "popcount_words": t["dense_row_words"], "cold_scatters": t["dense_cold_entries"]}}
    else:
        nbytes = 12 * t["n_r_kept"] + 8 * t["n_x"] + 4 * t["sparse_join_rows"]
        achieved = nbytes / (sp_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_sparse_light/k_sparse_heavy (SparseBMM count)", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(args.workload),
                "kernel_ms": sp_ms, "work": {"bytes": nbytes, "join_rows": t["sparse_join_rows"]}}

    out = {
        "metric": "distinct (x,z) pairs/sec",
        "value": total / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator, inputs resident in HBM)",
        "config": dict(desc, pairs=total, dense_pairs=dense, sparse_pairs=sparse, tau=st["tau"],
                       n_z_dense=st["n_z_dense"], k_hot=st["k_hot"], out_j=st["out_j"],
                       input_tuples_per_s=(inst.n_r + inst.n_s) / (ms * 1e-3),
                       kernel_ms={"sparse": sp_ms, "dense": de_ms, "execute": ex_ms},
                       tau_tuned=None if tune is None else {"tau": tune["tau"], "model_tau": tune["model_tau"],
                                                            "dense_kernel": tune["dense_kernel"],
                                                            "k_hot_max": tune["k_hot_max"],
                                                            "window_group": tune["window_group"]}),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_sample_mod)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

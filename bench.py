#!/usr/bin/env python3
"""Throughput of the Householder-aligned permutation test on one MI355X.

Metric: permuted statistics per second at d = 768.  One step is one call of
the whole hot path (alignment, Philox splits, group-sum product, statistic,
FP64 recheck, p-values) over the batched workload, inputs resident in HBM:
512 pairs of synthetic clouds, d = 768, B = 2000 splits per pair, group
sizes log-uniform on [20, 5000], split-BF16 group sums.  The same workload
is also timed with plain FP32 group sums (the comparison in the metric).

Prints one JSON line.  ``roofline`` is the group-sum kernel (the dominant
kernel) timed with HIP events on the library's stream; ``cpu_baseline`` is
the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 MFMA
INT8_PEAK_TOPS = 5000.0     # MI355X dense int8 MFMA
STAGES = ["align", "split", "groupsum", "stat", "recheck", "other", "centroid"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ["groupsum.hip", "hbt_internal.h"]:
        h.update((ROOT / "paper_2605_08048_amd" / "csrc" / f).read_bytes())
    return h.hexdigest()[:16]


def load_traffic(name, launches_per_step):
    """HBM bytes per launch of the group-sum kernel from the committed
    rocprofv3 counter summary, or None when it is missing or stale."""
    f = ROOT / "profiles" / name
    if not f.exists():
        return None
    try:
        rec = json.loads(f.read_text())
    except ValueError:
        return None
    if rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


TRAFFIC_FILE = "groupsum_bf16x2_batch512_d768_traffic.json"
COPY_BYTES = 1 << 30        # the calibration copy: 1 GiB read, 1 GiB written


def counter_pass(args):
    """One warm and one measured call of the batched split-BF16 path, then a
    plain 1 GiB device copy whose byte counts calibrate the HBM counters.
    Meant to run under ``rocprofv3 --pmc FETCH_SIZE`` (then WRITE_SIZE)."""
    import torch
    from paper_2605_08048_amd import hbt, synth
    dev = torch.device("cuda:0")
    batch = synth.batch_512_d768()
    Z = torch.from_numpy(batch.Z).to(dev)
    res = torch.zeros(hbt.RESULT_BYTES * batch.npairs, dtype=torch.uint8, device=dev)
    for _ in range(2):
        hbt.perm_test_batched(Z, batch.row_offset, batch.n, batch.m, batch.B, seed=batch.seed,
                              precision=args.counter_precision, sync=False, results=res)
    torch.cuda.synchronize()
    log(f"batched {args.counter_precision} calls done")
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log("1 GiB calibration copy done")


def write_traffic(fetch_csv, write_csv, command):
    """HBM bytes per launch of k_groupsum_bf16x2 from two rocprofv3 counter
    runs, each counter scaled by what it reads for the 1 GiB copy."""
    import csv
    from collections import defaultdict

    def rows(path):
        """(kernel, counter, value, dispatch) from rocprofv3's CSV or SQLite output."""
        if str(path).endswith(".db"):
            import sqlite3
            q = "select kernel_name, counter_name, value, dispatch_id from counters_collection"
            yield from sqlite3.connect(path).execute(q)
        else:
            for r in csv.DictReader(open(path)):
                yield r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]), r["Dispatch_Id"]

    def per_dispatch(path, counter):
        acc = defaultdict(lambda: defaultdict(float))
        for kern, name, val, disp in rows(path):
            if name == counter:
                acc[kern][disp] += float(val)
        return {k: sum(v.values()) / len(v) for k, v in acc.items()}

    def pick(d, key):
        hits = [v for k, v in d.items() if key in k]
        if len(hits) != 1:
            raise SystemExit(f"expected one kernel matching {key!r}, found {len(hits)}")
        return hits[0]

    f = per_dispatch(fetch_csv, "FETCH_SIZE")
    w = per_dispatch(write_csv, "WRITE_SIZE")
    f_copy, w_copy = pick(f, "copyBuffer"), pick(w, "copyBuffer")       # KiB per dispatch
    f_gs, w_gs = pick(f, "k_groupsum_bf16x2"), pick(w, "k_groupsum_bf16x2")
    sf, sw = COPY_BYTES / (f_copy * 1024), COPY_BYTES / (w_copy * 1024)
    rec = {
        "kernel": "k_groupsum_bf16x2", "workload": "batch_512_d768",
        "kernel_hash": kernel_source_hash(),
        "fetch_kib_per_dispatch": f_gs, "write_kib_per_dispatch": w_gs,
        "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
        "fetch_scale": sf, "write_scale": sw,
        "hbm_read_bytes_per_launch": f_gs * 1024 * sf, "hbm_write_bytes_per_launch": w_gs * 1024 * sw,
        "hbm_bytes_per_launch": f_gs * 1024 * sf + w_gs * 1024 * sw,
        "command": command,
    }
    (ROOT / "profiles" / TRAFFIC_FILE).write_text(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec))


def stage_times(L, ctypes):
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int64 * len(STAGES))()
    st = L.hbt_stage_times(ms, n)
    if st != 0:
        raise RuntimeError(L.hbt_last_error().decode())
    return list(ms), list(n)


def host_cpu():
    """What the host offers this process: nproc, the CPUs it may run on, the
    thread budget set for the job (OMP_NUM_THREADS) and the CPU model."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "omp_num_threads": omp or None,
            "cpu_model": model}


def cpu_baseline(batch, npairs_sample=176, splits=2000):
    from oracle import oracle as O
    host = host_cpu()
    # every core the job may use: the CPUs of its affinity mask, within the
    # thread budget the host sets for one GPU's job (OMP_NUM_THREADS)
    threads = host["affinity_cpus"] or 1
    if host["omp_num_threads"]:
        threads = min(threads, host["omp_num_threads"])
    sample = sorted(set(np.linspace(0, batch.npairs - 1, npairs_sample).round().astype(int).tolist()))
    t0 = time.perf_counter()
    total = 0
    for p in sample:
        pr = batch.pair(p)
        r = O.perm_test(pr.X, pr.Y, splits, seed=batch.seed, pair=pr.pair_index, nthreads=threads)
        assert r["status"] in (0, O.ERR_DEGENERATE)
        total += splits
    dt = time.perf_counter() - t0
    # the same oracle on one thread, on every 16th pair of that sample
    t1 = time.perf_counter()
    total1 = 0
    for p in sample[::16]:
        pr = batch.pair(p)
        r = O.perm_test(pr.X, pr.Y, splits, seed=batch.seed, pair=pr.pair_index, nthreads=1)
        assert r["status"] in (0, O.ERR_DEGENERATE)
        total1 += splits
    dt1 = time.perf_counter() - t1
    return {"value": total / dt, "unit": "permuted statistics/s", "cores": threads, "kind": "oracle",
            "host": host,
            "sample": f"{len(sample)} pairs evenly spaced over the workload's 512 (sizes spread as in the "
                      f"whole batch), first {splits} splits each ({total} statistics, {dt:.1f} s wall, "
                      f"FP64 C oracle, OpenMP over splits on {threads} threads)",
            "single_thread": {"value": total1 / dt1, "cores": 1,
                              "sample": f"every 16th of those pairs, first {splits} splits each "
                                        f"({total1} statistics, {dt1:.1f} s wall)"}}


# The paper's own runtime figure (Table 4), context only: another workload
# (BCCWJ token embeddings from BERT-large, d = 1024, B = 20,000 per test),
# other hardware.
PAPER_CONTEXT = {
    "paper_speedup_gpu_over_cpu": 23.0,
    "paper_ms_per_permutation": {"cpu": 1.588, "gpu": 0.069},
    "paper_workload": "Table 4: BCCWJ embeddings from BERT-large (d = 1024), B = 20,000 permutations per test",
    "paper_hardware": "CPU model not named; GPU not named in the table, the compute-budget note names two NVIDIA H100s",
    "note": "context only: not this workload, not this hardware",
}


def stage_errors(dev, pair, hbt, torch, sample_every=97):
    """Error of each stage of the reduced precisions against the library's
    FP64 path on the same splits: the squared group-sum norms the product
    yields, the mean resultant lengths r1, r2 and T_b (before any recheck).
    The FP64 path itself matches the FP64 CPU oracle to 1e-10 in the tests."""
    X = torch.from_numpy(pair.X).to(dev)
    Y = torch.from_numpy(pair.Y).to(dev)
    runs = {prec: hbt.perm_test(X, Y, pair.B, seed=pair.seed, precision=prec, want_T="norms")["T"]
            for prec in ("f64", "f32", "bf16x2", "i8x3", "bf16e4m3")}
    # the point-to-centroid route (X S^T, K = d): FP32 MFMA, and split BF16 in three terms
    for prec in ("f32", "bf16x2"):
        runs[f"{prec}_point_to_centroid"] = hbt.perm_test(X, Y, pair.B, seed=pair.seed, precision=prec,
                                                          stat_route=1, want_T="norms")["T"]
    ref = runs.pop("f64")
    idx = np.arange(0, pair.B, sample_every)
    n, m, d = pair.n, pair.m, pair.d
    rel = lambda a, b: float(np.max(np.abs(a - b) / np.abs(b)))
    f = lambda r: np.log(r * (d - r * r) / (1 - r * r))
    r1r, r2r = np.sqrt(ref[idx, 1]) / n, np.sqrt(ref[idx, 2]) / m
    scale = np.abs(f(r1r)) + np.abs(f(r2r))
    out = {"workload": f"{pair.meta.get('workload')}: n {n}, m {m}, d {d}, B {pair.B}; {len(idx)} sampled splits",
           "reference": "the library's FP64 group sums (FP64 MFMA), same splits"}
    for prec, T in runs.items():
        r1, r2 = np.sqrt(T[idx, 1]) / n, np.sqrt(T[idx, 2]) / m
        out[prec] = {"sq_norm_rel_max": max(rel(T[idx, 1], ref[idx, 1]), rel(T[idx, 2], ref[idx, 2])),
                     "r_rel_max": max(rel(r1, r1r), rel(r2, r2r)),
                     "T_abs_max": float(np.max(np.abs(T[idx, 0] - ref[idx, 0]))),
                     "T_rel_to_scale_max": float(np.max(np.abs(T[idx, 0] - ref[idx, 0]) / scale))}
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--i8-steps", type=int, default=3, help="timed steps of the int8 digit-plane variant")
    ap.add_argument("--f8-steps", type=int, default=3, help="timed steps of the BF16 hi + e4m3 lo variant")
    ap.add_argument("--lazy-steps", type=int, default=3,
                    help="timed steps of the lazy split-BF16 precision (hi plane first, lo near the threshold)")
    ap.add_argument("--single-steps", type=int, default=5,
                    help="timed calls per precision of the single-pair workloads (0 skips them)")
    ap.add_argument("--cloud-steps", type=int, default=5,
                    help="timed calls of the shared-clouds workload and of its pairs stored apart (0 skips them)")
    ap.add_argument("--route2-steps", type=int, default=2,
                    help="timed steps of the point-to-centroid route (0 skips them)")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="timed replays of the split-BF16 call captured as a HIP graph (0 skips them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the (untimed) autotuning of the launch parameters")
    ap.add_argument("--counter-precision", default="bf16x2", help="precision of the --counter-pass calls")
    ap.add_argument("--counter-pass", action="store_true",
                    help="run the batched path twice and a 1 GiB copy, for rocprofv3 --pmc")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH", "WRITE"),
                    help="turn two rocprofv3 counter outputs (CSV or SQLite) into the committed traffic summary")
    ap.add_argument("--traffic-command", default="", help="the commands that produced the CSVs")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, args.traffic_command)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the permutation test would shard by split ranges: perm_offset, B).", file=sys.stderr)
        sys.exit(2)

    if args.counter_pass:
        counter_pass(args)
        return

    import ctypes
    import torch
    from paper_2605_08048_amd import hbt, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = time.perf_counter()
    batch = synth.batch_512_d768()
    Z = torch.from_numpy(batch.Z).to(dev)
    log(f"workload generated and resident in HBM ({time.perf_counter() - t:.1f} s, {Z.numel() * 4 / 1e9:.2f} GB)")
    P = batch.npairs
    N = (batch.n + batch.m).astype(np.int64)
    d = batch.d
    stats_per_step = int(batch.B.sum())
    algo_flops = float(2 * d * np.sum(batch.B * N))       # 2 N d per permuted statistic
    L = hbt.lib()
    tuning = None
    if not args.no_tune:
        # the autotuner (untimed): tile widths, persistent grids, split
        # work-groups per CU and pipeline chunks, per precision
        tuning = {}
        for prec in ("bf16x2", "i8x3", "bf16e4m3"):
            hbt.tune_batched(Z, batch.row_offset, batch.n, batch.m, batch.B, seed=batch.seed, precision=prec)
            tuning[prec] = hbt.tune_entry_get(prec, d)
        tuning["pairs_at_256"] = int(np.sum(hbt.tile_widths(batch.B, d) == 256))
        log(f"tuned: {tuning}")

    def run(prec, steps, warmup, stat_route=0):
        res = torch.zeros(hbt.RESULT_BYTES * P, dtype=torch.uint8, device=dev)
        for _ in range(warmup):
            hbt.perm_test_batched(Z, batch.row_offset, batch.n, batch.m, batch.B, seed=batch.seed,
                                  precision=prec, sync=False, results=res, stat_route=stat_route)
        torch.cuda.synchronize()
        L.hbt_stage_timing(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            hbt.perm_test_batched(Z, batch.row_offset, batch.n, batch.m, batch.B, seed=batch.seed,
                                  precision=prec, sync=False, results=res, stat_route=stat_route)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms, launches = stage_times(L, ctypes)
        L.hbt_stage_timing(0)
        out = hbt.results_to_numpy(res)
        bad = int(np.sum(out["status"] != 0))
        return (t1 - t0), ms, launches, out, bad

    dt, ms, launches, out, bad = run("bf16x2", args.steps, args.warmup)
    log(f"split-BF16: {dt / args.steps * 1e3:.2f} ms/step")
    value = stats_per_step * args.steps / dt
    g_ms = ms[2] / max(launches[2], 1)
    achieved = algo_flops / (g_ms * 1e-3) / 1e12
    traffic = load_traffic(TRAFFIC_FILE, 1)
    # the alignment stage (column sums, finalize, reflection + split-BF16
    # storage): algorithmic bytes = every row read once by the column sums, the
    # X rows read again by the reflection, and the two BF16 planes written
    nx = int(batch.n.sum())
    align_bytes = 4.0 * d * (N.sum() + nx) + 4.0 * d * N.sum()
    align_ms = ms[0] / args.steps
    align = {"ms_per_step": align_ms, "algorithmic_bytes": align_bytes,
             "hbm_gbs": align_bytes / (align_ms * 1e-3) / 1e9,
             "frac_hbm_peak": align_bytes / (align_ms * 1e-3) / 8.0e12}

    graph = None
    if args.graph_steps > 0:
        # the same call captured once into a HIP graph and replayed
        need = hbt.batched_workspace_size(batch.row_offset, batch.n, batch.m, batch.B, d, precision="bf16x2")
        gws = torch.empty(need, dtype=torch.uint8, device=dev)
        gres = torch.zeros(hbt.RESULT_BYTES * P, dtype=torch.uint8, device=dev)
        call = lambda: hbt.perm_test_batched(Z, batch.row_offset, batch.n, batch.m, batch.B, seed=batch.seed,
                                             precision="bf16x2", sync=False, results=gres, workspace=gws)
        call()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            call()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.graph_steps):
            g.replay()
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
        gout = hbt.results_to_numpy(gres)
        graph = {"ms_per_step": dtg / args.graph_steps * 1e3, "value": stats_per_step * args.graph_steps / dtg,
                 "steps": args.graph_steps,
                 "counts_equal_to_eager": bool(np.array_equal(gout["count"], out["count"]))}
        log(f"graph replay: {graph['ms_per_step']:.2f} ms/step")
        del g, gws

    fp = None
    if args.fp32_steps > 0:
        dt32, ms32, l32, out32, bad32 = run("f32", args.fp32_steps, 1)
        log(f"FP32: {dt32 / args.fp32_steps * 1e3:.2f} ms/step")
        v32 = stats_per_step * args.fp32_steps / dt32
        g32 = ms32[2] / max(l32[2], 1)
        agree = int(np.sum(out32["count"] == out["count"]))
        fp = {"value": v32, "ms_per_step": dt32 / args.fp32_steps * 1e3,
              "groupsum_ms": g32, "groupsum_tflops": algo_flops / (g32 * 1e-3) / 1e12,
              "groupsum_frac_fp32_peak": algo_flops / (g32 * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
              "speedup_bf16x2_over_fp32": value / v32,
              "pairs_with_equal_counts": f"{agree}/{P}",
              "kernel": "k_groupsum_fp<float>: v_mfma_f32_16x16x4f32, 64x64 wave tiles, operands loaded "
                        "from global memory without LDS staging (a comparison path, not tuned like the "
                        "split-BF16 kernel)"}

    i8 = None
    if args.i8_steps > 0:
        dt8, ms8, l8, out8, bad8 = run("i8x3", args.i8_steps, 1)
        log(f"int8 digit planes: {dt8 / args.i8_steps * 1e3:.2f} ms/step")
        g8 = ms8[2] / max(l8[2], 1)
        i8 = {"value": stats_per_step * args.i8_steps / dt8, "ms_per_step": dt8 / args.i8_steps * 1e3,
              "groupsum_ms": g8, "groupsum_tops": algo_flops / (g8 * 1e-3) / 1e12,
              "groupsum_frac_int8_peak": algo_flops / (g8 * 1e-3) / 1e12 / INT8_PEAK_TOPS,
              "stages_ms_per_step": {k: ms8[i] / args.i8_steps for i, k in enumerate(STAGES)},
              "rechecked_splits_per_step": int(out8["n_recheck"].sum()),
              "pairs_bad_status": bad8,
              "pairs_with_counts_equal_to_bf16x2": f"{int(np.sum(out8['count'] == out['count']))}/{P}"}

    f8 = None
    if args.f8_steps > 0:
        dtf, msf, lf, outf, badf = run("bf16e4m3", args.f8_steps, 1)
        log(f"BF16 hi + e4m3 lo: {dtf / args.f8_steps * 1e3:.2f} ms/step")
        gf = msf[2] / max(lf[2], 1)
        f8 = {"value": stats_per_step * args.f8_steps / dtf, "ms_per_step": dtf / args.f8_steps * 1e3,
              "groupsum_ms": gf, "groupsum_tflops": algo_flops / (gf * 1e-3) / 1e12,
              "groupsum_frac_bf16_peak": algo_flops / (gf * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
              "stages_ms_per_step": {k: msf[i] / args.f8_steps for i, k in enumerate(STAGES)},
              "rechecked_splits_per_step": int(outf["n_recheck"].sum()),
              "pairs_bad_status": badf,
              "pairs_with_counts_equal_to_bf16x2": f"{int(np.sum(outf['count'] == out['count']))}/{P}",
              "kernel": "k_groupsum_bf16x2<4, 8, false, 1>: bf16 MFMA on the hi plane, "
                        "v_mfma_scale_f32_32x32x64_f8f6f4 on the e4m3 lo plane, one FP32 accumulator"}

    lazy = None
    if args.lazy_steps > 0:
        dtl, msl, ll, outl, badl = run("bf16lazy", args.lazy_steps, 1)
        log(f"lazy split BF16: {dtl / args.lazy_steps * 1e3:.2f} ms/step")
        gl = msl[2] / args.lazy_steps  # both products of a call (hi plane, then the listed splits)
        lazy = {"value": stats_per_step * args.lazy_steps / dtl, "ms_per_step": dtl / args.lazy_steps * 1e3,
                "speedup_over_split_bf16": (stats_per_step * args.lazy_steps / dtl) / value,
                "groupsum_ms_per_step": gl, "groupsum_tflops": algo_flops / (gl * 1e-3) / 1e12,
                "groupsum_frac_bf16_peak": algo_flops / (gl * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                "stages_ms_per_step": {k: msl[i] / args.lazy_steps for i, k in enumerate(STAGES)},
                "rechecked_splits_per_step": int(outl["n_recheck"].sum()),
                "pairs_bad_status": badl,
                "pairs_with_counts_equal_to_bf16x2": f"{int(np.sum(outl['count'] == out['count']))}/{P}",
                "pairs_with_n_recheck_equal_to_bf16x2":
                    f"{int(np.sum(outl['n_recheck'] == out['n_recheck']))}/{P}",
                "kernels": "k_groupsum_bf16x2<4, 8, false, 2> (hi plane, every split), then "
                           "k_groupsum_bf16x2<2, 4, false, 3> (both planes, the splits within the hi "
                           "plane's error band of the threshold)"}

    # single-pair workloads (the per-pair call), every precision on the same input
    single = None
    if args.single_steps > 0:
        single = {}
        for name, pair in (("pair_d768", synth.pair_d768()), ("null_pair_d1024", synth.null_pair_d1024())):
            X = torch.from_numpy(pair.X).to(dev)
            Y = torch.from_numpy(pair.Y).to(dev)
            row = {"n": pair.n, "m": pair.m, "d": pair.d, "B": pair.B}
            counts = {}
            for prec in ("f32", "bf16x2", "i8x3", "bf16e4m3", "bf16lazy"):
                call = lambda: hbt.perm_test(X, Y, pair.B, seed=pair.seed, precision=prec, sync=False)
                call()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.single_steps):
                    r = call()
                torch.cuda.synchronize()
                dt1 = (time.perf_counter() - t0) / args.single_steps
                res = hbt.results_to_numpy(r["result"])[0]
                counts[prec] = int(res["count"])
                row[prec] = {"ms_per_call": dt1 * 1e3, "value": pair.B / dt1, "count": int(res["count"]),
                             "p": float(res["p"]), "n_recheck": int(res["n_recheck"]),
                             "status": int(res["status"])}
            row["speedup_bf16x2_over_f32"] = row["f32"]["ms_per_call"] / row["bf16x2"]["ms_per_call"]
            row["counts_equal"] = len(set(counts.values())) == 1
            single[name] = row
            log(f"single pair {name}: " + ", ".join(f"{k} {row[k]['ms_per_call']:.3f} ms" for k in counts))

    # the point-to-centroid route (statistic route 1 of the ABI): the same
    # workloads with the norms reduced from Q = Z S^T
    route2 = None
    if args.route2_steps > 0:
        route2 = {}
        centroid_flops = lambda n, m, B: 2.0 * (n + m) * d * B  # Q = Z S^T, K = d
        for prec in ("bf16x2", "f32"):
            dt2, ms2, l2, out2, bad2 = run(prec, args.route2_steps, 1, stat_route=1)
            c_ms = ms2[6] / args.route2_steps
            route2[f"batch_512_{prec}"] = {
                "ms_per_step": dt2 / args.route2_steps * 1e3, "value": stats_per_step * args.route2_steps / dt2,
                "centroid_ms": c_ms, "centroid_tflops": algo_flops / (c_ms * 1e-3) / 1e12,
                "pairs_with_counts_equal_to_route0": f"{int(np.sum(out2['count'] == out['count']))}/{P}"
                if prec == "bf16x2" else None,
                "pairs_bad_status": bad2}
            log(f"route 2 batched {prec}: {route2[f'batch_512_{prec}']['ms_per_step']:.2f} ms/step, "
                f"centroid {c_ms:.2f} ms")
        pair = synth.pair_d768()
        X = torch.from_numpy(pair.X).to(dev)
        Y = torch.from_numpy(pair.Y).to(dev)
        for prec in ("bf16x2", "f32"):
            call = lambda: hbt.perm_test(X, Y, pair.B, seed=pair.seed, precision=prec, stat_route=1, sync=False)
            call()
            torch.cuda.synchronize()
            L.hbt_stage_timing(1)
            t0 = time.perf_counter()
            for _ in range(args.route2_steps):
                r = call()
            torch.cuda.synchronize()
            dt1 = (time.perf_counter() - t0) / args.route2_steps
            ms1, _ = stage_times(L, ctypes)
            L.hbt_stage_timing(0)
            c_ms = ms1[6] / args.route2_steps
            res = hbt.results_to_numpy(r["result"])[0]
            route2[f"pair_d768_{prec}"] = {
                "ms_per_call": dt1 * 1e3, "value": pair.B / dt1, "centroid_ms": c_ms,
                "centroid_tflops": centroid_flops(pair.n, pair.m, pair.B) / (c_ms * 1e-3) / 1e12,
                "count": int(res["count"]), "status": int(res["status"])}
            log(f"route 2 pair_d768 {prec}: {dt1 * 1e3:.3f} ms/call, centroid {c_ms:.3f} ms")

    # shared clouds: the same kind of batch with each word's cloud in many
    # pairs, stored once (Householder fold), against the batched call on the
    # same pairs stored pair by pair
    clouds = None
    if args.cloud_steps > 0:
        wc = synth.word_clouds(d=d)
        pb = wc.pairs_batch()
        Zc = torch.from_numpy(wc.Z).to(dev)
        Zp = torch.from_numpy(pb.Z).to(dev)
        rc_res = torch.zeros(hbt.RESULT_BYTES * len(wc.B), dtype=torch.uint8, device=dev)
        rb_res = torch.zeros_like(rc_res)
        c_call = lambda: hbt.perm_test_clouds(Zc, wc.offset, wc.rows, wc.pair_x, wc.pair_y, wc.B, seed=wc.seed,
                                              sync=False, results=rc_res)
        b_call = lambda: hbt.perm_test_batched(Zp, pb.row_offset, pb.n, pb.m, pb.B, seed=pb.seed, sync=False,
                                               results=rb_res)
        timing = {}
        for name, call in (("clouds", c_call), ("batched", b_call)):
            call()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.cloud_steps):
                call()
            torch.cuda.synchronize()
            timing[name] = (time.perf_counter() - t0) / args.cloud_steps * 1e3
        oc, ob = hbt.results_to_numpy(rc_res), hbt.results_to_numpy(rb_res)
        nst = int(wc.B.sum())
        clouds = {"workload": f"word_clouds: {len(wc.rows)} word clouds (n log-uniform [20, 5000]), "
                              f"{len(wc.B)} pairs of distinct words, d={d}, B=2000",
                  "ms_per_call_shared_clouds": timing["clouds"], "ms_per_call_pairs_stored_apart": timing["batched"],
                  "value_shared_clouds": nst / (timing["clouds"] * 1e-3),
                  "rows_stored_shared": int(wc.rows.sum()), "rows_stored_apart": int(pb.Z.shape[0]),
                  "pairs_with_equal_counts": f"{int(np.sum(oc['count'] == ob['count']))}/{len(wc.B)}",
                  "pairs_bad_status": int(np.sum(oc["status"] != 0))}
        log(f"shared clouds: {timing['clouds']:.2f} ms/call vs {timing['batched']:.2f} ms stored apart")
        del Zc, Zp

    errors = None
    if args.single_steps > 0:
        errors = stage_errors(dev, synth.null_pair_d1024(), hbt, torch)
        log("stage errors at null_pair_d1024 done")

    line = {
        "metric": "permuted statistics/s at d=768 (batched split-BF16 MFMA; plain FP32 in fp32_plain)",
        "value": value,
        "unit": "permuted statistics/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "batch_512_d768: 512 pairs, d=768, B=2000 splits/pair, n,m log-uniform [20,5000], "
                               "split-BF16 group sums (hi+lo, FP32 accumulation), FP64 statistic + recheck",
                   "pairs": P, "d": d, "splits_per_step": stats_per_step, "rows": int(N.sum())},
        "roofline": {"bound": "mfma", "kernel": "k_groupsum_bf16x2", "achieved": achieved,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS,
                     "traffic": traffic,
                     "algorithmic_flops_per_launch": algo_flops, "avg_launch_ms": g_ms,
                     "executed_mfma_tflops": 2 * achieved},
        "whole_call": {"algorithmic_tflops": algo_flops / (dt / args.steps) / 1e12,
                       "frac_bf16_peak": algo_flops / (dt / args.steps) / 1e12 / BF16_PEAK_TFLOPS},
        "stages_ms_per_step": {k: ms[i] / args.steps for i, k in enumerate(STAGES)},
        "align_stage": align,
        "graph_replay": graph,
        "pairs_bad_status": bad,
        "rechecked_splits_per_step": int(out["n_recheck"].sum()),
        "fp32_plain": fp,
        "int8_planes": i8,
        "bf16_hi_e4m3_lo": f8,
        "lazy_split_bf16": lazy,
        "point_to_centroid": route2,
        "shared_clouds": clouds,
        "single_pair": single,
        "tuning": tuning,
        "stage_errors_null_pair_d1024": errors,
        "context": PAPER_CONTEXT,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(batch)
        log("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the Smith-Waterman CAL scorer on one MI355X.

Workload: the chromosome-scale plain configuration — a 100 Mbp synthetic
reference (uniform ACGT with 5% planted repeats), 1,000,000 reads of 100 bp
(1% substitutions, 0.1% indels), Poisson(6)+1 CALs per read drawn from the true
locus, repeat homologs and uniform decoys, window = read +/- 32 bp, both
strands, int16 dynamic programming.

One step is one pass of the whole scoring path over the batch with the
references already resident in HBM: 2-bit packing of the reads, CAL expansion,
the Gotoh sweep of every (CAL, strand) task, and the per-read, per-reference
best-score reduction.  GCUPS = sum over computed tasks of read length x
(clipped) window width, divided by the step time.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS + aligned reads/s (batched vs plain kernel); p50/p99 request latency"
ALIGNED_THRESHOLD = 40
OPS_PER_CELL = 12  # algorithmic integer ops per DP cell (E: 3, F: 3, substitution: 2, diagonal add: 1, H: 2, max: 1)
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 32-bit lane-ops/s; packed 16-bit ops do two per lane.
PEAK_INT16_TOPS = 256 * 64 * 2.4e9 * 2 / 1e12
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("sw_kernels.hip", "sw_device.h"):
        with open(os.path.join(ROOT, "paper_1805_00106_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(PROFILE_DIR, f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cells_of(batch) -> int:
    """Sum of L x W over the requested tasks (W clipped at the reference ends)."""
    r_of = np.repeat(np.arange(batch.n_reads), np.diff(batch.cal_ptr))
    L = batch.read_len[r_of].astype(np.int64)
    ref_len = batch.ref_len[batch.cal_ref.astype(np.int64)]
    band = batch.scoring.band
    W = np.minimum(ref_len, batch.cal_pos + L + band) - np.maximum(0, batch.cal_pos - band)
    nstr = ((batch.strand & 1) > 0).astype(np.int64) + ((batch.strand & 2) > 0).astype(np.int64)
    return int((L * W * nstr).sum())


def cpu_baseline(batch, target_s: float = 15.0):
    """Time the oracle (as it stands) on a bounded sample of the same workload."""
    from oracle import oracle as orc

    cores = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(12345)
    probe = batch.subset_reads(np.sort(rng.choice(batch.n_reads, 200, replace=False)))
    t0 = time.perf_counter()
    orc.align_batch(probe, n_threads=cores)
    rate = cells_of(probe) / max(time.perf_counter() - t0, 1e-6)
    n = int(min(batch.n_reads, max(200, 200 * target_s * rate / max(cells_of(probe), 1))))
    sample = batch.subset_reads(np.sort(rng.choice(batch.n_reads, n, replace=False)))
    t0 = time.perf_counter()
    orc.align_batch(sample, n_threads=cores)
    dt = time.perf_counter() - t0
    return {"value": round(cells_of(sample) / dt / 1e9, 3), "unit": "GCUPS", "cores": cores, "kind": "oracle",
            "sample": f"{n} of {batch.n_reads} reads ({sample.n_cals} CALs, both strands, "
                      f"{cells_of(sample):.3e} cells) in {dt:.1f} s",
            "reads_per_s": round(n / dt, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reads", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run an elementwise copy of this size (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the scoring path has no "
                                   "multi-GPU mode (reads shard across GPUs with no collective)"}))
        sys.exit(2)

    import torch

    import paper_1805_00106_amd as sw
    from paper_1805_00106_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    batch = wl.config2(n_reads=args.reads)
    t_gen = time.perf_counter() - t_gen
    sc = batch.scoring
    scoring = sw.Scoring.make(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band, sw.PREC_INT16,
                              sw.KERNEL_INTER, int(batch.read_len.max()))
    stream = torch.cuda.current_stream()

    # references resident in HBM (outside the timed region)
    refs = sw.RefSet.from_codes(torch.from_numpy(batch.ref_codes).to(dev), batch.ref_off, batch.ref_len)
    # inputs resident in HBM: read codes and CAL arrays
    read_codes = torch.from_numpy(batch.read_codes).to(dev)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
    db = sw.DeviceBatch(torch.empty((read_codes.numel() + 15) // 16, dtype=torch.int32, device=dev),
                        t(batch.read_off // 16, torch.int64), t(batch.read_len, torch.int32),
                        t(batch.cal_ptr, torch.int64), t(batch.cal_pos, torch.int64), t(batch.cal_ref, torch.int16),
                        t(batch.strand, torch.uint8))
    out = sw.Outputs(db.n_cals, dev)
    ws = torch.empty(sw.workspace_bytes(db.n_reads, db.n_cals, scoring), dtype=torch.uint8, device=dev)
    bs = torch.empty(db.n_reads * batch.n_refs, dtype=torch.int32, device=dev)
    bl = torch.empty(db.n_reads * batch.n_refs, dtype=torch.int64, device=dev)
    nt = torch.empty(db.n_reads * batch.n_refs, dtype=torch.int32, device=dev)
    L = sw.lib()
    import ctypes

    def step(k_events=None):
        rc = L.sw_pack_2bit(sw._ptr(read_codes), read_codes.numel(), sw._ptr(db.reads2bit), sw._stream(stream))
        assert rc == 0
        if k_events is not None:
            k_events[0].record(stream)
        sw.align_batch(db, refs, scoring, out, ws, stream)
        if k_events is not None:
            k_events[1].record(stream)
        rc = L.sw_reduce_best(sw._ptr(db.cal_ptr), sw._ptr(db.cal_ref), db.n_reads, batch.n_refs,
                              sw._ptr(out.score), sw._ptr(bs), sw._ptr(bl), sw._ptr(nt), sw._stream(stream))
        assert rc == 0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        step(ev[k])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / args.steps
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib * (1 << 18), dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    cells = cells_of(batch)
    gcups = cells / (step_ms * 1e-3) / 1e9
    best = bs.view(db.n_reads, batch.n_refs).max(dim=1).values
    aligned = float((best >= ALIGNED_THRESHOLD).float().mean().item())

    parity = None
    if not args.no_parity:
        from oracle import oracle as orc
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(batch.n_reads, min(300, batch.n_reads), replace=False))
        sub = batch.subset_reads(idx)
        s, r, e, _ = orc.align_batch(sub, n_threads=min(16, os.cpu_count() or 1))
        sel = np.concatenate([np.arange(batch.cal_ptr[i], batch.cal_ptr[i + 1]) for i in idx])
        slots = np.stack([2 * sel, 2 * sel + 1], 1).reshape(-1)
        gs, gr, ge = (out.score.cpu().numpy()[slots], out.ref_end.cpu().numpy()[slots],
                      out.read_end.cpu().numpy()[slots])
        parity = bool(np.array_equal(gs, s) and np.array_equal(gr, r) and np.array_equal(ge, e))

    achieved = OPS_PER_CELL * cells / (kern_ms * 1e-3) / 1e12
    traffic = load_traffic("inter16", "config2")
    roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_INT16_TOPS, 2),
            "unit": "Tops/s (int16 lane-ops)", "frac": round(achieved / PEAK_INT16_TOPS, 4), "traffic": traffic,
            "kernel": "k_inter16", "kernel_ms": round(kern_ms, 3),
            "kernel_gcups": round(cells / (kern_ms * 1e-3) / 1e9, 1),
            "gcups_peak": round(PEAK_INT16_TOPS * 1e12 / OPS_PER_CELL / 1e9, 1)}
    res = {
        "metric": METRIC, "value": round(gcups, 1), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int16", "data": "synthetic",
        "config": {"workload": "config2: 100 Mbp reference (5% planted repeats), 1M x 100 bp reads, "
                               "Poisson(6)+1 CALs/read, band 32, both strands, int16",
                   "reads": db.n_reads, "cals": db.n_cals, "tasks": 2 * db.n_cals, "cells": cells,
                   "path": "plain (one launch per batch)"},
        "reads_per_s": round(db.n_reads / (step_ms * 1e-3), 1),
        "aligned_fraction": round(aligned, 4), "aligned_threshold": ALIGNED_THRESHOLD,
        "wall_s_timed": round(wall, 3), "gen_s": round(t_gen, 1), "parity_sample_ok": parity,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(batch)
    print(json.dumps(res))


if __name__ == "__main__":
    main()

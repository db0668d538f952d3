"""Benchmark of the Smith-Waterman CAL scorer on one MI355X.

Workload: the chromosome-scale configuration — a 100 Mbp synthetic reference
(uniform ACGT with 5% planted repeats), 1,000,000 reads of 100 bp (1%
substitutions, 0.1% indels), Poisson(6)+1 CALs per read drawn from the true
locus, repeat homologs and uniform decoys, window = read +/- 32 bp, both
strands, int16 dynamic programming.

One step is one pass of the whole scoring path over the batch with the
references already resident in HBM: 2-bit packing of the reads, CAL expansion,
the Gotoh sweep of every (CAL, strand) task, and the per-read, per-reference
best-score reduction.  GCUPS = sum over computed tasks of read length x
(clipped) window width, divided by the step time.  The batched path (length
bins, persistent work queue, HIP graph) is the reported value; the plain path
(one launch per batch, static tiles) is timed on the same inputs beside it and
must give bit-identical outputs.  A second leg runs the uneven-length workload
(L uniform 75..250, geometric CAL counts) where binning matters.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import dataclasses
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
# The bound the scoring kernels reach: VALU instruction issue, one instruction per lane per cycle
# on every SIMD (256 CUs x 64 lanes x 2.4 GHz), packed or not.
ISSUE_PEAK = 256 * 64 * 2.4e9
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("sw_kernels.hip", "sw_device.h", "sw_halfmax.h", "sw_launch.h", "sw_lanes.h"):
        with open(os.path.join(ROOT, "paper_1805_00106_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def seeding_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("sw_index.hip", "sw_index.h", "sw_filter.hip", "sw_filter.h", "sw_seed.cpp"):
        with open(os.path.join(ROOT, "paper_1805_00106_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# The kernels of each seeding stage whose HBM bytes the traffic profile holds.
SEED_STAGE_KERNELS = {"index_build": ("k_index_seeds", "k_index_ptr"), "find": ("k_find_count", "k_find_write"),
                      "filter": ("k_filter_count_wave", "k_filter_write_wave")}


def load_seeding_traffic(workload: str = "chromosome_scale"):
    """Per-kernel HBM bytes of the seeding and filter kernels from the committed
    rocprofv3 counter summary, if it was taken on the current seeding source."""
    path = os.path.join(PROFILE_DIR, f"traffic_seeding_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != seeding_source_hash():
        return None
    return rec.get("kernels")


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


def load_issue(kernel: str, workload: str):
    """VALU instructions per cell pair and VALU busy fraction from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(PROFILE_DIR, f"valu_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


def profile_kernel(plan: str, int32: bool, final_row: bool) -> str:
    """Name of the counter profiles of the kernel a batched plan runs: the plain
    kernel where the tuner kept the plan without bins, else the queue kernel."""
    kind = "plain" if "unbinned" in plan else "queue"
    return f"inter{32 if int32 else 16}_{kind}" + ("_final_row" if final_row else "")


def roofline(kernel: str, workload: str, cells: int, kern_ms: float, packed: bool) -> dict:
    """VALU-issue roofline of one scoring kernel.  `achieved` = VALU lane-instructions
    the kernel issues per second: its lane-instructions per cell, from the rocprofv3
    counter profile taken on the current kernel source (SQ_INSTS_VALU x 64 / cells),
    times the cells, over the kernel time measured here; `peak` = one instruction
    per lane per cycle on every SIMD.  The 12-algorithmic-op view is kept apart: the
    kernels do those 12 ops in fewer instructions (one three-way maximum does a
    maximum and its clamp, one byte permutation gives both strands' substitution
    scores), so it is not a fraction of any peak."""
    rec = {"bound": "alu", "unit": "T VALU lane-instructions/s", "peak": round(ISSUE_PEAK / 1e12, 2),
           "kernel": kernel, "kernel_ms": round(kern_ms, 3),
           "kernel_gcups": round(cells / (kern_ms * 1e-3) / 1e9, 1)}
    v = load_issue(kernel, workload)
    if v:
        issued = v["lane_insts_per_cell"] * cells / (kern_ms * 1e-3)
        rec.update(achieved=round(issued / 1e12, 3), frac=round(issued / ISSUE_PEAK, 4),
                   lane_insts_per_cell=v["lane_insts_per_cell"], valu_busy_profiled=v.get("valu_busy"),
                   profile=f"profiles/valu_{kernel}_{workload}.json")
    else:
        rec.update(achieved=None, frac=None,
                   note="no VALU counter profile taken on the current kernel source")
    alg_peak = PEAK_INT16_TOPS if packed else PEAK_INT32_TOPS
    alg = OPS_PER_CELL * cells / (kern_ms * 1e-3) / 1e12
    rec["alg_ops_per_s"] = {"ops_per_cell": OPS_PER_CELL, "achieved_tops": round(alg, 2),
                            "published_int_peak_tops": round(alg_peak, 2), "ratio": round(alg / alg_peak, 4)}
    return rec


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

    # one oracle thread per host core this process may use, up to the 16 cores that
    # are one GPU's share of the host on this machine class
    nproc = os.cpu_count() or 1
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    cores = max(1, min(usable, 16))
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
    # one core on a smaller sample of the same reads (about a third of the time budget)
    n1 = int(min(n, max(20, n * (target_s / 3) / max(dt * cores, 1e-6))))
    one = batch.subset_reads(np.sort(rng.choice(batch.n_reads, n1, replace=False)))
    t0 = time.perf_counter()
    orc.align_batch(one, n_threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": round(cells_of(sample) / dt / 1e9, 3), "unit": "GCUPS", "cores": cores, "kind": "oracle",
            "nproc": nproc, "usable_cores": usable,
            "sample": f"{n} of {batch.n_reads} reads ({sample.n_cals} CALs, both strands, "
                      f"{cells_of(sample):.3e} cells) in {dt:.1f} s",
            "reads_per_s": round(n / dt, 1),
            "one_core": {"value": round(cells_of(one) / dt1 / 1e9, 3), "unit": "GCUPS",
                         "sample": f"{n1} reads ({cells_of(one):.3e} cells) in {dt1:.1f} s"}}


def parity_sample(batch, out, n=None, seed=7, final_row=False):
    """Compare a random sample of reads (default 1% of them, at least 300) against
    the oracle (not timed)."""
    from oracle import oracle as orc
    rng = np.random.default_rng(seed)
    if n is None:
        n = max(300, batch.n_reads // 100)
    idx = np.sort(rng.choice(batch.n_reads, min(n, batch.n_reads), replace=False))
    sub = batch.subset_reads(idx)
    s, r, e, _ = orc.align_batch(sub, n_threads=min(16, os.cpu_count() or 1), final_row=final_row)
    sel = np.concatenate([np.arange(batch.cal_ptr[i], batch.cal_ptr[i + 1]) for i in idx])
    slots = np.stack([2 * sel, 2 * sel + 1], 1).reshape(-1)
    gs, gr, ge = (out.score.cpu().numpy()[slots], out.ref_end.cpu().numpy()[slots],
                  out.read_end.cpu().numpy()[slots])
    return bool(np.array_equal(gs, s) and np.array_equal(gr, r) and np.array_equal(ge, e))


def small_reference_leg(reps=20):
    """The small-reference workload (1000 x 76 bp reads, 2 CALs each, both strands,
    int32): one plain call per kernel family, CALs and reads resident."""
    import torch
    import paper_1805_00106_amd as sw
    from paper_1805_00106_amd import workloads as wl
    b = wl.small_reference()
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    out = sw.Outputs(db.n_cals)
    cells = cells_of(b)
    res = {"reads": b.n_reads, "cals": b.n_cals, "cells": cells}
    outs = {}
    for name, kern in (("inter_int32", sw.KERNEL_INTER), ("intra_int32", sw.KERNEL_INTRA),
                       ("auto_int32", sw.KERNEL_AUTO)):
        sc = sw.Scoring.make(2, -3, 5, 2, 32, sw.PREC_INT32, kern, 76)
        ws = torch.empty(max(1, sw.workspace_bytes(db.n_reads, db.n_cals, sc)), dtype=torch.uint8, device="cuda")
        for _ in range(3):
            sw.align_batch(db, refs, sc, out, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            sw.align_batch(db, refs, sc, out, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"us": round(ms * 1e3, 1), "gcups": round(cells / (ms * 1e-3) / 1e9, 1),
                     "reads_per_s": round(b.n_reads / (ms * 1e-3), 1)}
        outs[name] = out.score.clone()
    res["same_outputs"] = bool(all(torch.equal(outs["inter_int32"], v) for v in outs.values()))
    return res


def small_batch_latency(batch, n_reads=24, reps=20):
    """Latency of one tiny plain call (a few reads' CALs) with each kernel family:
    one CAL per lane leaves most of the GPU idle and runs each alignment serially
    in one lane; one wavefront per task spreads each alignment over 64 lanes."""
    import torch
    import paper_1805_00106_amd as sw
    sub = batch.subset_reads(np.arange(n_reads))
    refs = sw.RefSet.from_codes(torch.from_numpy(sub.ref_codes).cuda(), sub.ref_off, sub.ref_len)
    db = sw.DeviceBatch.upload(sub)
    out = sw.Outputs(db.n_cals)
    res = {"reads": n_reads, "cals": sub.n_cals}
    results = {}
    for name, kern, prec in (("inter_int16", sw.KERNEL_INTER, sw.PREC_INT16),
                             ("inter_int32", sw.KERNEL_INTER, sw.PREC_INT32),
                             ("intra_int16", sw.KERNEL_INTRA, sw.PREC_INT16),
                             ("intra_int32", sw.KERNEL_INTRA, sw.PREC_INT32),
                             ("auto", sw.KERNEL_AUTO, sw.PREC_AUTO)):
        sc = sw.Scoring.make(2, -3, 5, 2, 32, prec, kern, 100)
        ws = torch.empty(max(1, sw.workspace_bytes(db.n_reads, db.n_cals, sc)), dtype=torch.uint8, device="cuda")
        for _ in range(3):
            sw.align_batch(db, refs, sc, out, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            sw.align_batch(db, refs, sc, out, ws)
        e1.record()
        torch.cuda.synchronize()
        res[name + "_us"] = round(e0.elapsed_time(e1) / reps * 1e3, 1)
        results[name] = out.score.clone()
    res["same_outputs"] = bool(all(torch.equal(results["inter_int16"], v) for v in results.values()))
    return res


class Leg:
    """One workload resident on the GPU, timed on the plain and the batched path."""

    def __init__(self, batch, max_read_len, steps, warmup):
        import torch
        import paper_1805_00106_amd as sw
        self.torch, self.sw = torch, sw
        self.batch, self.steps, self.warmup = batch, steps, warmup
        dev = torch.device("cuda:0")
        sc = batch.scoring
        self.scoring = sw.Scoring.make(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band, sw.PREC_INT16,
                                       sw.KERNEL_INTER, max_read_len)
        self.stream = torch.cuda.current_stream()
        # references resident in HBM (outside the timed region)
        self.refs = sw.RefSet.from_codes(torch.from_numpy(batch.ref_codes).to(dev), batch.ref_off, batch.ref_len)
        # inputs resident in HBM: read codes and CAL arrays
        self.read_codes = torch.from_numpy(batch.read_codes).to(dev)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
        self.db = sw.DeviceBatch(torch.empty((self.read_codes.numel() + 15) // 16, dtype=torch.int32, device=dev),
                                 t(batch.read_off // 16, torch.int64), t(batch.read_len, torch.int32),
                                 t(batch.cal_ptr, torch.int64), t(batch.cal_pos, torch.int64),
                                 t(batch.cal_ref, torch.int16), t(batch.strand, torch.uint8))
        db = self.db
        self.out = sw.Outputs(db.n_cals, dev)
        self.ws = torch.empty(sw.workspace_bytes(db.n_reads, db.n_cals, self.scoring), dtype=torch.uint8, device=dev)
        self.bs = torch.empty(db.n_reads * batch.n_refs, dtype=torch.int32, device=dev)
        self.bl = torch.empty(db.n_reads * batch.n_refs, dtype=torch.int64, device=dev)
        self.nt = torch.empty(db.n_reads * batch.n_refs, dtype=torch.int32, device=dev)
        self.ctx = sw.Context(db.n_reads, db.n_cals)
        self.cells = cells_of(batch)
        self.parity_reads = True

    def step(self, batched, k_events=None):
        sw, db, L, st = self.sw, self.db, self.sw.lib(), self.stream
        assert L.sw_pack_2bit(sw._ptr(self.read_codes), self.read_codes.numel(), sw._ptr(db.reads2bit),
                              sw._stream(st)) == 0
        if k_events is not None:
            k_events[0].record(st)
        if batched:
            self.ctx.align(db, self.refs, self.scoring, self.out, st)
        else:
            sw.align_batch(db, self.refs, self.scoring, self.out, self.ws, st)
        if k_events is not None:
            k_events[1].record(st)
        assert L.sw_reduce_best(sw._ptr(db.cal_ptr), sw._ptr(db.cal_ref), db.n_reads, self.batch.n_refs, db.n_cals,
                                sw._ptr(self.out.score), sw._ptr(self.bs), sw._ptr(self.bl), sw._ptr(self.nt),
                                sw._stream(st)) == 0

    def timed(self, batched):
        torch = self.torch
        for _ in range(self.warmup):
            self.step(batched)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(self.steps)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(self.stream)
        for k in range(self.steps):
            self.step(batched, ev[k])
        e1.record(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / self.steps, float(np.mean([a.elapsed_time(b) for a, b in ev])), wall

    def run(self):
        torch = self.torch
        plain_ms, plain_kern, _ = self.timed(False)
        plain = (self.out.score.clone(), self.out.ref_end.clone(), self.out.read_end.clone())
        batched_ms, batched_kern, wall = self.timed(True)
        same = bool(torch.equal(plain[0], self.out.score) and torch.equal(plain[1], self.out.ref_end)
                    and torch.equal(plain[2], self.out.read_end))
        best = self.bs.view(self.db.n_reads, self.batch.n_refs).max(dim=1).values
        aligned = float((best >= ALIGNED_THRESHOLD).float().mean().item())
        g = lambda ms: round(self.cells / (ms * 1e-3) / 1e9, 1)
        return {"plain_ms": plain_ms, "plain_kern_ms": plain_kern, "batched_ms": batched_ms,
                "batched_kern_ms": batched_kern, "wall": wall, "plain_gcups": g(plain_ms),
                "batched_gcups": g(batched_ms), "plain_equals_batched": same, "aligned_fraction": aligned,
                "plan": self.ctx.last_plan()}

    def end_to_end(self, steps=3):
        """Whole-batch rate with the PCIe transfers in the timed region: read codes
        and CAL arrays uploaded from pinned host memory, the batched path, and every
        output (slots and per-read best) downloaded to pinned host memory."""
        torch, sw, db, b = self.torch, self.sw, self.db, self.batch
        pin = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).pin_memory()
        ups = [(pin(b.read_codes, torch.uint8), self.read_codes), (pin(b.read_off // 16, torch.int64), db.read_word_off),
               (pin(b.read_len, torch.int32), db.read_len), (pin(b.cal_ptr, torch.int64), db.cal_ptr),
               (pin(b.cal_pos, torch.int64), db.cal_pos), (pin(b.cal_ref, torch.int16), db.cal_ref),
               (pin(b.strand, torch.uint8), db.strand)]
        downs = [(torch.empty_like(t, device="cpu").pin_memory(), t)
                 for t in (self.out.score, self.out.ref_end, self.out.read_end, self.bs, self.bl, self.nt)]
        nbytes = sum(h.numel() * h.element_size() for h, _ in ups + downs)

        def step():
            with torch.cuda.stream(self.stream):
                for h, d in ups:
                    d.copy_(h, non_blocking=True)
            self.step(True)
            with torch.cuda.stream(self.stream):
                for h, d in downs:
                    h.copy_(d, non_blocking=True)

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        return {"ms_per_step": round(ms, 3), "reads_per_s": round(db.n_reads / (ms * 1e-3), 1),
                "gcups": round(self.cells / (ms * 1e-3) / 1e9, 1), "pcie_bytes_per_step": nbytes,
                "note": "inputs from and outputs to pinned host memory inside the timed region"}

    def variants(self, steps=5):
        """The same resident chromosome-scale batch on the batched path with other
        scorings: int32 values (one strand per lane, the precision of the
        small-reference workload) and the final-row mode (int16).  Outputs are checked against the
        oracle on a read sample (not timed)."""
        torch, sw = self.torch, self.sw
        sc = self.batch.scoring
        res = {}
        measured = {"int32": sw.alu_peak(32) / 1e12, "final_row_int16": sw.alu_peak(16) / 1e12}
        for name, prec, mode in (("int32", sw.PREC_INT32, sw.MODE_LOCAL),
                                 ("final_row_int16", sw.PREC_INT16, sw.MODE_FINAL_ROW)):
            scv = sw.Scoring.make(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band, prec,
                                  sw.KERNEL_INTER, self.scoring.max_read_len, mode)
            out = sw.Outputs(self.db.n_cals, self.db.read_len.device)
            for _ in range(2):
                self.ctx.align(self.db, self.refs, scv, out, self.stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(self.stream)
            for _ in range(steps):
                self.ctx.align(self.db, self.refs, scv, out, self.stream)
            e1.record(self.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            gcups = self.cells / (ms * 1e-3) / 1e9
            plan = self.ctx.last_plan()
            kern = profile_kernel(plan, prec == sw.PREC_INT32, mode == sw.MODE_FINAL_ROW)
            res[name] = {"ms_per_step": round(ms, 3), "gcups": round(gcups, 1),
                         "roofline": roofline(kern, "chromosome_scale", self.cells, ms, prec != sw.PREC_INT32),
                         "peak_measured_tops": round(measured[name], 2),
                         "plan": plan}
            if self.parity_reads:
                res[name]["parity_sample_ok"] = parity_sample(self.batch, out,
                                                              final_row=mode == sw.MODE_FINAL_ROW)
        return res

    def traceback(self, reps=5, cap=64, parity_reads=200):
        """Start + CIGAR of every read's best slot (from the last scoring step's
        outputs), timed with HIP events on the leg's stream."""
        torch, sw, db = self.torch, self.sw, self.db
        slots = self.bl.view(db.n_reads, self.batch.n_refs)[:, 0].contiguous()
        n = slots.numel()
        dev = slots.device
        rs = torch.empty(n, dtype=torch.int64, device=dev)
        qs = torch.empty(n, dtype=torch.int16, device=dev)
        nops = torch.empty(n, dtype=torch.int32, device=dev)
        cig = torch.zeros(n * cap, dtype=torch.int32, device=dev)
        nb = sw.lib().sw_traceback_workspace_bytes(n, db.n_cals, ctypes.byref(self.scoring))
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        st = self.stream
        P = sw._ptr

        def call():
            rc = sw.lib().sw_traceback(P(db.reads2bit), P(db.read_word_off), P(db.read_len), db.n_reads, self.refs.c,
                                       P(db.cal_ptr), P(db.cal_pos), P(db.cal_ref), db.n_cals,
                                       ctypes.byref(self.scoring), P(self.out.score), P(self.out.ref_end),
                                       P(self.out.read_end), P(slots), n, cap, P(rs), P(qs), P(nops), P(cig),
                                       P(ws), nb, sw._stream(st))
            assert rc == 0, rc

        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            call()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # cells of the rebuilt rectangles: (read_end + 1) x (ref_end - window start + 1)
        ok = slots >= 0
        sl = slots.clamp(min=0)
        ws0 = (db.cal_pos[sl >> 1] - self.batch.scoring.band).clamp(min=0)
        rect = (self.out.read_end[sl].to(torch.int64) + 1) * (self.out.ref_end[sl] - ws0 + 1)
        cells = int(torch.where(ok & (self.out.score[sl] > 0), rect, torch.zeros_like(rect)).sum().item())
        res = {"reads": n, "ms": round(ms, 3), "reads_per_s": round(n / (ms * 1e-3), 1),
               "rectangle_cells": cells, "rectangle_gcups": round(cells / (ms * 1e-3) / 1e9, 1),
               "traced_fraction": round(float((nops > 0).float().mean().item()), 4),
               "kernel": ("one slot per wavefront" if self.scoring.kernel == sw.KERNEL_INTRA else
                          "slots per lane (two per lane in int16 halves where that layout holds)"),
               "workspace_mb": round(nb / 2**20, 1)}
        # the other kernel family (one traced slot per wavefront) on the same slots: time and agreement
        sc = self.scoring
        scw = sw.Scoring.make(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band, sc.precision,
                              sw.KERNEL_INTRA, sc.max_read_len)
        nbw = sw.lib().sw_traceback_workspace_bytes(n, db.n_cals, ctypes.byref(scw))
        wsw = torch.empty(max(nbw, 1), dtype=torch.uint8, device=dev)
        rs2, qs2, nops2 = torch.empty_like(rs), torch.empty_like(qs), torch.empty_like(nops)
        cig2 = torch.zeros_like(cig)

        def call_wave():
            rc = sw.lib().sw_traceback(P(db.reads2bit), P(db.read_word_off), P(db.read_len), db.n_reads, self.refs.c,
                                       P(db.cal_ptr), P(db.cal_pos), P(db.cal_ref), db.n_cals, ctypes.byref(scw),
                                       P(self.out.score), P(self.out.ref_end), P(self.out.read_end), P(slots), n, cap,
                                       P(rs2), P(qs2), P(nops2), P(cig2), P(wsw), nbw, sw._stream(st))
            assert rc == 0, rc

        call_wave()
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(2):
            call_wave()
        e1.record(st)
        torch.cuda.synchronize()
        res["wavefront_per_slot_ms"] = round(e0.elapsed_time(e1) / 2, 3)
        res["kernels_agree"] = bool(torch.equal(rs, rs2) and torch.equal(qs, qs2) and torch.equal(nops, nops2)
                                    and torch.equal(cig, cig2))
        del wsw
        if parity_reads:
            res["parity_sample_ok"] = self._trace_parity(slots, rs, qs, nops, cig.view(n, cap), cap, parity_reads)
        return res

    def pipeline(self, seed_len=22, stride=1, limit=16, reps=3):
        """The whole method on the device: seed index of the resident reference
        (built once), CALs from every overlapping seed of every read, the CAL
        filter (exact duplicates), Smith-Waterman on the kept CALs and the
        per-read best.  Stage times are wall-clock between device
        synchronisations (the finder and the filter each read one count back)."""
        torch, sw, db = self.torch, self.sw, self.db
        sync = torch.cuda.synchronize
        sync()
        t0 = time.perf_counter()
        ix = sw.SeedIndex(self.refs, seed_len=seed_len)
        sync()
        build_s = time.perf_counter() - t0
        times = {"find": [], "filter": [], "score": [], "reduce": []}
        for _ in range(reps):
            t = time.perf_counter()
            found = ix.find(db, stride=stride, max_cals_per_seed=limit, max_read_len=int(self.batch.read_len.max()))
            sync()
            times["find"].append(time.perf_counter() - t)
            t = time.perf_counter()
            kept, cmap = sw.cal_filter(found, 0)
            sync()
            times["filter"].append(time.perf_counter() - t)
            t = time.perf_counter()
            ws = torch.empty(sw.workspace_bytes(db.n_reads, kept.n_cals, self.scoring), dtype=torch.uint8,
                             device=db.read_len.device)
            out = sw.align_batch(kept, self.refs, self.scoring, None, ws)
            sync()
            times["score"].append(time.perf_counter() - t)
            t = time.perf_counter()
            bs, bl, nt = sw.reduce_best(kept, self.batch.n_refs, out.score)
            sync()
            times["reduce"].append(time.perf_counter() - t)
        ms = {k: round(1e3 * float(np.median(v)), 3) for k, v in times.items()}
        total_ms = sum(ms.values())
        # planted locus recovered: best CAL within 8 bases of the sampled position, right strand
        b = self.batch
        best = bl[:, 0].cpu().numpy()
        kpos = kept.cal_pos.cpu().numpy()
        okb = best >= 0
        hit = okb & (np.abs(kpos[np.maximum(best, 0) // 2] - b.true_pos) <= 8) & \
            ((best % 2 == 1) == np.asarray(b.true_strand, bool))
        info = ix.info()
        ix.close()
        # HBM rate of each stage: its kernels' bytes (from the counter profile) over its time here
        traffic = load_seeding_traffic()
        gbps = None
        if traffic:
            gbps = {}
            for stage, kernels in SEED_STAGE_KERNELS.items():
                nbytes = sum(traffic[k]["fetch_bytes"] + traffic[k]["write_bytes"] for k in kernels if k in traffic)
                t_s = build_s if stage == "index_build" else ms[stage] * 1e-3
                gbps[stage] = round(nbytes / t_s / 1e9, 1)
        return {"seed_len": seed_len, "stride": stride, "max_cals_per_seed": limit,
                "hbm_gbps": gbps, "hbm_note": "bytes of each stage's own kernels (counter profile) over its "
                                              "wall time between synchronisations; peak 8000 GB/s",
                "index_build_s": round(build_s, 3), "index_entries": info["entries"],
                "index_gb": round(info["device_bytes"] / 1e9, 3),
                "raw_cals": found.n_cals, "kept_cals": kept.n_cals,
                "stage_ms": ms, "total_ms": round(total_ms, 3),
                "reads_per_s": round(db.n_reads / (total_ms * 1e-3), 1),
                "planted_locus_recovered": round(float(hit.mean()), 4)}

    def _trace_parity(self, slots, rs, qs, nops, cig, cap, n, seed=11):
        from oracle import oracle as orc
        b = self.batch
        rng = np.random.default_rng(seed)
        idx = np.sort(rng.choice(b.n_reads, min(n, b.n_reads), replace=False))
        sub = b.subset_reads(idx)
        s, r, e, _ = orc.align_batch(sub, n_threads=min(16, os.cpu_count() or 1))
        _, bl, _ = orc.reduce_best(sub.cal_ptr, sub.cal_ref, sub.n_reads, sub.n_refs, s)
        ors, oqs, onops, ocig = orc.traceback(sub, s, r, e, bl[:, 0], cap=cap)
        g = lambda t: t.cpu().numpy()[idx]
        gcig = cig.cpu().numpy().view(np.uint32)[idx]
        # the sub-batch renumbers slots, so compare the traced alignments themselves
        return bool(np.array_equal(g(rs), ors) and np.array_equal(g(qs), oqs) and np.array_equal(g(nops), onops)
                    and np.array_equal(gcig, ocig))

    def free(self):
        self.ctx.close()


def classification_leg(n_reads: int, threshold: int = ALIGNED_THRESHOLD, parity: bool = True):
    """Two references (A random, B = A diverged by 15% substitutions and
    2%/base indels); reads 70/30 from B/A; each read goes to the reference with
    the strictly higher best score (section 6.2).  Reports the outcome fractions
    against the planted source and the scoring throughput."""
    import torch
    import paper_1805_00106_amd as sw
    from paper_1805_00106_amd import workloads as wl

    t_gen = time.perf_counter()
    b = wl.two_references(n_reads=n_reads)
    t_gen = time.perf_counter() - t_gen
    leg = Leg(b, 150, 3, 1)
    cls_t = torch.empty(b.n_reads, dtype=torch.int32, device="cuda")
    for _ in range(2):
        leg.step(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(leg.stream)
    leg.step(True)
    assert sw.lib().sw_classify(sw._ptr(leg.bs), b.n_reads, b.n_refs, threshold, sw._ptr(cls_t),
                                sw._stream(leg.stream)) == 0
    e1.record(leg.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cls = cls_t.cpu().numpy()
    truth = b.true_ref
    frac = lambda m: round(float(np.mean(m)), 5)
    # the threshold against the scores decoy CALs reach (uniform positions, no homology) and
    # the scores of the planted loci: T must sit above the first and below the second
    p4 = parity_sample(b, leg.out) if parity else None
    score = leg.out.score.cpu().numpy().reshape(-1, 2).max(axis=1)
    r_of = np.repeat(np.arange(b.n_reads), np.diff(b.cal_ptr))
    best_decoy = np.full(b.n_reads, -1, np.int64)
    best_true = np.full(b.n_reads, -1, np.int64)
    dmask = b.cal_decoy.astype(bool)
    np.maximum.at(best_decoy, r_of[dmask], score[dmask])
    np.maximum.at(best_true, r_of[~dmask], score[~dmask])
    pct = lambda a, q: int(np.percentile(a, q))
    out = {"workload": f"two references: A = {int(b.ref_len[0]):,} bp random, B = A + 15% substitutions + 2%/base indels "
                       f"({int(b.ref_len[1]):,} bp); {b.n_reads:,} reads of 150 bp, 70% from B / 30% from A, "
                       "1% substitutions; homologous locus + Poisson(2) decoys per reference; band 32; both strands",
           "threshold": threshold, "cals": b.n_cals, "cells": leg.cells,
           "ms_per_step": round(ms, 3), "gcups": round(leg.cells / (ms * 1e-3) / 1e9, 1),
           "reads_per_s": round(b.n_reads / (ms * 1e-3), 1),
           "correct": frac(cls == truth), "incorrect": frac((cls >= 0) & (cls != truth)),
           "tie": frac(cls == -2), "unaligned": frac(cls == -1),
           "by_source": {src: {"correct": frac(cls[truth == k] == k), "tie": frac(cls[truth == k] == -2),
                               "unaligned": frac(cls[truth == k] == -1)} for k, src in ((0, "A"), (1, "B"))},
           "decoy_best_score": {"p50": pct(best_decoy, 50), "p99": pct(best_decoy, 99),
                                "p99.9": pct(best_decoy, 99.9), "max": int(best_decoy.max()),
                                "reads_at_or_above_threshold": frac(best_decoy >= threshold)},
           "homologous_best_score": {"p0.1": pct(best_true, 0.1), "p1": pct(best_true, 1), "p50": pct(best_true, 50)},
           "parity_sample_ok": p4, "gen_s": round(t_gen, 1)}
    leg.free()
    return out


def sat_reads_of(pool, rounds, dt):
    return rounds * sum(b.n_reads for b in pool) / dt


def served_leg(scale: float, pool_size: int, per_load: int, loads=(0.3, 0.6, 0.9), step_cals: int = 1 << 20,
               parity_requests: int = 24, depth: int = 0):
    """Served requests: two resident references, Poisson arrivals of log-uniform request
    sizes, p50/p99 latency (scheduled arrival -> completion) at three loads
    relative to the measured saturated throughput."""
    import threading
    import torch
    import paper_1805_00106_amd as sw
    from paper_1805_00106_amd import workloads as wl

    t_gen = time.perf_counter()
    pack = wl.served_reference_pack(scale=scale, progress=progress)
    refs = [pack[0][int(o):int(o) + int(n)] for o, n in zip(pack[1], pack[2])]  # views, no second copy
    codes = torch.from_numpy(pack[0]).cuda()
    rs = sw.RefSet.from_codes(codes, pack[1], pack[2])
    torch.cuda.synchronize()
    del codes
    torch.cuda.empty_cache()
    _, sizes = wl.served_arrivals(1.0, pool_size, seed=0)
    pool = [wl.served_request(refs, int(n), 10_000 + k, ref_pack=pack) for k, n in enumerate(sizes)]
    pool_cells = [cells_of(b) for b in pool]
    t_gen = time.perf_counter() - t_gen
    progress(f"served: references resident, pool of {pool_size} requests drawn ({t_gen:.0f} s)")
    sc = sw.Scoring.make(2, -3, 5, 2, 32, sw.PREC_AUTO, max_read_len=250)
    srv = sw.Server(sc, memory_budget=4 << 30, max_step_reads=65536, max_step_cals=step_cals, max_step_chunks=1024,
                    max_steps_in_flight=depth)
    srv.set_refs(rs)

    # saturated throughput: the whole pool queued at once
    for b in pool[:8]:  # warm-up
        srv.wait(srv.submit_batch(b))
    # the pool eight times over (about 8.5 M reads, some 130 steps), so the pipeline's
    # ramp-up and drain (two or three steps) are a small part of the window
    rounds = 8
    preps = [srv.prepare_batch(b) for _ in range(rounds) for b in pool]
    n_clients = 4  # client threads submitting at once (the library calls release the GIL)
    hs = [None] * len(preps)

    def client(k):
        for i in range(k, len(preps), n_clients):
            hs[i] = srv.submit_prepared(preps[i])

    t0 = time.monotonic()
    clients = [threading.Thread(target=client, args=(k,)) for k in range(n_clients)]
    for th in clients:
        th.start()
    for th in clients:
        th.join()
    for h in hs:
        srv.wait(h)
    dt = time.monotonic() - t0
    for h in hs:
        srv.release(h)
    # results of the first pass over the pool: every later submission of the same
    # request, in whatever mix of other requests, must give exactly these
    first = [(h.score, h.ref_end, h.read_end, h.best_score, h.best_slot, h.n_tied) for h in hs[:pool_size]]
    del preps, hs
    # per-request oracle parity on a seeded sample of the pool (not timed)
    from oracle import oracle as orc
    prng = np.random.default_rng(5)
    sample = np.sort(prng.choice(pool_size, min(parity_requests, pool_size), replace=False)) if parity_requests else []
    parity_ok = True
    for k in sample:
        b = pool[int(k)]
        s_, r_, e_, _ = orc.align_batch(b, n_threads=min(16, os.cpu_count() or 1))
        bs_, bl_, nt_ = orc.reduce_best(b.cal_ptr, b.cal_ref, b.n_reads, b.n_refs, s_)
        got = first[int(k)]
        parity_ok &= all(np.array_equal(x, y) for x, y in zip(got, (s_, r_, e_, bs_.reshape(-1), bl_.reshape(-1),
                                                                  nt_.reshape(-1))))
    progress(f"served: saturated {sat_reads_of(pool, rounds, dt):.0f} reads/s; oracle parity on "
             f"{len(sample)} requests: {parity_ok}")
    sat_reads = sat_reads_of(pool, rounds, dt)
    sat_gcups = rounds * sum(pool_cells) / dt / 1e9
    mean_reads = float(np.mean([b.n_reads for b in pool]))

    results = []
    same_in_every_mix = True
    for load in loads:
        rate = load * sat_reads / mean_reads          # requests per second
        g = np.random.default_rng(int(load * 1000))
        arrivals = np.cumsum(g.exponential(1.0 / rate, per_load))
        picks = g.integers(0, pool_size, per_load)
        handles = [srv.prepare_batch(pool[k]) for k in picks]   # outputs allocated before the clock starts
        st0 = srv.stats()
        start = time.monotonic() + 0.05

        def feeder():
            for i in range(per_load):
                delay = start + arrivals[i] - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
                srv.submit_prepared(handles[i])

        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        lat = np.zeros(per_load)
        admit = np.zeros(per_load)                     # submission to admission (arena space)
        done_last = 0.0
        for i, h in enumerate(handles):
            srv.wait(h)
            _, t_sub, t_adm, t_done = srv.info(h)
            lat[i] = t_done - (start + arrivals[i])
            admit[i] = t_adm - t_sub
            done_last = max(done_last, t_done)
            srv.release(h)
            same_in_every_mix &= all(np.array_equal(x, y) for x, y in zip(
                (h.score, h.ref_end, h.read_end, h.best_score, h.best_slot, h.n_tied), first[int(picks[i])]))
        st1 = srv.stats()
        n_steps = st1["steps"] - st0["steps"]
        keep = lat[per_load // 10:]                    # 10% warm-up dropped
        sizes = np.array([pool[int(k)].n_reads for k in picks])[per_load // 10:]
        small, large = keep[sizes <= 100], keep[sizes >= 1000]
        span = done_last - start
        results.append({"load": load, "offered_requests_per_s": round(rate, 1), "requests": per_load,
                        "p50_ms": round(float(np.percentile(keep, 50)) * 1e3, 3),
                        "p99_ms": round(float(np.percentile(keep, 99)) * 1e3, 3),
                        "mean_ms": round(float(keep.mean()) * 1e3, 3),
                        # by request size (reads): how much of the latency is queueing behind larger requests
                        "p50_ms_upto_100_reads": round(float(np.percentile(small, 50)) * 1e3, 3) if len(small) else None,
                        "p50_ms_from_1000_reads": round(float(np.percentile(large, 50)) * 1e3, 3) if len(large) else None,
                        "mean_admission_wait_ms": round(float(admit[per_load // 10:].mean()) * 1e3, 3),
                        # device steps of the phase and their mean size
                        "steps": n_steps, "steps_launched_early": st1["steps_launched_early"] - st0["steps_launched_early"],
                        "mean_step_reads": round((st1["step_reads"] - st0["step_reads"]) / max(n_steps, 1), 1),
                        "phase_ms_per_step": round(span * 1e3 / max(n_steps, 1), 3),
                        "achieved_reads_per_s": round(sum(pool[k].n_reads for k in picks) / span, 1),
                        "achieved_gcups": round(sum(pool_cells[k] for k in picks) / span / 1e9, 1)})
        progress(f"served: load {load}: p50 {results[-1]['p50_ms']} ms, p99 {results[-1]['p99_ms']} ms")
    stats = srv.stats()
    srv.close()
    return {"workload": f"served requests: resident references of {int(pack[2][0]):,} and {int(pack[2][1]):,} bp "
                        f"(random + 5% planted repeats, {sum(int(x) for x in pack[2]) / 4e9:.2f} GB 2-bit), "
                        f"Poisson arrivals, requests log-uniform 1..10000 reads (pool of {pool_size}), "
                        "L U{75..250}, CALs U{1..32} per read, band 32, both strands",
            "saturated": {"reads_per_s": round(sat_reads, 1), "gcups": round(sat_gcups, 1),
                          "requests_per_s": round(rounds * pool_size / dt, 1)},
            "mean_request_reads": round(mean_reads, 1), "loads": results, "steps": stats["steps"], "steps_launched_early": stats["steps_launched_early"],
            "parity_sample_ok": bool(parity_ok), "parity_requests": len(sample),
            "same_result_in_every_mix": bool(same_in_every_mix),
            "max_step_cals": step_cals, "max_steps_in_flight": depth or "adaptive",
            "gen_s": round(t_gen, 1)}


def progress(msg):
    """One line per finished leg on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def guarded(name, fn):
    """Run one secondary leg; a Python-level failure is reported in its place in
    the JSON line (and on stderr) instead of losing the whole line."""
    try:
        return fn()
    except Exception as e:  # noqa: BLE001 - reported, not hidden
        progress(f"{name} failed: {e!r}")
        return {"error": repr(e)[:500]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reads", type=int, default=1_000_000)
    ap.add_argument("--uneven-reads", type=int, default=2_000_000,
                    help="reads of the uneven-length leg (0 skips it)")
    ap.add_argument("--uneven-bands", default="16,32,64", help="bands of the uneven-length leg")
    ap.add_argument("--two-ref-reads", type=int, default=4_000_000,
                    help="reads of the two-reference classification leg (0 skips it)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="reference size scale of the served leg (1.0 = 3.2 + 2.7 Gbp; 0 skips it)")
    ap.add_argument("--serve-pool", type=int, default=300)
    ap.add_argument("--serve-step-cals", type=int, default=1 << 20, help="CALs per device step of the server")
    ap.add_argument("--serve-depth", type=int, default=0, help="steps the server keeps queued on the device (0: adaptive, its default)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per load level")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pipeline", type=int, default=1, help="1: also time seeds -> CALs -> filter -> score")
    ap.add_argument("--variants", type=int, default=1, help="1: also time int32 and final-row scoring and the small-reference workload")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run an elementwise copy of this size (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the scoring path has no "
                                   "multi-GPU mode (reads shard across GPUs with no collective)"}))
        sys.exit(2)

    import torch

    from paper_1805_00106_amd import workloads as wl

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    batch = wl.chromosome_scale(n_reads=args.reads)
    t_gen = time.perf_counter() - t_gen
    leg = Leg(batch, int(batch.read_len.max()), args.steps, args.warmup)
    r2 = leg.run()
    progress(f"chromosome scale: batched {r2['batched_gcups']} GCUPS, plain {r2['plain_gcups']} GCUPS")
    parity = None if args.no_parity else parity_sample(batch, leg.out)
    leg.parity_reads = not args.no_parity
    e2e = leg.end_to_end()
    variants = guarded("variants", leg.variants) if args.variants else None
    progress("variants done")
    trace = guarded("traceback", lambda: leg.traceback(parity_reads=0 if args.no_parity else 200))
    progress("traceback done")
    pipe = guarded("seed-to-score", leg.pipeline) if args.pipeline else None
    progress("seed-to-score done")
    small = guarded("small batch", lambda: small_batch_latency(batch))
    n_reads, n_cals, cells = leg.db.n_reads, leg.db.n_cals, leg.cells
    leg.free()
    del leg

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib * (1 << 18), dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    def uneven_leg():
        base3 = wl.uneven_lengths(n_reads=args.uneven_reads, band=32)  # reads and CALs do not depend on the band
        out3 = {}
        for band in [int(x) for x in args.uneven_bands.split(",")]:
            b3 = dataclasses.replace(base3, scoring=dataclasses.replace(base3.scoring, band=band),
                                     name=f"uneven_lengths_band{band}")
            leg3 = Leg(b3, 250, max(3, args.steps // 4), 1)
            r3 = leg3.run()
            p3 = None if args.no_parity else parity_sample(b3, leg3.out)
            out3[f"band{band}"] = {
                "workload": f"uneven lengths: same 100 Mbp reference, {b3.n_reads} reads with L uniform 75..250, geometric CALs "
                            f"(mean 8, cap 64), band {band}, both strands, int16",
                "cals": b3.n_cals, "cells": leg3.cells,
                "plain_gcups": r3["plain_gcups"], "batched_gcups": r3["batched_gcups"],
                "plain_ms_per_step": round(r3["plain_ms"], 3), "batched_ms_per_step": round(r3["batched_ms"], 3),
                "plain_reads_per_s": round(b3.n_reads / (r3["plain_ms"] * 1e-3), 1),
                "batched_reads_per_s": round(b3.n_reads / (r3["batched_ms"] * 1e-3), 1),
                "speedup_batched_vs_plain": round(r3["plain_ms"] / r3["batched_ms"], 3),
                "plain_equals_batched": r3["plain_equals_batched"], "parity_sample_ok": p3, "plan": r3["plan"]}
            leg3.free()
            del leg3
            progress(f"uneven lengths band {band}: batched {r3['batched_gcups']} GCUPS")
        return out3

    c3 = guarded("uneven lengths", uneven_leg) if args.uneven_reads else None

    c4 = guarded("two references", lambda: classification_leg(args.two_ref_reads, parity=not args.no_parity)) \
        if args.two_ref_reads else None
    progress("two references done")
    served = guarded("served", lambda: served_leg(args.serve_scale, args.serve_pool, args.serve_requests,
                                                  step_cals=args.serve_step_cals, depth=args.serve_depth)) \
        if args.serve_scale > 0 else None
    if served and "error" not in served:
        progress("served done")

    step_ms, kern_ms = r2["batched_ms"], r2["batched_kern_ms"]
    gcups = cells / (step_ms * 1e-3) / 1e9
    import paper_1805_00106_amd as sw
    measured = sw.alu_peak(16) / 1e12  # sustained packed-int16 add/max rate on this device
    kern_label = profile_kernel(r2["plan"], False, False)
    roof = roofline(kern_label, "chromosome_scale", cells, kern_ms, True)
    roof["traffic"] = load_traffic(kern_label, "chromosome_scale")
    roof["peak_measured_alu_tops"] = round(measured, 2)
    res = {
        "metric": METRIC, "value": round(gcups, 1), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int16", "data": "synthetic",
        "config": {"workload": "chromosome scale: 100 Mbp reference (5% planted repeats), 1M x 100 bp reads, "
                               "Poisson(6)+1 CALs/read, band 32, both strands, int16",
                   "reads": n_reads, "cals": n_cals, "tasks": 2 * n_cals, "cells": cells,
                   "path": "batched context (tuned plan: length bins or input order; tiles popped from a device queue; HIP graph)",
                   "plan": r2["plan"]},
        "reads_per_s": round(n_reads / (step_ms * 1e-3), 1),
        "plain": {"gcups": r2["plain_gcups"], "ms_per_step": round(r2["plain_ms"], 3),
                  "reads_per_s": round(n_reads / (r2["plain_ms"] * 1e-3), 1),
                  "kernel_ms": round(r2["plain_kern_ms"], 3)},
        "plain_equals_batched": r2["plain_equals_batched"],
        "small_batch_latency": small,
        "end_to_end_with_pcie": e2e,
        "variants": variants,
        "small_reference": guarded("small reference", small_reference_leg) if args.variants else None,
        "traceback": trace,
        "seed_to_score": pipe,
        "aligned_fraction": round(r2["aligned_fraction"], 4), "aligned_threshold": ALIGNED_THRESHOLD,
        "wall_s_timed": round(r2["wall"], 3), "gen_s": round(t_gen, 1), "parity_sample_ok": parity,
        "roofline": roof,
    }
    if c3:
        res["uneven_lengths"] = c3
    if c4:
        res["two_references"] = c4
    if served:
        res["served"] = served
        if "loads" in served:
            res["p50_ms"] = served["loads"][-1]["p50_ms"]
            res["p99_ms"] = served["loads"][-1]["p99_ms"]
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = guarded("cpu baseline", lambda: cpu_baseline(batch))
    print(json.dumps(res))


if __name__ == "__main__":
    main()

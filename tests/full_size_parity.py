"""Full-size parity of the batched path against the oracle (GPU host, minutes).

TEST INFRASTRUCTURE, run by hand (pytest does not collect it):

    python tests/full_size_parity.py uneven_lengths --band 16
    python tests/full_size_parity.py two_references --reads 4000000
    python tests/full_size_parity.py chromosome_scale --final-row

The whole batch is scored once on the GPU (batched context, per-read best);
the oracle then scores it in chunks of reads on the host cores, and every slot
output (score, ref_end, read_end) and every per-read, per-reference best (score,
slot, tie count) is compared.  One progress line per chunk.
"""
import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_1805_00106_amd as sw  # noqa: E402
from oracle import oracle as orc  # noqa: E402
from paper_1805_00106_amd import workloads as wl  # noqa: E402


def make_batch(name, reads, band):
    if name == "small_reference":
        return wl.small_reference(), sw.PREC_INT32, 76
    if name == "chromosome_scale":
        return wl.chromosome_scale(n_reads=reads or 1_000_000), sw.PREC_INT16, 100
    if name == "uneven_lengths":
        return wl.uneven_lengths(n_reads=reads or 2_000_000, band=band), sw.PREC_INT16, 250
    if name == "two_references":
        return wl.two_references(n_reads=reads or 4_000_000), sw.PREC_INT16, 150
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["small_reference", "chromosome_scale", "uneven_lengths", "two_references"])
    ap.add_argument("--reads", type=int, default=0, help="reads (0: the workload's full size)")
    ap.add_argument("--band", type=int, default=32, help="band of uneven_lengths")
    ap.add_argument("--chunk", type=int, default=100_000, help="reads per oracle chunk")
    ap.add_argument("--final-row", action="store_true", help="read-end-anchored scoring (the final-row mode)")
    ap.add_argument("--int32", action="store_true", help="score in int32 (one strand per lane)")
    args = ap.parse_args()
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    b, prec, mrl = make_batch(args.workload, args.reads, args.band)
    if args.int32:
        prec = sw.PREC_INT32
    sc0 = b.scoring
    print(f"{args.workload}: {b.n_reads} reads, {b.n_cals} CALs, band {sc0.band}, generated in "
          f"{time.perf_counter() - t0:.0f} s", flush=True)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    mode = sw.MODE_FINAL_ROW if args.final_row else sw.MODE_LOCAL
    sc = sw.Scoring.make(sc0.match, sc0.mismatch, sc0.gap_open, sc0.gap_extend, sc0.band, prec, sw.KERNEL_AUTO, mrl, mode)
    ctx = sw.Context(db.n_reads, db.n_cals)
    out = sw.Outputs(db.n_cals)
    ctx.align(db, refs, sc, out)
    bs, bl, nt = sw.reduce_best(db, b.n_refs, out.score)
    torch.cuda.synchronize()
    plan = ctx.last_plan()
    gs, gr, ge = out.score.cpu().numpy(), out.ref_end.cpu().numpy(), out.read_end.cpu().numpy()
    gbs, gbl, gnt = bs.cpu().numpy(), bl.cpu().numpy(), nt.cpu().numpy()
    ctx.close()
    del refs, db, out, bs, bl, nt
    torch.cuda.empty_cache()
    t1 = time.perf_counter()
    bad_slots = bad_best = 0
    for a in range(0, b.n_reads, args.chunk):
        idx = np.arange(a, min(a + args.chunk, b.n_reads))
        sub = b.subset_reads(idx)
        s, r, e, _ = orc.align_batch(sub, n_threads=threads, final_row=args.final_row)
        obs, obl, ont = orc.reduce_best(sub.cal_ptr, sub.cal_ref, sub.n_reads, sub.n_refs, s)
        c0 = int(b.cal_ptr[idx[0]])
        sl = slice(2 * c0, 2 * int(b.cal_ptr[idx[-1] + 1]))
        bad_slots += int((gs[sl] != s).sum() + (gr[sl] != r).sum() + (ge[sl] != e).sum())
        obl = np.where(obl >= 0, obl + 2 * c0, obl)  # sub-batch slots -> batch slots
        bad_best += int((gbs[idx] != obs).sum() + (gbl[idx] != obl).sum() + (gnt[idx] != ont).sum())
        print(f"{args.workload}: reads {idx[-1] + 1}/{b.n_reads}, differing slot entries {bad_slots}, "
              f"differing best entries {bad_best}, {time.perf_counter() - t1:.0f} s", flush=True)
    print(f"{args.workload} (band {sc0.band}{', final row' if args.final_row else ''}{', int32' if args.int32 else ''}): {b.n_reads} reads, {2 * b.n_cals} slots, batched path [{plan}] vs "
          f"oracle on {threads} threads: differing slot entries {bad_slots}, differing per-read best entries "
          f"{bad_best}; oracle {time.perf_counter() - t1:.0f} s", flush=True)
    sys.exit(1 if bad_slots or bad_best else 0)


if __name__ == "__main__":
    main()

"""Helpers for the GPU tests: run the HIP path and the oracle on the same batch."""
import numpy as np
import torch

import paper_1805_00106_amd as sw
from oracle import oracle as orc


def scoring_for(batch, precision, kernel=0, max_read_len=None, mode=sw.MODE_LOCAL):
    sc = batch.scoring
    mrl = int(batch.read_len.max()) if max_read_len is None and batch.n_reads else (max_read_len or 0)
    return sw.Scoring.make(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band, precision, kernel,
                           max(mrl, 1) if mrl else 0, mode)


def gpu_align(batch, precision=sw.PREC_AUTO, kernel=0, max_read_len=None, reduce=True, mode=sw.MODE_LOCAL,
              topk=0):
    refs = sw.RefSet.from_codes(torch.from_numpy(batch.ref_codes).cuda(), batch.ref_off, batch.ref_len)
    db = sw.DeviceBatch.upload(batch)
    scoring = scoring_for(batch, precision, kernel, max_read_len, mode)
    out = sw.align_batch(db, refs, scoring)
    res = dict(score=out.score, ref_end=out.ref_end, read_end=out.read_end)
    if reduce:
        bs, bl, nt = sw.reduce_best(db, batch.n_refs, out.score)
        res.update(best_score=bs, best_slot=bl, n_tied=nt)
    if topk:
        ts, tl = sw.topk(db, out.score, topk)
        res.update(top_score=ts, top_slot=tl, tied=sw.tied_flags(db, out.score))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def oracle_align(batch, threads=8, mode=sw.MODE_LOCAL, topk=0):
    s, r, e, errs = orc.align_batch(batch, n_threads=threads, final_row=mode == sw.MODE_FINAL_ROW)
    bs, bl, nt = orc.reduce_best(batch.cal_ptr, batch.cal_ref, batch.n_reads, batch.n_refs, s)
    res = dict(score=s, ref_end=r, read_end=e, best_score=bs, best_slot=bl, n_tied=nt)
    if topk:
        ts, tl = orc.topk(batch.cal_ptr, batch.n_reads, s, topk)
        res.update(top_score=ts, top_slot=tl, tied=orc.tied_flags(batch.cal_ptr, batch.n_reads, s))
    return res, errs


# the per-slot outputs of a scoring call (without the Score Tracker's per-read ones)
SLOTS = ("score", "ref_end", "read_end")


def assert_same(got, exp, what="", keys=None):
    """Element-wise equality of the outputs named by `keys` (default: every
    output in `exp`).  An output missing from `got` fails: a dropped output must
    not pass."""
    for k in (exp.keys() if keys is None else keys):
        if k not in got:
            raise AssertionError(f"{what}: output {k} missing from the GPU results")
        if k not in exp:
            raise AssertionError(f"{what}: output {k} missing from the expected results")
        g, e = got[k], exp[k]
        if g.shape != e.shape:
            raise AssertionError(f"{what}: {k} has shape {g.shape}, expected {e.shape}")
        if not np.array_equal(g, e):
            bad = np.nonzero(g.reshape(-1) != e.reshape(-1))[0]
            i = int(bad[0])
            raise AssertionError(f"{what}: {k} differs in {len(bad)} of {e.size} entries; first at {i}: "
                                 f"gpu={g.reshape(-1)[i]} oracle={e.reshape(-1)[i]}")

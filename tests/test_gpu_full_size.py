"""GPU parity at the benchmark's full sizes, in the launch configuration bench.py
times (batched context: length bins, persistent work queue, HIP graph,
autotuned plan): a seeded sample of reads is compared with the oracle read by
read, and every slot is checked against properties that hold at any size
(plain and batched paths bit-identical, score bounds, end cells inside the
window, score 0 exactly when both ends are -1)."""
import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from oracle import oracle as orc
from paper_1805_00106_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run(b, mrl, plain=True, mode=sw.MODE_LOCAL):
    sc0 = b.scoring
    sc = sw.Scoring.make(sc0.match, sc0.mismatch, sc0.gap_open, sc0.gap_extend, sc0.band, sw.PREC_INT16,
                         sw.KERNEL_AUTO, mrl, mode)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    ctx = sw.Context(db.n_reads, db.n_cals)
    out = sw.Outputs(db.n_cals)
    ctx.align(db, refs, sc, out)   # captures the graph
    ctx.align(db, refs, sc, out)   # replays it, as the timed steps do
    bs, bl, nt = sw.reduce_best(db, b.n_refs, out.score)
    torch.cuda.synchronize()
    got = dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(),
               read_end=out.read_end.cpu().numpy(), best_score=bs.cpu().numpy(), best_slot=bl.cpu().numpy(),
               n_tied=nt.cpu().numpy())
    ctx.close()
    if plain:
        p = sw.align_batch(db, refs, sc)
        torch.cuda.synchronize()
        for k, v in (("score", p.score), ("ref_end", p.ref_end), ("read_end", p.read_end)):
            assert np.array_equal(v.cpu().numpy(), got[k]), f"plain and batched differ in {k}"
    return got


def _properties(b, got, final_row=False):
    sc = b.scoring
    owner = np.repeat(np.arange(b.n_reads), np.diff(b.cal_ptr))
    L = np.repeat(b.read_len[owner].astype(np.int64), 2)
    ref_len = b.ref_len[b.cal_ref.astype(np.int64)]
    ws = np.repeat(np.maximum(0, b.cal_pos - sc.band), 2)
    we = np.repeat(np.minimum(ref_len, b.cal_pos + b.read_len[owner] + sc.band), 2)
    s, re, qe = got["score"].astype(np.int64), got["ref_end"], got["read_end"].astype(np.int64)
    assert (s >= 0).all() and (s <= sc.match * L).all()                 # both strands requested, none invalid
    zero = s == 0
    assert ((re == -1) == zero).all() and ((qe == -1) == zero).all()
    nz = ~zero
    assert ((qe[nz] >= 0) & (qe[nz] < L[nz])).all()
    if final_row:
        assert (qe[nz] == L[nz] - 1).all()   # the alignment ends at the read's last base
    assert ((re[nz] >= ws[nz]) & (re[nz] < we[nz])).all()
    # per read and reference: the best is the maximum of the read's slots on that
    # reference, the best slot the lowest one holding it, the tie count how many do
    counts = np.diff(b.cal_ptr)
    assert (counts > 0).all()
    starts = 2 * b.cal_ptr[:-1]
    slot_ix = np.arange(2 * b.n_cals, dtype=np.int64)
    for k in range(b.n_refs):
        sk = np.where(np.repeat(b.cal_ref == k, 2), s, -1)
        mx = np.maximum.reduceat(sk, starts)
        hit = (sk == np.repeat(mx, 2 * counts)) & (sk >= 0)
        nt = np.add.reduceat(hit.astype(np.int64), starts)
        bl = np.minimum.reduceat(np.where(hit, slot_ix, 1 << 62), starts)
        bl = np.where(mx >= 0, bl, -1)
        np.testing.assert_array_equal(got["best_score"][:, k], mx)
        np.testing.assert_array_equal(got["n_tied"][:, k], nt)
        np.testing.assert_array_equal(got["best_slot"][:, k], bl)


def _sample(b, got, n=1500, seed=11, final_row=False):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(b.n_reads, n, replace=False))
    sub = b.subset_reads(idx)
    s, r, e, _ = orc.align_batch(sub, n_threads=16, final_row=final_row)
    bs, bl, nt = orc.reduce_best(sub.cal_ptr, sub.cal_ref, sub.n_reads, sub.n_refs, s)
    sel = np.concatenate([np.arange(b.cal_ptr[i], b.cal_ptr[i + 1]) for i in idx])
    slots = np.stack([2 * sel, 2 * sel + 1], 1).reshape(-1)
    np.testing.assert_array_equal(got["score"][slots], s)
    np.testing.assert_array_equal(got["ref_end"][slots], r)
    np.testing.assert_array_equal(got["read_end"][slots], e)
    np.testing.assert_array_equal(got["best_score"][idx], bs)
    np.testing.assert_array_equal(got["n_tied"][idx], nt)
    # the sample's slots renumbered to the full batch
    first = np.concatenate([[0], np.cumsum(np.diff(b.cal_ptr)[idx])])[:-1]
    shift = 2 * (b.cal_ptr[idx] - first)
    exp_bl = np.where(bl >= 0, bl + shift[:, None], bl)
    np.testing.assert_array_equal(got["best_slot"][idx], exp_bl)


def test_chromosome_scale_full_size():
    """1 M x 100 bp reads, 7.0 M CALs, band 32, both strands, int16."""
    b = wl.chromosome_scale()
    got = _run(b, 100)
    _properties(b, got)
    _sample(b, got)


_UNEVEN = {}


@pytest.mark.parametrize("band", [16, 32, 64])
def test_uneven_lengths_full_size(band):
    """2 M reads of 75..250 bp, 16.0 M CALs (geometric counts), bands 16, 32 and 64, int16
    (the reads and CALs do not depend on the band)."""
    import dataclasses
    if "base" not in _UNEVEN:
        _UNEVEN["base"] = wl.uneven_lengths(band=32)
    base = _UNEVEN["base"]
    b = dataclasses.replace(base, scoring=dataclasses.replace(base.scoring, band=band))
    got = _run(b, 250, plain=False)
    _properties(b, got)
    _sample(b, got, n=800, seed=11 + band)


def test_two_references_full_size():
    """4 M x 150 bp reads against two 500 Mbp references, 24.0 M CALs, band 32, int16;
    the two-reference classification of the sample against the oracle's."""
    b = wl.two_references()
    got = _run(b, 150, plain=False)
    _properties(b, got)
    _sample(b, got, n=1000)
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(b.n_reads, 1000, replace=False))
    cls = sw.classify(torch.from_numpy(got["best_score"]).cuda(), 40).cpu().numpy()
    np.testing.assert_array_equal(cls[idx], orc.classify(got["best_score"][idx], 40))


def test_chromosome_scale_full_size_final_row():
    """The chromosome-scale workload in read-end-anchored (final-row) scoring."""
    b = wl.chromosome_scale()
    got = _run(b, 100, mode=sw.MODE_FINAL_ROW)
    _properties(b, got, final_row=True)
    _sample(b, got, n=1000, final_row=True)


def test_traceback_full_size_best_slots():
    """Start and CIGAR of every read's best slot on the chromosome-scale workload
    (1 M traced slots): a seeded sample against the oracle, and every CIGAR spans
    its read and ends at the reported end cell."""
    b = wl.chromosome_scale()
    sc0 = b.scoring
    sc = sw.Scoring.make(sc0.match, sc0.mismatch, sc0.gap_open, sc0.gap_extend, sc0.band, sw.PREC_INT16,
                         sw.KERNEL_AUTO, 100)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    out = sw.align_batch(db, refs, sc)
    bs, bl, _ = sw.reduce_best(db, b.n_refs, out.score)
    slots = bl[:, 0].contiguous()
    rs, qs, nops, cig = sw.traceback(db, refs, sc, out, slots, cap=64)
    torch.cuda.synchronize()
    slots_h, nops_h = slots.cpu().numpy(), nops.cpu().numpy()
    rs_h, qs_h = rs.cpu().numpy(), qs.cpu().numpy()
    cig_h = cig.cpu().numpy().view(np.uint32).reshape(b.n_reads, 64)
    score, ref_end = out.score.cpu().numpy(), out.ref_end.cpu().numpy()
    assert (slots_h >= 0).all() and (nops_h > 0).all()
    # every CIGAR: read bases consumed = L, reference span ends at ref_end
    n = nops_h.astype(np.int64)
    mask = np.arange(64)[None, :] < n[:, None]
    length, op = (cig_h >> 4).astype(np.int64) * mask, (cig_h & 15) * mask
    read_ops = np.isin(op, (1, 4, 7, 8)) & mask
    ref_ops = np.isin(op, (2, 7, 8)) & mask
    np.testing.assert_array_equal((length * read_ops).sum(1), b.read_len.astype(np.int64))
    np.testing.assert_array_equal(rs_h + (length * ref_ops).sum(1) - 1, ref_end[slots_h])
    # a sample against the oracle (its slots renumbered to the sample's batch)
    rng = np.random.default_rng(13)
    idx = np.sort(rng.choice(b.n_reads, 500, replace=False))
    sub = b.subset_reads(idx)
    s, r, e, _ = orc.align_batch(sub, n_threads=16)
    obs, obl, _ = orc.reduce_best(sub.cal_ptr, sub.cal_ref, sub.n_reads, sub.n_refs, s)
    ors, oqs, onops, ocig = orc.traceback(sub, s, r, e, obl[:, 0].astype(np.int64), cap=64, max_read_len=100)
    np.testing.assert_array_equal(rs_h[idx], ors)
    np.testing.assert_array_equal(qs_h[idx], oqs)
    np.testing.assert_array_equal(nops_h[idx], onops)
    np.testing.assert_array_equal(cig_h[idx], ocig.reshape(len(idx), 64))

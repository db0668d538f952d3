"""Parity on a reference longer than 2^32 bases, with reads and CALs around
positions 2^31 and 2^32 and near both ends: every kernel family (one CAL per
lane in int16 and int32, one wavefront per task, the batched queue kernels,
both traceback kernels, the served path) against the oracle, bit for bit.
Window starts at or past 2^31 are where the one-wavefront-per-task kernel once
sign-extended the low half of its 64-bit lane broadcast."""
import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from oracle import oracle as orc
from paper_1805_00106_amd import workloads as wl
from tests.gpu_util import SLOTS, assert_same

pytestmark = pytest.mark.gpu

_CACHE = {}


def batch_and_refs():
    if "b" not in _CACHE:
        b = wl.long_reference()
        # the references on the device: zeros, then each random patch, then packed
        codes = torch.zeros(b.ref_codes.shape[0], dtype=torch.uint8, device="cuda")
        for k, a, n in b.ref_patches:
            lo = int(b.ref_off[k]) + a
            codes[lo:lo + n] = torch.from_numpy(np.ascontiguousarray(b.ref_codes[lo:lo + n])).cuda()
        refs = sw.RefSet.from_codes(codes, b.ref_off, b.ref_len)
        torch.cuda.synchronize()
        del codes
        torch.cuda.empty_cache()
        s, r, e, errs = orc.align_batch(b, n_threads=8)
        assert errs == 0
        bs, bl, nt = orc.reduce_best(b.cal_ptr, b.cal_ref, b.n_reads, b.n_refs, s)
        _CACHE.update(b=b, refs=refs, exp=dict(score=s, ref_end=r, read_end=e, best_score=bs, best_slot=bl,
                                               n_tied=nt))
    return _CACHE["b"], _CACHE["refs"], _CACHE["exp"]


def _scoring(b, precision, kernel=sw.KERNEL_AUTO):
    sc = b.scoring
    return sw.Scoring.make(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band, precision, kernel,
                           int(b.read_len.max()))


def test_long_reference_reaches_past_2_32():
    b, refs, exp = batch_and_refs()
    assert int(b.ref_len[1]) > (1 << 32) and int(b.cal_pos.max()) > (1 << 32)
    assert ((b.cal_pos >= (1 << 31)) & (b.cal_pos < (1 << 32))).sum() > 50
    # the planted locus of every read is found (scores near 2L)
    best = exp["best_score"].max(axis=1)
    assert (best >= 2 * b.read_len - 5 * 4 * np.ceil(b.read_len / 100)).mean() > 0.95


@pytest.mark.parametrize("precision,kernel", [(sw.PREC_INT16, sw.KERNEL_INTER), (sw.PREC_INT32, sw.KERNEL_INTER),
                                              (sw.PREC_INT16, sw.KERNEL_INTRA), (sw.PREC_INT32, sw.KERNEL_INTRA),
                                              (sw.PREC_AUTO, sw.KERNEL_AUTO)])
def test_plain_kernels_match_oracle(precision, kernel):
    b, refs, exp = batch_and_refs()
    db = sw.DeviceBatch.upload(b)
    out = sw.align_batch(db, refs, _scoring(b, precision, kernel))
    bs, bl, nt = sw.reduce_best(db, b.n_refs, out.score)
    torch.cuda.synchronize()
    got = dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(), read_end=out.read_end.cpu().numpy(),
               best_score=bs.cpu().numpy(), best_slot=bl.cpu().numpy(), n_tied=nt.cpu().numpy())
    assert_same(got, exp, f"long reference, precision {precision}, kernel {kernel}")


@pytest.mark.parametrize("precision", [sw.PREC_INT16, sw.PREC_INT32])
def test_batched_matches_oracle(precision):
    b, refs, exp = batch_and_refs()
    db = sw.DeviceBatch.upload(b)
    ctx = sw.Context(db.n_reads, db.n_cals, autotune=False)
    out = ctx.align(db, refs, _scoring(b, precision))
    torch.cuda.synchronize()
    got = dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(), read_end=out.read_end.cpu().numpy())
    ctx.close()
    assert_same(got, exp, f"long reference, batched, precision {precision}", keys=SLOTS)


@pytest.mark.parametrize("kernel", [sw.KERNEL_INTER, sw.KERNEL_INTRA])
def test_traceback_matches_oracle(kernel):
    b, refs, exp = batch_and_refs()
    db = sw.DeviceBatch.upload(b)
    sc = _scoring(b, sw.PREC_AUTO, kernel)
    out = sw.align_batch(db, refs, _scoring(b, sw.PREC_AUTO))
    slots = torch.from_numpy(exp["best_slot"].max(axis=1).astype(np.int64)).cuda()
    rs, qs, nops, cig = sw.traceback(db, refs, sc, out, slots)
    torch.cuda.synchronize()
    ers, eqs, enops, ecig = orc.traceback(b, exp["score"], exp["ref_end"], exp["read_end"],
                                          exp["best_slot"].max(axis=1), cap=64)
    assert_same(dict(ref_start=rs.cpu().numpy(), read_start=qs.cpu().numpy(), n_ops=nops.cpu().numpy(),
                     cigar=cig.cpu().numpy().astype(np.uint32)),
                dict(ref_start=ers, read_start=eqs, n_ops=enops, cigar=ecig.astype(np.uint32)),
                f"long reference, traceback kernel {kernel}")

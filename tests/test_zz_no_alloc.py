"""The no-allocation scoring entry point (sw_align_batch_noalloc, through the C
ABI): on two calls in a row, the second on a smaller batch, its outputs equal
those of sw_align_batch on the same inputs and the oracle's, bit for bit; a
call whose scratch would not fit the static array is rejected."""
import ctypes

import pytest
import torch

import paper_1805_00106_amd as sw
from paper_1805_00106_amd import workloads as wl
from tests.gpu_util import SLOTS, assert_same, oracle_align, scoring_for

pytestmark = pytest.mark.gpu


_BATCHES = {}


def _batches():
    if not _BATCHES:
        _BATCHES["big"] = wl.uneven_lengths(n_reads=3000, band=32)
        _BATCHES["small"] = wl.random_small_batch(61, n_reads=90, read_len=(1, 160), band=16)
    return _BATCHES["big"], _BATCHES["small"]


def _host(out):
    torch.cuda.synchronize()
    return dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(), read_end=out.read_end.cpu().numpy())


@pytest.mark.parametrize("precision,kernel", [(sw.PREC_INT16, sw.KERNEL_INTER), (sw.PREC_INT32, sw.KERNEL_INTER),
                                              (sw.PREC_INT32, sw.KERNEL_INTRA), (sw.PREC_AUTO, sw.KERNEL_AUTO)])
def test_noalloc_equals_align_batch_on_two_calls(precision, kernel):
    big, small = _batches()
    for k, b in enumerate((big, small)):        # the second call is smaller
        refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
        db = sw.DeviceBatch.upload(b)
        sc = scoring_for(b, precision, kernel=kernel, max_read_len=250 if k == 0 else None)
        want = _host(sw.align_batch(db, refs, sc))
        out = sw.Outputs(db.n_cals)
        for t in (out.score, out.ref_end, out.read_end):
            t.fill_(-7)
        got = _host(sw.align_batch_noalloc(db, refs, sc, out))
        assert_same(got, want, f"call {k}: noalloc vs align_batch, precision {precision}, kernel {kernel}")
        exp, _ = oracle_align(b)
        assert_same(got, exp, f"call {k}: noalloc vs oracle", keys=SLOTS)


def test_noalloc_rejects_scratch_beyond_the_static_array():
    b = wl.random_small_batch(62, n_reads=40, read_len=(1, 100), band=16)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    sc = sw.Scoring.make(2, -3, 5, 2, 16, sw.PREC_INT16, sw.KERNEL_INTER, 100)
    assert sw.workspace_bytes(db.n_reads, db.n_cals, sc) <= sw.NOALLOC_SCRATCH_BYTES
    # a CAL count whose owner-read array alone exceeds the array: rejected before any launch
    huge = sw.NOALLOC_SCRATCH_BYTES // 4 + 1
    assert sw.workspace_bytes(1, huge, sc) > sw.NOALLOC_SCRATCH_BYTES
    p = torch.zeros(8, dtype=torch.int64, device="cuda")
    rc = sw.lib().sw_align_batch_noalloc(sw._ptr(db.reads2bit), sw._ptr(db.read_word_off), sw._ptr(db.read_len),
                                         db.n_reads, refs.c, sw._ptr(db.cal_ptr), sw._ptr(p), sw._ptr(p),
                                         sw._ptr(p), huge, ctypes.byref(sc), sw._ptr(p), sw._ptr(p), sw._ptr(p),
                                         sw._stream())
    assert rc == -5

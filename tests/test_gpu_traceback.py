"""GPU parity of the traceback (start position + CIGAR) against the oracle:
bit-exact starts, operation counts and CIGAR entries, with the same walk
rules on both sides; every traced CIGAR is also rescored independently."""
import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from oracle import oracle as orc
from paper_1805_00106_amd import workloads as wl
from tests.gpu_util import SLOTS, assert_same, oracle_align, scoring_for

pytestmark = pytest.mark.gpu


def _gpu_trace(batch, slots, cap, precision=sw.PREC_AUTO, max_read_len=None, mode=sw.MODE_LOCAL,
               kernel=sw.KERNEL_AUTO):
    refs = sw.RefSet.from_codes(torch.from_numpy(batch.ref_codes).cuda(), batch.ref_off, batch.ref_len)
    db = sw.DeviceBatch.upload(batch)
    sc = scoring_for(batch, precision, kernel=kernel, max_read_len=max_read_len, mode=mode)
    out = sw.align_batch(db, refs, sc)
    rs, qs, nops, cig = sw.traceback(db, refs, sc, out, torch.as_tensor(np.asarray(slots, np.int64)), cap=cap)
    torch.cuda.synchronize()
    return (dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(),
                 read_end=out.read_end.cpu().numpy()),
            dict(ref_start=rs.cpu().numpy(), read_start=qs.cpu().numpy(), n_ops=nops.cpu().numpy(),
                 cigar=cig.cpu().numpy().view(np.uint32)))


def _oracle_trace(batch, slots, cap, max_read_len, mode=sw.MODE_LOCAL):
    exp, _ = oracle_align(batch, mode=mode)
    rs, qs, nops, cig = orc.traceback(batch, exp["score"], exp["ref_end"], exp["read_end"], slots, cap=cap,
                                      max_read_len=max_read_len)
    return exp, dict(ref_start=rs, read_start=qs, n_ops=nops, cigar=cig)


def _case(batch, slots=None, cap=64, max_read_len=None, mode=sw.MODE_LOCAL, **kw):
    if slots is None:
        slots = np.arange(2 * batch.n_cals, dtype=np.int64)
    mrl = max_read_len or max(int(batch.read_len.max()), 1)
    exp_s, exp_t = _oracle_trace(batch, slots, cap, mrl, mode=mode)
    # both kernel families: one traced slot per lane, one per wavefront
    for kernel in (sw.KERNEL_INTER, sw.KERNEL_INTRA):
        got_s, got_t = _gpu_trace(batch, slots, cap, max_read_len=mrl, mode=mode, kernel=kernel, **kw)
        assert_same(got_s, exp_s, f"{batch.name} scores kernel={kernel}", keys=SLOTS)
        assert_same(got_t, exp_t, f"{batch.name} traceback cap={cap} kernel={kernel}")
    # every traced CIGAR spans the read exactly and ends where the score says
    for t, slot in enumerate(slots):
        n = int(exp_t["n_ops"][t])
        if n <= 0:
            continue
        ops = [(int(v) >> 4, int(v) & 15) for v in exp_t["cigar"][t][:n]]
        c = int(slot) >> 1
        r = int(np.searchsorted(batch.cal_ptr, c, side="right") - 1)
        assert sum(k for k, op in ops if op in (1, 4, 7, 8)) == batch.read_len[r]
        assert exp_t["ref_start"][t] + sum(k for k, op in ops if op in (2, 7, 8)) - 1 == exp_s["ref_end"][slot]
    return exp_t


@pytest.mark.parametrize("seed", range(4))
def test_trace_ragged_all_slots(seed):
    """Every slot of a ragged batch (1..120 bp, clipped windows, strand masks)."""
    _case(wl.random_small_batch(70 + seed, n_reads=80, read_len=(1, 120), band=12))


def test_trace_long_reads_lds_planes():
    """L up to 250, band 32: per-task bit planes held in LDS."""
    b = wl.random_small_batch(75, n_reads=40, read_len=(150, 250), ref_len=(300, 3000), band=32)
    _case(b, max_read_len=250)


def test_trace_long_reads_device_planes():
    """L up to 250, band 64: the planes exceed the LDS budget and live in device memory."""
    b = wl.random_small_batch(76, n_reads=40, read_len=(150, 250), ref_len=(300, 3000), band=64)
    _case(b, max_read_len=250)


def test_trace_very_long_reads():
    b = wl.random_small_batch(77, n_reads=12, read_len=(500, 1000), ref_len=(1200, 4000), band=16)
    _case(b, max_read_len=1000, cap=256)


def test_trace_chromosome_scale_best_slots():
    """Chromosome-scale generator: trace each read's best slot (the usual caller)."""
    b = wl.chromosome_scale(n_reads=3000)
    exp, _ = oracle_align(b)
    slots = exp["best_slot"][:, 0].astype(np.int64)
    assert (slots >= 0).all()
    t = _case(b, slots=slots, max_read_len=100)
    assert (t["n_ops"] > 0).all()


def test_trace_final_row_mode():
    b = wl.random_small_batch(78, n_reads=60, read_len=(1, 100), band=10)
    t = _case(b, mode=sw.MODE_FINAL_ROW)
    for k in np.nonzero(t["n_ops"] > 0)[0]:
        assert (int(t["cigar"][k][t["n_ops"][k] - 1]) & 15) in (7, 8)   # never a tail clip


def test_trace_skip_invalid_and_capacity():
    b = wl.random_small_batch(79, n_reads=50, read_len=(20, 80), band=10)
    n = 2 * b.n_cals
    slots = np.array([-1, 0, 1, n, n + 5, -7, 2, 3] + list(range(4, n)), np.int64)
    sw.error_count(reset=True)
    t = _case(b, slots=slots, cap=3)
    assert t["n_ops"][0] == 0 and t["n_ops"][3] == -2 and t["n_ops"][4] == -2 and t["n_ops"][5] == -2
    assert (t["n_ops"] == -1).any() and (t["n_ops"] > 0).any()
    assert sw.error_count() == 3 * 2   # three invalid slots, traced by both kernel families



@pytest.mark.parametrize("sc", [wl.Scoring(1, -4, 6, 1, 12), wl.Scoring(3, -200, 10, 3, 12)],
                         ids=["small-scores", "mismatch-200"])
def test_trace_other_scorings(sc):
    """Other scorings; a mismatch below -128 takes the compare-and-select
    substitution of the one-slot-per-lane sweep instead of the byte permutation."""
    import dataclasses
    b = wl.random_small_batch(79, n_reads=60, read_len=(1, 120), band=12)
    _case(dataclasses.replace(b, scoring=sc))

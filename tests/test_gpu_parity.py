"""GPU parity: the HIP path against the CPU oracle, element by element.

Scores and end positions are integers, so the bar is bit-exact equality of
every output (score, ref_end, read_end, best_score, best_slot, n_tied).
"""
import dataclasses

import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from paper_1805_00106_amd import workloads as wl
from tests.gpu_util import assert_same, gpu_align, oracle_align

pytestmark = pytest.mark.gpu

PRECISIONS = [sw.PREC_INT16, sw.PREC_INT32]


def _case(batch, precision, **kw):
    exp, _ = oracle_align(batch)
    if precision in (sw.PREC_INT16, sw.PREC_INT32) and "kernel" not in kw:
        # both kernel families: one CAL (int16) or one CAL strand (int32) per lane, and
        # one wavefront per task (int16: one CAL, both strands in the halves)
        for kernel in (sw.KERNEL_INTER, sw.KERNEL_INTRA):
            got = gpu_align(batch, precision, kernel=kernel, **kw)
            assert_same(got, exp, f"{batch.name} prec={precision} kernel={kernel} {kw}")
        return
    kw.setdefault("kernel", sw.KERNEL_INTER)
    got = gpu_align(batch, precision, **kw)
    assert_same(got, exp, f"{batch.name} prec={precision} {kw}")


def test_small_reference_int32_full():
    """Small-reference workload: 1000 x 76 bp reads, 2 CALs, both strands, int32."""
    _case(wl.small_reference(), sw.PREC_INT32)


def test_small_reference_int16():
    _case(wl.small_reference(), sw.PREC_INT16)


def test_auto_kernel_choice_small_and_large():
    """AUTO picks the wavefront-per-task kernel for tiny batches, one CAL per lane otherwise."""
    small = wl.random_small_batch(50, n_reads=20, read_len=(30, 150), band=20)
    _case(small, sw.PREC_AUTO, kernel=sw.KERNEL_AUTO)
    _case(wl.small_reference(n_reads=2000), sw.PREC_AUTO, kernel=sw.KERNEL_AUTO)


@pytest.mark.parametrize("seed", range(3))
def test_intra_long_reads_many_strips(seed):
    """Wide windows: several 64-column strips handed over through LDS (int32; int16
    pairs up to the 255-base read bound of the int16 path)."""
    b = wl.random_small_batch(60 + seed, n_reads=25, read_len=(150, 400), ref_len=(500, 5000), band=100)
    _case(b, sw.PREC_INT32, kernel=sw.KERNEL_INTRA, max_read_len=400)
    b16 = wl.random_small_batch(63 + seed, n_reads=25, read_len=(120, 255), ref_len=(500, 5000), band=150)
    _case(b16, sw.PREC_INT16, kernel=sw.KERNEL_INTRA, max_read_len=255)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("seed", range(6))
def test_random_ragged_small(seed, precision):
    """Ragged reads (1..60 bp), CALs near both reference ends (clipped windows),
    mixed strand masks, zero-CAL reads, two references."""
    _case(wl.random_small_batch(seed, n_reads=80, read_len=(1, 60), band=8), precision)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_long_reads_wide_band(precision):
    """L up to 250 with band 64: windows up to 378 columns (several 64-column tiles and strips)."""
    b = wl.random_small_batch(11, n_reads=40, read_len=(180, 250), ref_len=(300, 3000), band=64)
    _case(b, precision)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_homopolymers_maximal_ties(precision):
    b = wl.random_small_batch(12, n_reads=40, read_len=(1, 90), band=20, homopolymer=True)
    _case(b, precision)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_single_base_reads(precision):
    _case(wl.random_small_batch(13, n_reads=60, read_len=(1, 1), band=3), precision)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("sc", [wl.Scoring(1, 0, 0, 1, 10), wl.Scoring(3, -1, 1, 1, 10),
                                wl.Scoring(2, -3, 0, 2, 10), wl.Scoring(1, -4, 6, 1, 10),
                                wl.Scoring(2, -20, 5, 2, 10)])
def test_other_scorings(sc, precision):
    """Several scorings; a mismatch below -15 takes the int32 compare-and-select
    substitution instead of the byte permutation."""
    b = wl.random_small_batch(14, n_reads=60, read_len=(1, 80), band=10)
    b = dataclasses.replace(b, scoring=sc)
    _case(b, precision)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("mrl", [76, 100, 150, 250])
def test_strip_heights(mrl, precision):
    """Different read-length bounds pick different strip heights (rows per lane)."""
    b = wl.random_small_batch(15, n_reads=50, read_len=(1, min(mrl, 250)), band=16, ref_len=(300, 2000))
    _case(b, precision, max_read_len=mrl)


def test_invalid_cals_flagged():
    b = wl.random_small_batch(16, n_reads=30, max_cals=3)
    b.cal_pos = b.cal_pos.copy()
    b.cal_ref = b.cal_ref.copy()
    b.cal_pos[0] = b.ref_len[int(b.cal_ref[0])]
    b.cal_ref[1] = b.n_refs
    b.cal_pos[2] = -5
    sw.error_count(reset=True)
    exp, errs = oracle_align(b)
    got = gpu_align(b, sw.PREC_INT16)
    assert_same(got, exp, "invalid cals")
    assert sw.error_count() == errs > 0


def test_three_references_reduce_and_classify():
    b = wl.random_small_batch(17, n_refs=3, n_reads=100, max_cals=6, band=12)
    exp, _ = oracle_align(b)
    got = gpu_align(b, sw.PREC_INT16)
    assert_same(got, exp, "3 refs")
    from oracle import oracle as orc
    bs = torch.from_numpy(got["best_score"]).cuda()
    for thr in (0, 10, 40):
        cls = sw.classify(bs, thr).cpu().numpy()
        np.testing.assert_array_equal(cls, orc.classify(exp["best_score"], thr))


def test_chromosome_scale_shape_moderate():
    """Chromosome-scale generator (100 Mbp reference with repeats, 100 bp reads, Poisson(6)+1
    CALs, band 32, int16) at 5000 reads: full oracle parity."""
    _case(wl.chromosome_scale(n_reads=5000), sw.PREC_INT16)


def test_uneven_lengths_shape_moderate():
    """Uneven-lengths generator (L uniform 75..250, geometric CAL counts) at 1500 reads."""
    b = wl.uneven_lengths(n_reads=1500, band=64)
    _case(b, sw.PREC_INT16, max_read_len=250)


def test_maximum_read_length_and_wide_band():
    """Reads up to the library maximum (1024 bp) with band 200 (windows up to 1424
    columns): int32 on both kernel families; int16's bound does not hold here."""
    b = wl.random_small_batch(18, n_reads=10, read_len=(900, 1024), ref_len=(3000, 6000), band=200, max_cals=2)
    _case(b, sw.PREC_INT32, max_read_len=1024)
    with pytest.raises(sw.SwError):
        gpu_align(b, sw.PREC_INT16, max_read_len=1024)


def test_half_max_order_on_device():
    """The int16 sweep takes its three-way maxima from the packed half-precision
    maximum; every pair of operand patterns must keep the integer order."""
    assert sw.check_half_max() == 0


# The int16 sweep keeps (V + beta) * 2^K + tag in each half, plus r * gap_extend *
# 2^K on row r of a strip (at most 50 rows), beta covering the largest single
# penalty (|mismatch|, gap_open + gap_extend + 1, 256 / 2^K + gap_extend) and K the
# widest of 6, 5, 4 with (beta + match * max_read_len + 1 + 49 * gap_extend) * 2^K
# <= 0x7BFF.  Each case sits at an edge of that layout: values at the top of the
# range, each term setting beta, and each tag width.
TAG_EDGES = [
    # (match, mismatch, gap_open, gap_extend, max_read_len, read lengths): K, beta
    ((2, -3, 5, 2), 194, (150, 194)),     # K 6, beta 8: (8 + 388 + 1 + 98) * 64 = 31680, just inside
    ((2, -3, 5, 2), 195, (150, 195)),     # K 5 from one base more (beta 10 from the padding rows)
    ((2, -500, 5, 2), 250, (150, 250)),   # K 4, beta from the mismatch
    ((1, -1, 300, 2), 80, (1, 80)),       # K 6, beta 303 from the gap terms
    ((1, -400, 0, 1), 100, (1, 100)),     # K 5, beta 400 from the mismatch, no gap opening
    ((3, -1, 1, 1), 146, (100, 146)),     # K 6, beta 5 from the padding rows: (5 + 438 + 1 + 49) * 64 = 31552
    ((3, -1, 10, 29), 170, (150, 170)),   # K 4, beta 45, row offsets up to 49 * 29: (45 + 510 + 1 + 1421) * 16 = 31632
]


@pytest.mark.parametrize("mode", [sw.MODE_LOCAL, sw.MODE_FINAL_ROW])
@pytest.mark.parametrize("edge", TAG_EDGES, ids=[f"{e[0]}-L{e[1]}" for e in TAG_EDGES])
def test_int16_tag_width_and_bias_edges(edge, mode):
    (m, x, go, ge), mrl, lens = edge
    sc = wl.Scoring(m, x, go, ge, 12)
    for seed, homo in ((21, True), (22, False)):
        # homopolymer reads on homopolymer references reach the largest values the
        # layout must hold (every cell of the top rows scores match * row)
        b = wl.random_small_batch(seed, n_reads=30, read_len=lens, ref_len=(400, 1500), band=12,
                                  homopolymer=homo)
        b = dataclasses.replace(b, scoring=sc)
        if homo:
            # full windows and both strands for every CAL (the other seed keeps CALs
            # near the reference ends, with mixed strand masks)
            b = dataclasses.replace(b, cal_pos=np.full_like(b.cal_pos, 12), strand=np.full_like(b.strand, 3))
        exp, _ = oracle_align(b, mode=mode)
        for kernel in (sw.KERNEL_INTER, sw.KERNEL_INTRA):
            got = gpu_align(b, sw.PREC_INT16, kernel=kernel, max_read_len=mrl, mode=mode)
            assert_same(got, exp, f"{edge} homopolymer={homo} mode={mode} kernel={kernel}")
        if homo:
            # the top of the range is reached: the longest read with a CAL scores match * L
            has_cal = np.diff(b.cal_ptr) > 0
            assert int(exp["score"].max()) == m * int(b.read_len[has_cal].max())


# The int32 one-CAL-per-lane sweep holds V * 4096 + tag plus r * gap_extend * 4096
# on row r of a strip (match * max_read_len + 49 * gap_extend <= 2^19 - 2), and its
# substitution is one byte permutation when s + gap_extend lies in [-15, 16] for
# both scores, else a compare and select.
INT32_EDGES = [
    ((14, -3, 5, 2), 60, (1, 60)),          # match + ge = 16: byte permutation at its top
    ((15, -3, 5, 2), 60, (1, 60)),          # 17: compare and select
    ((2, -17, 5, 2), 60, (1, 60)),          # mismatch + ge = -15: byte permutation at its bottom
    ((2, -18, 5, 2), 60, (1, 60)),          # -16: compare and select
    ((511, -3, 5, 20), 1024, (900, 1024)),  # top of the range: 511 * 1024 + 49 * 20 = 524244
]


@pytest.mark.parametrize("mode", [sw.MODE_LOCAL, sw.MODE_FINAL_ROW])
@pytest.mark.parametrize("edge", INT32_EDGES, ids=[f"{e[0]}-L{e[1]}" for e in INT32_EDGES])
def test_int32_range_and_substitution_edges(edge, mode):
    (m, x, go, ge), mrl, lens = edge
    sc = wl.Scoring(m, x, go, ge, 12)
    for seed, homo in ((25, True), (26, False)):
        b = wl.random_small_batch(seed, n_reads=20, read_len=lens, ref_len=(1200, 3000), band=12,
                                  homopolymer=homo)
        b = dataclasses.replace(b, scoring=sc)
        if homo:
            b = dataclasses.replace(b, cal_pos=np.full_like(b.cal_pos, 12), strand=np.full_like(b.strand, 3))
        exp, _ = oracle_align(b, mode=mode)
        for kernel in (sw.KERNEL_INTER, sw.KERNEL_INTRA):
            got = gpu_align(b, sw.PREC_INT32, kernel=kernel, max_read_len=mrl, mode=mode)
            assert_same(got, exp, f"{edge} homopolymer={homo} mode={mode} kernel={kernel}")
        if homo:
            has_cal = np.diff(b.cal_ptr) > 0
            assert int(exp["score"].max()) == m * int(b.read_len[has_cal].max())


def test_empty_inputs():
    """No CALs at all, and reads without CALs: calls succeed and touch nothing."""
    b = wl.random_small_batch(19, n_reads=5, max_cals=0)
    assert b.n_cals == 0
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    sc = sw.Scoring.make(2, -3, 5, 2, 8, sw.PREC_AUTO, max_read_len=60)
    out = sw.align_batch(db, refs, sc)
    assert out.score.numel() == 0
    bs, bl, nt = sw.reduce_best(db, b.n_refs, out.score)
    torch.cuda.synchronize()
    assert (bs.cpu().numpy() == -1).all() and (bl.cpu().numpy() == -1).all() and (nt.cpu().numpy() == 0).all()
    ctx = sw.Context(5, 1)
    ctx.align(db, refs, sc, out)
    ctx.close()

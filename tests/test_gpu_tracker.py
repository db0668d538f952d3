"""GPU parity of the Score Tracker variants and the final-row (read-end-anchored)
mode against the oracle: bit-exact scores, ends, top-k lists and tie flags."""
import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from paper_1805_00106_amd import workloads as wl
from tests.gpu_util import SLOTS, assert_same, gpu_align, oracle_align, scoring_for

pytestmark = pytest.mark.gpu

FR = sw.MODE_FINAL_ROW
KERNELS = [(sw.PREC_INT16, sw.KERNEL_INTER), (sw.PREC_INT16, sw.KERNEL_INTRA), (sw.PREC_INT32, sw.KERNEL_INTER),
           (sw.PREC_INT32, sw.KERNEL_INTRA)]


def _fr_case(batch, **kw):
    exp, _ = oracle_align(batch, mode=FR)
    for prec, kern in KERNELS:
        got = gpu_align(batch, prec, kernel=kern, mode=FR, **kw)
        assert_same(got, exp, f"{batch.name} final-row prec={prec} kernel={kern} {kw}")
    assert np.all((exp["read_end"] == batch.read_len[_slot_read(batch)] - 1) | (exp["score"] <= 0))


def _slot_read(batch):
    return np.repeat(np.repeat(np.arange(batch.n_reads), np.diff(batch.cal_ptr)), 2)


@pytest.mark.parametrize("seed", range(4))
def test_final_row_ragged(seed):
    """Ragged reads 1..120 bp (several strips of rows), clipped windows, strand masks."""
    _fr_case(wl.random_small_batch(40 + seed, n_reads=90, read_len=(1, 120), band=10))


def test_final_row_long_reads_many_tiles():
    """Windows up to 378 columns: several 64-column tiles per strip."""
    b = wl.random_small_batch(45, n_reads=40, read_len=(150, 250), ref_len=(300, 3000), band=64)
    _fr_case(b, max_read_len=250)


def test_final_row_chromosome_scale_shape():
    _fr_case(wl.chromosome_scale(n_reads=2000))


def test_final_row_single_base_and_homopolymers():
    _fr_case(wl.random_small_batch(46, n_reads=60, read_len=(1, 1), band=3))
    _fr_case(wl.random_small_batch(47, n_reads=40, read_len=(1, 90), band=20, homopolymer=True))


def test_final_row_batched_context_replays():
    b = wl.uneven_lengths(n_reads=600, band=32)
    exp, _ = oracle_align(b, mode=FR)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    ctx = sw.Context(b.n_reads, b.n_cals)
    out = sw.Outputs(db.n_cals)
    for mode in (FR, sw.MODE_LOCAL, FR):
        want = exp if mode == FR else oracle_align(b)[0]
        sc = scoring_for(b, sw.PREC_INT16, max_read_len=250, mode=mode)
        for rep in range(2):
            out.score.fill_(-7)
            torch.cuda.synchronize()
            ctx.align(db, refs, sc, out)
            torch.cuda.synchronize()
            got = dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(),
                       read_end=out.read_end.cpu().numpy())
            assert_same(got, want, f"ctx mode={mode} rep={rep} ({ctx.last_plan()})", keys=SLOTS)
    ctx.close()


@pytest.mark.parametrize("k", [1, 3, 8, sw.MAX_TOPK])
def test_topk_and_tied_flags(k):
    b = wl.random_small_batch(50, n_reads=150, max_cals=12, n_refs=2, band=6, read_len=(1, 40))
    exp, _ = oracle_align(b, topk=k)
    got = gpu_align(b, sw.PREC_INT16, topk=k)
    assert_same(got, exp, f"top-{k}")


def test_topk_many_ties_and_invalid_slots():
    """Homopolymer reads give many equal scores; invalid CALs (INT32_MIN) and
    unrequested strands (-1) must be skipped."""
    b = wl.random_small_batch(51, n_reads=80, max_cals=10, band=8, read_len=(1, 30), homopolymer=True)
    b.cal_pos = b.cal_pos.copy()
    b.cal_pos[::5] = -3
    exp, errs = oracle_align(b, topk=4)
    assert errs > 0
    got = gpu_align(b, sw.PREC_INT16, topk=4)
    assert_same(got, exp, "top-4 with ties and invalid slots")


def test_alu_peak_is_plausible():
    """The calibration kernel's sustained rate is positive and below the
    published peak (256 CUs x 64 lanes x 2.4 GHz, x2 for packed 16-bit)."""
    p16 = sw.alu_peak(16, 1 << 14)
    p32 = sw.alu_peak(32, 1 << 14)
    assert 0.2 * 7.864e13 < p16 <= 1.02 * 7.864e13
    assert 0.2 * 3.932e13 < p32 <= 1.02 * 3.932e13


def test_malformed_row_pointer_is_clamped():
    """Rows of a malformed CSR row pointer (negative start, end past n_cals,
    decreasing entries) are clamped to [0, n_cals]: the best, top-k and tie-flag
    reductions equal the same reductions over the clamped rows, computed here."""
    b = wl.random_small_batch(61, n_reads=40, max_cals=4)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    sc = scoring_for(b, sw.PREC_INT16)
    out = sw.align_batch(db, refs, sc)
    n = db.n_cals
    bad = b.cal_ptr.copy()
    bad[3], bad[7], bad[8], bad[20], bad[-1] = -5, n + 100, 2, n + 3, n + 7
    rows = []
    for r in range(b.n_reads):
        a = min(max(int(bad[r]), 0), n)
        rows.append((a, min(max(int(bad[r + 1]), a), n)))
    bad_db = sw.DeviceBatch(db.reads2bit, db.read_word_off, db.read_len, torch.from_numpy(bad).cuda(), db.cal_pos,
                            db.cal_ref, db.strand)
    k = 3
    bs, bl, nt = sw.reduce_best(bad_db, b.n_refs, out.score)
    ts, tl = sw.topk(bad_db, out.score, k)
    fl_dev = torch.full((2 * n,), 7, dtype=torch.uint8, device="cuda")
    sw.lib().sw_tied_flags(sw._ptr(bad_db.cal_ptr), b.n_reads, n, sw._ptr(out.score), sw._ptr(fl_dev), None)
    torch.cuda.synchronize()
    s = out.score.cpu().numpy()
    ref = b.cal_ref.astype(np.int64)
    fl = fl_dev.cpu().numpy()
    cover = np.zeros(2 * n, dtype=np.int64)  # clamped rows may overlap: flags are checked where one row writes
    for a, e in rows:
        cover[2 * a:2 * e] += 1
    for r, (a, e) in enumerate(rows):
        slots = [(int(s[t]), t) for t in range(2 * a, 2 * e) if s[t] >= 0]
        for kk in range(b.n_refs):
            mine = [(v, t) for v, t in slots if ref[t // 2] == kk]
            best = max((v for v, _ in mine), default=-1)
            first = min((t for v, t in mine if v == best), default=-1)
            ties = sum(1 for v, _ in mine if v == best) if mine else 0
            assert (bs[r, kk].item(), bl[r, kk].item(), nt[r, kk].item()) == (best, first, ties), (r, kk)
        order = sorted(slots, key=lambda x: (-x[0], x[1]))[:k]
        want_s = [v for v, _ in order] + [-1] * (k - len(order))
        want_l = [t for _, t in order] + [-1] * (k - len(order))
        assert ts[r].cpu().tolist() == want_s and tl[r].cpu().tolist() == want_l, r
        top = max((v for v, _ in slots), default=-1)
        for t in range(2 * a, 2 * e):
            if cover[t] == 1:
                assert fl[t] == (1 if top >= 0 and s[t] == top else 0), (r, t)
    assert (fl[cover == 0] == 7).all()  # slots outside every row are not written

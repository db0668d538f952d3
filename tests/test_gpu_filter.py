"""GPU parity of the CAL Filter against the oracle (bit-exact kept CALs, strand
unions and input-to-kept map), and scoring through the filter: with exact
duplicates, every input CAL's result read through the map equals the oracle's
unfiltered result."""
import dataclasses

import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from oracle import oracle as orc
from paper_1805_00106_amd import workloads as wl
from tests.gpu_util import scoring_for

pytestmark = pytest.mark.gpu


def _gpu_filter(b, bits):
    db = sw.DeviceBatch.upload(b)
    kept, cmap = sw.cal_filter(db, bits)
    torch.cuda.synchronize()
    return db, kept, cmap


def _compare(b, bits):
    db, kept, cmap = _gpu_filter(b, bits)
    op, pos, ref, st, om = orc.cal_filter(b.cal_ptr, b.cal_pos, b.cal_ref, b.strand, b.n_reads, bits)
    np.testing.assert_array_equal(kept.cal_ptr.cpu().numpy(), op)
    np.testing.assert_array_equal(kept.cal_pos.cpu().numpy(), pos)
    np.testing.assert_array_equal(kept.cal_ref.cpu().numpy(), ref)
    np.testing.assert_array_equal(kept.strand.cpu().numpy(), st)
    np.testing.assert_array_equal(cmap.cpu().numpy(), om)
    return db, kept, cmap


@pytest.mark.parametrize("bits", [0, 2, 5, 12])
def test_filter_small_duplicated(bits):
    b = wl.with_duplicate_cals(wl.random_small_batch(95, n_reads=200, max_cals=6, band=8), 4)
    _compare(b, bits)


def test_filter_many_cals_one_read_and_empty_reads():
    rng = np.random.default_rng(96)
    ref = wl.uniform_genome(rng, 5000)
    reads = [wl.uniform_genome(rng, 50) for _ in range(5)]
    cals = [[], [(int(p), 0, int(s)) for p, s in zip(rng.integers(0, 300, 900), rng.integers(1, 4, 900))], [],
            [(7, 0, 1)] * 40, []]
    b = wl._pack_batch([ref], reads, cals, wl.Scoring(band=8), None, None, None, "many")
    for bits in (0, 3):
        _compare(b, bits)


def test_filter_chromosome_scale_scores_through_map():
    base = wl.chromosome_scale(n_reads=2000)
    b = wl.with_duplicate_cals(base, 5, jitter_frac=0.0)
    db, kept, cmap = _compare(b, 0)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    sc = scoring_for(b, sw.PREC_INT16, max_read_len=100)
    out = sw.align_batch(kept, refs, sc)
    torch.cuda.synchronize()
    s, r, e, _ = orc.align_batch(b, n_threads=8)
    cm = cmap.cpu().numpy()
    gs, gr, ge = out.score.cpu().numpy(), out.ref_end.cpu().numpy(), out.read_end.cpu().numpy()
    for h in (0, 1):
        req = (b.strand & (1 << h)) > 0
        c = np.nonzero(req)[0]
        k = 2 * cm[c] + h
        np.testing.assert_array_equal(gs[k], s[2 * c + h])
        np.testing.assert_array_equal(gr[k], r[2 * c + h])
        np.testing.assert_array_equal(ge[k], e[2 * c + h])
    assert kept.n_cals < b.n_cals / 2

"""The synthetic workloads follow their stated recipes (CPU, reduced sizes):
read lengths, CAL-count distributions, the true locus among each read's CALs,
the sequencing-error rate, planted repeats, the two-reference split, and the
served request and arrival distributions."""
import math

import numpy as np

from paper_1805_00106_amd import workloads as wl


def _forward_read(b, r):
    """Read r in forward orientation (undo the reverse complement of reverse-strand reads)."""
    q = b.read(r).astype(np.int64)
    return (3 - q[::-1]) if b.true_strand[r] else q


def _cal_rows(b):
    return [set(zip(b.cal_ref[b.cal_ptr[r]:b.cal_ptr[r + 1]].tolist(), b.cal_pos[b.cal_ptr[r]:b.cal_ptr[r + 1]].tolist()))
            for r in range(b.n_reads)]


def test_small_reference_recipe():
    b = wl.small_reference()
    assert b.n_reads == 1000 and b.n_refs == 1 and int(b.ref_len[0]) == 10_000
    assert (b.read_len == 76).all() and (np.diff(b.cal_ptr) == 2).all() and (b.strand == 3).all()
    comp = np.bincount(b.reference(0), minlength=4) / 10_000
    assert np.abs(comp - 0.25).max() < 0.02                      # uniform ACGT
    rows = _cal_rows(b)
    assert all((0, int(b.true_pos[r])) in rows[r] for r in range(b.n_reads))   # true locus is a CAL
    # substitution rate on reads without an indel (an indel shifts the rest of the read)
    ref = b.reference(0).astype(np.int64)
    ham = np.array([int((_forward_read(b, r) != ref[b.true_pos[r]:b.true_pos[r] + 76]).sum())
                    for r in range(b.n_reads)])
    clean = ham <= 6
    assert clean.mean() > 0.85
    assert 0.007 < ham[clean].sum() / (76 * clean.sum()) < 0.013   # 1% substitutions
    assert 0.4 < b.true_strand.mean() < 0.6


def test_chromosome_scale_recipe():
    b = wl.chromosome_scale(n_reads=20_000, ref_len=2_000_000)
    assert (b.read_len == 100).all() and b.scoring.band == 32
    counts = np.diff(b.cal_ptr)
    assert counts.min() >= 1 and abs(counts.mean() - 7.0) < 0.1     # Poisson(6) + 1
    assert abs(counts.var() - 6.0) < 0.4
    rows = _cal_rows(b)
    assert all((0, int(b.true_pos[r])) in rows[r] for r in range(b.n_reads))
    genome, copies = wl.chromosome_genome(2_000_000)
    covered = sum(int(c[2]) for c in copies)
    assert 0.045 < covered / 2_000_000 < 0.07                       # ~5% planted repeats
    lens = np.array([int(c[2]) for c in copies])
    assert lens.min() >= 300 * 0.8 and lens.max() <= 6000 * 1.2     # copies of 300..6000 bp sources


def test_uneven_lengths_recipe():
    b = wl.uneven_lengths(n_reads=20_000, ref_len=2_000_000, band=64)
    assert b.read_len.min() == 75 and b.read_len.max() == 250
    assert abs(b.read_len.mean() - 162.5) < 1.5                     # uniform on 75..250
    assert len(np.unique(b.read_len)) == 176
    counts = np.diff(b.cal_ptr)
    assert counts.min() >= 1 and counts.max() <= 64                # geometric, capped at 64
    assert abs(counts.mean() - 8.0) < 0.2                           # mean 8
    assert abs((counts == 1).mean() - 1 / 8) < 0.01                 # P(1) = p = 1/8
    assert b.scoring.band == 64


def test_two_references_recipe():
    b = wl.two_references(n_reads=20_000, ref_len=1_000_000)
    assert b.n_refs == 2 and (b.read_len == 150).all()
    assert abs(int(b.ref_len[1]) - int(b.ref_len[0])) < 0.01 * int(b.ref_len[0])   # indels roughly balanced
    assert abs(b.true_ref.mean() - 0.7) < 0.015                     # 70% of reads from B
    counts = np.diff(b.cal_ptr)
    assert abs(counts.mean() - 6.0) < 0.1                           # 2 homologous + Poisson(2) decoys per reference
    for r in range(0, b.n_reads, 97):
        sl = slice(b.cal_ptr[r], b.cal_ptr[r + 1])
        homologous = b.cal_decoy[sl] == 0
        assert sorted(b.cal_ref[sl][homologous].tolist()) == [0, 1]  # one homologous CAL on each reference
        src = int(b.true_ref[r])
        assert int(b.true_pos[r]) in b.cal_pos[sl][homologous & (b.cal_ref[sl] == src)].tolist()


def test_served_request_and_arrival_recipe():
    refs = wl.served_references(scale=0.001)
    assert [len(x) for x in refs] == [3_200_000, 2_700_000]
    b = wl.served_request(refs, 2_000, seed=3)
    assert b.read_len.min() >= 75 and b.read_len.max() <= 250
    counts = np.diff(b.cal_ptr)
    assert counts.min() >= 1 and counts.max() <= 32 and abs(counts.mean() - 16.5) < 0.6   # U{1..32}
    first = b.cal_ptr[:-1]
    assert (b.cal_ref[first] == b.true_ref).all() and (b.cal_pos[first] == b.true_pos).all()
    t, sizes = wl.served_arrivals(100.0, 5_000, seed=0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.01) < 0.0006 and abs(gaps.std() / gaps.mean() - 1) < 0.06   # exponential gaps
    assert sizes.min() >= 1 and sizes.max() <= 10_000
    assert 80 <= np.median(sizes) <= 125                            # log-uniform on [1, 10000]: median ~ 100
    assert abs((sizes <= 10).mean() - math.log(11) / math.log(10001)) < 0.03

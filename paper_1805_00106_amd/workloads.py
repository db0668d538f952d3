"""Seeded synthetic workloads: genomes, short reads and candidate alignment locations.

This module only *draws data*.  It holds none of the alignment arithmetic:
no scoring, no dynamic programming, no 2-bit packing and no window clipping.
Both the CPU oracle (through the tests) and the GPU path consume what it
returns, so it is the one piece of code they share.

Alphabet: every base is a code in {0, 1, 2, 3} standing for A, C, G, T, the
code order of the paper's index figure (section 3.1, Fig. 3).  Sequences are
returned as numpy ``uint8`` code arrays.

Layout of a batch (``Batch``):

* ``ref_codes``  uint8, all references concatenated; reference ``k`` occupies
  ``ref_codes[ref_off[k] : ref_off[k] + ref_len[k]]`` and ``ref_off[k]`` is a
  multiple of 16 (padding codes are 0).
* ``read_codes`` uint8, all reads concatenated the same way (each read starts
  at a multiple of 16).
* ``cal_ptr``    int64 [n_reads + 1], CSR row pointer of the CAL lists.
* ``cal_pos``    int64, forward-strand reference position of base 0 of the
  oriented read at that candidate location.
* ``cal_ref``    int16, reference id of each CAL.
* ``strand``     uint8, strand mask per CAL: 1 forward, 2 reverse, 3 both.

The workload recipes follow the shapes the paper reports: 75-250 bp reads
(abstract), 76 bp and 100 bp reads (sections 3.3 and 6.2), a long-tailed
CALs-per-read distribution (section 5.2, Fig. 9), a strand bit per CAL
(section 3.1) and a two-genome classification case study (section 6).  The
paper's data sets are not available; these seeded draws stand in for them.

Reverse-strand reads are simulated by sequencing the opposite strand of the
sampled locus (complement ``3 - code`` and reversal): that is part of the
sequencer model, independent of how the aligner treats strands.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

ROOT_SEED = 180500106
# Stream indices spawned from the root seed of every workload.
_STREAMS = ("reference", "repeats", "reads", "errors", "cals", "arrivals")


def seed_streams(config_index: int, extra: int = 0):
    """Independent PCG64 generators for one workload (one per draw stream)."""
    ss = np.random.SeedSequence([ROOT_SEED + config_index, extra])
    kids = ss.spawn(len(_STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k)) for name, k in zip(_STREAMS, kids)}


@dataclasses.dataclass
class Scoring:
    match: int = 2
    mismatch: int = -3
    gap_open: int = 5
    gap_extend: int = 2
    band: int = 32


@dataclasses.dataclass
class Batch:
    ref_codes: np.ndarray
    ref_off: np.ndarray
    ref_len: np.ndarray
    read_codes: np.ndarray
    read_off: np.ndarray
    read_len: np.ndarray
    cal_ptr: np.ndarray
    cal_pos: np.ndarray
    cal_ref: np.ndarray
    strand: np.ndarray
    scoring: Scoring
    # planted truth per read: source reference, forward start, strand (0 fwd / 1 rev)
    true_ref: Optional[np.ndarray] = None
    true_pos: Optional[np.ndarray] = None
    true_strand: Optional[np.ndarray] = None
    name: str = ""
    # per CAL: 1 if it was drawn as a decoy (uniform position), when the generator knows
    cal_decoy: Optional[np.ndarray] = None

    @property
    def n_reads(self) -> int:
        return int(self.read_len.shape[0])

    @property
    def n_cals(self) -> int:
        return int(self.cal_pos.shape[0])

    @property
    def n_refs(self) -> int:
        return int(self.ref_len.shape[0])

    def reference(self, k: int) -> np.ndarray:
        o = int(self.ref_off[k])
        return self.ref_codes[o:o + int(self.ref_len[k])]

    def read(self, r: int) -> np.ndarray:
        o = int(self.read_off[r])
        return self.read_codes[o:o + int(self.read_len[r])]

    def subset_reads(self, idx: np.ndarray) -> "Batch":
        """A batch holding only the reads ``idx`` (same references)."""
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.read_len[idx]
        offs, total = aligned_offsets(lens)
        codes = np.zeros(total, dtype=np.uint8)
        for k, r in enumerate(idx):
            codes[offs[k]:offs[k] + lens[k]] = self.read(int(r))
        counts = self.cal_ptr[idx + 1] - self.cal_ptr[idx]
        ptr = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(counts, out=ptr[1:])
        sel = np.concatenate([np.arange(self.cal_ptr[r], self.cal_ptr[r + 1]) for r in idx]) \
            if len(idx) else np.zeros(0, dtype=np.int64)
        sel = sel.astype(np.int64)
        pick = (lambda a: None if a is None else a[idx])
        return Batch(self.ref_codes, self.ref_off, self.ref_len, codes, offs, lens.astype(np.int32),
                     ptr, self.cal_pos[sel], self.cal_ref[sel], self.strand[sel], self.scoring,
                     pick(self.true_ref), pick(self.true_pos), pick(self.true_strand), self.name,
                     None if self.cal_decoy is None else self.cal_decoy[sel])


def aligned_offsets(lengths: np.ndarray, align: int = 16):
    """Start offsets placing each sequence at a multiple of ``align``."""
    lengths = np.asarray(lengths, dtype=np.int64)
    padded = (lengths + align - 1) // align * align
    offs = np.zeros(len(lengths), dtype=np.int64)
    if len(lengths):
        np.cumsum(padded[:-1], out=offs[1:])
    total = int(padded.sum()) if len(lengths) else 0
    return offs, total


def concat_aligned(seqs: List[np.ndarray]):
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offs, total = aligned_offsets(lens)
    out = np.zeros(total, dtype=np.uint8)
    for s, o in zip(seqs, offs):
        out[o:o + len(s)] = s
    return out, offs, lens


def uniform_genome(rng: np.random.Generator, n: int, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Uniform i.i.d. ACGT codes (four codes per random byte).  With ``out`` (a
    uint8 array of n codes), the codes are written there in place."""
    nbytes = (n + 3) // 4
    raw = rng.integers(0, 256, nbytes, dtype=np.uint8)
    if out is None:
        full = np.empty(nbytes * 4, dtype=np.uint8)
        for k in range(4):
            full[k::4] = (raw >> (2 * k)) & 3
        return full[:n]
    assert out.dtype == np.uint8 and out.shape == (n,)
    for k in range(4):
        dst = out[k::4]
        np.bitwise_and(np.right_shift(raw[:dst.shape[0]], 2 * k), 3, out=dst)
    return out


def _substitute(rng: np.random.Generator, codes: np.ndarray, rate: float) -> np.ndarray:
    """Replace each base with probability ``rate`` by one of the 3 other bases."""
    hit = rng.random(codes.shape) < rate
    shift = rng.integers(1, 4, codes.shape, dtype=np.uint8)
    return np.where(hit, (codes + shift) & 3, codes).astype(np.uint8)


def _mutate_with_indels(rng: np.random.Generator, seq: np.ndarray, sub_rate: float,
                        indel_rate: float):
    """Substitutions plus indel events (length U{1..3}, insertion/deletion 50/50).

    Returns the mutated sequence and, for every input position, the index of the
    output base it became (or the next surviving one for deleted bases).
    """
    n = len(seq)
    out = _substitute(rng, seq, sub_rate)
    n_ev = rng.binomial(n, indel_rate) if indel_rate > 0 else 0
    keep = np.ones(n, dtype=np.int64)
    ins_after = np.zeros(n, dtype=np.int64)
    if n_ev:
        pos = rng.integers(0, n, n_ev)
        ln = rng.integers(1, 4, n_ev)
        is_del = rng.random(n_ev) < 0.5
        dp, dl = pos[is_del], ln[is_del]
        for k in range(3):  # deletion lengths are 1..3
            sel = dl > k
            keep[np.minimum(dp[sel] + k, n - 1)] = 0
        np.add.at(ins_after, pos[~is_del], ln[~is_del])
    counts = keep + ins_after
    total = int(counts.sum())
    res = np.empty(total, dtype=np.uint8)
    starts = np.zeros(n, dtype=np.int64)
    np.cumsum(counts[:-1], out=starts[1:])
    kept = keep.astype(bool)
    res[starts[kept]] = out[kept]
    if n_ev:
        # inserted bases fill the slots after each kept/deleted position
        slot_mask = np.ones(total, dtype=bool)
        slot_mask[starts[kept]] = False
        res[slot_mask] = rng.integers(0, 4, int(slot_mask.sum()), dtype=np.uint8)
    return res, starts


def plant_repeats(rng: np.random.Generator, genome: np.ndarray, fraction: float):
    """Overwrite ``fraction`` of the genome with diverged copies of repeat families.

    Families have a source of length U[300, 6000]; each copy is placed at a random
    position and diverged by U[2%, 10%] (90% substitutions, 10% short indels).
    Returns a list of copies ``(family, start, length)``.
    """
    n = len(genome)
    target = int(fraction * n)
    copies = []
    covered = 0
    fam = 0
    while covered < target:
        src_len = int(rng.integers(300, 6001))
        src = uniform_genome(rng, src_len)
        n_copies = int(rng.integers(2, 11))
        for _ in range(n_copies):
            div = float(rng.uniform(0.02, 0.10))
            cp, _ = _mutate_with_indels(rng, src, 0.9 * div, 0.1 * div / 2.0)
            start = int(rng.integers(0, max(1, n - len(cp))))
            genome[start:start + len(cp)] = cp[: n - start]
            copies.append((fam, start, min(len(cp), n - start)))
            covered += len(cp)
            if covered >= target:
                break
        fam += 1
    return copies


def _repeat_index(copies):
    if not copies:
        return None
    arr = np.array(copies, dtype=np.int64)
    order = np.argsort(arr[:, 1])
    return arr[order]


def _sample_reads_matrix(rng_reads, rng_err, genome: np.ndarray, lens: np.ndarray, sub_rate: float,
                         indel_rate: float, strand_p_rev: float = 0.5):
    """Draw reads from ``genome`` with the sequencer error model.

    Returns ([n, max_len] uint8 code matrix, row r valid up to lens[r]; start
    positions; strand flags).
    """
    n = len(lens)
    glen = len(genome)
    lens = np.asarray(lens, dtype=np.int64)
    span = lens + 8
    pos = (rng_reads.random(n) * (glen - span)).astype(np.int64)
    rev = rng_reads.random(n) < strand_p_rev
    maxspan = int(span.max()) if n else 0
    Lmax = int(lens.max()) if n else 0
    idx = pos[:, None] + np.arange(maxspan)[None, :]
    np.minimum(idx, glen - 1, out=idx)
    seg = _substitute(rng_err, genome[idx], sub_rate)
    mat = np.ascontiguousarray(seg[:, :Lmax])
    n_ev = rng_err.binomial(lens, indel_rate) if indel_rate > 0 else np.zeros(n, np.int64)
    for r in np.nonzero(n_ev)[0]:
        L = int(lens[r])
        row = seg[r].copy()
        for _ in range(int(n_ev[r])):
            p = int(rng_err.integers(2, L - 2))
            ln = int(rng_err.integers(1, 4))
            if rng_err.random() < 0.5:
                row = np.concatenate([row[:p], row[p + ln:]])
            else:
                row = np.concatenate([row[:p], rng_err.integers(0, 4, ln, dtype=np.uint8), row[p:]])
        if len(row) < L:  # many deletions ate the slack: extend with random bases
            row = np.concatenate([row, rng_err.integers(0, 4, L - len(row), dtype=np.uint8)])
        mat[r, :L] = row[:L]
    col = np.arange(Lmax)[None, :]
    rr = np.nonzero(rev)[0]
    if len(rr):
        src = lens[rr, None] - 1 - col
        ok = src >= 0
        vals = 3 - mat[rr[:, None], np.maximum(src, 0)]
        mat[rr] = np.where(ok, vals, 0).astype(np.uint8)
    mat[col >= lens[:, None]] = 0
    return mat, pos, rev


def _sample_reads(rng_reads, rng_err, genome: np.ndarray, lens: np.ndarray, sub_rate: float,
                  indel_rate: float, strand_p_rev: float = 0.5):
    """As _sample_reads_matrix, with the reads as a list of code arrays."""
    mat, pos, rev = _sample_reads_matrix(rng_reads, rng_err, genome, lens, sub_rate, indel_rate, strand_p_rev)
    return [mat[r, :int(lens[r])].copy() for r in range(len(lens))], pos, rev


def _pack_batch(refs, reads, cal_lists, scoring, true_ref, true_pos, true_strand, name):
    ref_codes, ref_off, ref_len = concat_aligned(refs)
    read_codes, read_off, read_len = concat_aligned(reads)
    counts = np.array([len(c) for c in cal_lists], dtype=np.int64)
    ptr = np.zeros(len(reads) + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    if len(cal_lists):
        allc = np.concatenate([np.asarray(c, dtype=np.int64).reshape(-1, 3) for c in cal_lists]) \
            if counts.sum() else np.zeros((0, 3), np.int64)
    else:
        allc = np.zeros((0, 3), np.int64)
    return Batch(ref_codes, ref_off, ref_len.astype(np.int64), read_codes, read_off,
                 read_len.astype(np.int32), ptr, allc[:, 0].astype(np.int64),
                 allc[:, 1].astype(np.int16), allc[:, 2].astype(np.uint8), scoring,
                 true_ref, true_pos, true_strand, name)


def _vector_batch(refs, read_codes_mat, lens, cal_counts, cal_pos, cal_ref, strand, scoring,
                  true_ref, true_pos, true_strand, name):
    """Fast path when reads come as a dense [n, Lmax] matrix."""
    ref_codes, ref_off, ref_len = concat_aligned(refs)
    offs, total = aligned_offsets(lens)
    rc = np.zeros(total, dtype=np.uint8)
    Lmax = read_codes_mat.shape[1]
    col = np.arange(Lmax)
    m = col[None, :] < lens[:, None]
    dst = (offs[:, None] + col[None, :])[m]
    rc[dst] = read_codes_mat[m]
    ptr = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(cal_counts, out=ptr[1:])
    return Batch(ref_codes, ref_off, ref_len.astype(np.int64), rc, offs, lens.astype(np.int32), ptr,
                 cal_pos.astype(np.int64), cal_ref.astype(np.int16), strand.astype(np.uint8), scoring,
                 true_ref, true_pos, true_strand, name)


def _reads_matrix(reads, lens):
    Lmax = int(lens.max()) if len(lens) else 0
    mat = np.zeros((len(reads), Lmax), dtype=np.uint8)
    for i, r in enumerate(reads):
        mat[i, :len(r)] = r
    return mat


def _shuffle_rows(rng, counts, *arrays):
    """Shuffle CAL order inside each read's list (CSR groups)."""
    n = int(counts.sum())
    grp = np.repeat(np.arange(len(counts)), counts)
    key = grp.astype(np.float64) + rng.random(n) * 0.5
    order = np.argsort(key, kind="stable")
    return [a[order] for a in arrays]


# --------------------------------------------------------------------------- configs

def small_reference(n_reads: int = 1000, ref_len: int = 10_000, read_len: int = 76) -> Batch:
    """Plain, small: 10 kbp uniform reference, 76 bp reads, true locus + 1 decoy CAL."""
    g = seed_streams(1)
    genome = uniform_genome(g["reference"], ref_len)
    lens = np.full(n_reads, read_len, dtype=np.int64)
    mat, pos, rev = _sample_reads_matrix(g["reads"], g["errors"], genome, lens, 0.01, 0.001)
    decoy = g["cals"].integers(0, ref_len, n_reads)
    counts = np.full(n_reads, 2, dtype=np.int64)
    cal_pos = np.stack([pos, decoy], 1).reshape(-1)
    cal_ref = np.zeros(2 * n_reads, dtype=np.int64)
    strand = np.full(2 * n_reads, 3, dtype=np.int64)
    cal_pos, cal_ref, strand = _shuffle_rows(g["cals"], counts, cal_pos, cal_ref, strand)
    sc = Scoring(2, -3, 5, 2, 32)
    return _vector_batch([genome], mat, lens, counts, cal_pos, cal_ref, strand,
                         sc, np.zeros(n_reads, np.int64), pos, rev.astype(np.int64), "small_reference")


def _repeat_genome(config_index: int, ref_len: int, repeat_fraction: float = 0.05):
    g = seed_streams(config_index)
    genome = uniform_genome(g["reference"], ref_len)
    copies = plant_repeats(g["repeats"], genome, repeat_fraction)
    return genome, copies


_GENOME_CACHE = {}


def chromosome_genome(ref_len: int = 100_000_000):
    """The 100 Mbp reference shared by the chromosome-scale workloads (seeded once)."""
    key = ref_len
    if key not in _GENOME_CACHE:
        _GENOME_CACHE[key] = _repeat_genome(2, ref_len)
    return _GENOME_CACHE[key]


def _homolog_cals(rng, rep, pos, lens, want):
    """Up to ``want[r]`` positions in other copies of a repeat family the read overlaps."""
    out = [[] for _ in range(len(pos))]
    if rep is None:
        return out
    starts = rep[:, 1]
    ends = rep[:, 1] + rep[:, 2]
    fam_of = rep[:, 0]
    by_fam = {}
    for k, f in enumerate(fam_of):
        by_fam.setdefault(int(f), []).append(k)
    # candidate copy: the last copy starting at or before the read
    k = np.searchsorted(starts, pos, side="right") - 1
    for r in np.nonzero((k >= 0) & (want > 0))[0]:
        kk = int(k[r])
        if pos[r] + lens[r] > ends[kk] + lens[r] // 2:
            continue
        off = int(pos[r] - starts[kk])
        sib = [j for j in by_fam[int(fam_of[kk])] if j != kk]
        rng.shuffle(sib)
        for j in sib[: int(want[r])]:
            out[r].append(int(starts[j] + off))
    return out


def _multi_cal_batch(g, genome, copies, n_reads, lens, counts, band, name, sc_int16=True,
                     sub_rate=0.01, indel_rate=0.001):
    ref_len = len(genome)
    mat, pos, rev = _sample_reads_matrix(g["reads"], g["errors"], genome, lens, sub_rate, indel_rate)
    rep = _repeat_index(copies)
    homs = _homolog_cals(g["cals"], rep, pos, lens, counts - 1)
    total = int(counts.sum())
    cal_pos = g["cals"].integers(0, ref_len, total).astype(np.int64)  # decoys by default
    starts = np.zeros(n_reads, dtype=np.int64)
    np.cumsum(counts[:-1], out=starts[1:])
    cal_pos[starts] = pos
    for r in range(n_reads):
        h = homs[r]
        if h:
            cal_pos[starts[r] + 1: starts[r] + 1 + len(h)] = np.minimum(np.array(h, np.int64), ref_len - 1)
    cal_ref = np.zeros(total, dtype=np.int64)
    strand = np.full(total, 3, dtype=np.int64)
    cal_pos, cal_ref, strand = _shuffle_rows(g["cals"], counts, cal_pos, cal_ref, strand)
    sc = Scoring(2, -3, 5, 2, band)
    return _vector_batch([genome], mat, lens, counts, cal_pos, cal_ref, strand,
                         sc, np.zeros(n_reads, np.int64), pos, rev.astype(np.int64), name)


def chromosome_scale(n_reads: int = 1_000_000, ref_len: int = 100_000_000, read_len: int = 100,
            reads_seed: int = 0) -> Batch:
    """Plain, chromosome scale: 100 Mbp with 5% planted repeats, 100 bp reads,
    Poisson(6)+1 CALs (true locus, repeat homologs, uniform decoys), band 32."""
    genome, copies = chromosome_genome(ref_len)
    g = seed_streams(2, 1 + reads_seed)
    lens = np.full(n_reads, read_len, dtype=np.int64)
    counts = g["cals"].poisson(6.0, n_reads).astype(np.int64) + 1
    return _multi_cal_batch(g, genome, copies, n_reads, lens, counts, 32, "chromosome_scale")


def uneven_lengths(n_reads: int = 2_000_000, ref_len: int = 100_000_000, band: int = 32,
            reads_seed: int = 0) -> Batch:
    """Batched, uneven: same reference, L uniform in [75, 250], CAL count
    geometric with mean 8 capped at 64, band in {16, 32, 64}."""
    genome, copies = chromosome_genome(ref_len)
    g = seed_streams(3, 1 + reads_seed)
    lens = g["reads"].integers(75, 251, n_reads).astype(np.int64)
    counts = np.minimum(g["cals"].geometric(1.0 / 8.0, n_reads), 64).astype(np.int64)
    return _multi_cal_batch(g, genome, copies, n_reads, lens, counts, band, f"uneven_lengths_band{band}")


def two_references(n_reads: int = 4_000_000, ref_len: int = 500_000_000, read_len: int = 150,
            reads_seed: int = 0) -> Batch:
    """Two-reference classification: A uniform, B = A + 15% substitutions + 2%/base
    indel events; reads 70% from B, 30% from A; per reference the homologous locus
    plus Poisson(2) uniform decoys; band 32, both strands."""
    g = seed_streams(4)
    A = uniform_genome(g["reference"], ref_len)
    B, a2b = _mutate_with_indels(g["repeats"], A, 0.15, 0.02 / 2.0)
    gr = seed_streams(4, 1 + reads_seed)
    lens = np.full(n_reads, read_len, dtype=np.int64)
    from_b = gr["reads"].random(n_reads) < 0.7
    nb = int(from_b.sum())
    mat = np.zeros((n_reads, read_len), dtype=np.uint8)
    src_pos = np.zeros(n_reads, dtype=np.int64)
    rev = np.zeros(n_reads, dtype=bool)
    for flag, genome in ((True, B), (False, A)):
        idx = np.nonzero(from_b == flag)[0]
        mm, pp, vv = _sample_reads_matrix(gr["reads"], gr["errors"], genome, lens[idx], 0.01, 0.0)
        mat[idx] = mm
        src_pos[idx] = pp
        rev[idx] = vv
    # homologous locus on the other reference through the coordinate map
    b2a = np.clip(np.searchsorted(a2b, np.minimum(src_pos, len(B) - 1), side="right") - 1, 0, ref_len - 1)
    pos_a = np.where(from_b, b2a, src_pos)
    pos_b = np.where(from_b, src_pos, a2b[np.minimum(src_pos, ref_len - 1)])
    nd_a = gr["cals"].poisson(2.0, n_reads)
    nd_b = gr["cals"].poisson(2.0, n_reads)
    counts = 2 + nd_a + nd_b
    total = int(counts.sum())
    cal_pos = np.zeros(total, dtype=np.int64)
    cal_ref = np.zeros(total, dtype=np.int64)
    starts = np.zeros(n_reads, dtype=np.int64)
    np.cumsum(counts[:-1], out=starts[1:])
    cal_pos[starts] = pos_a
    cal_ref[starts] = 0
    cal_pos[starts + 1] = pos_b
    cal_ref[starts + 1] = 1
    grp = np.repeat(np.arange(n_reads), counts)
    rank = np.arange(total) - starts[grp]
    dec = rank >= 2
    dec_ref = (rank - 2 >= nd_a[grp]).astype(np.int64)
    cal_ref[dec] = dec_ref[dec]
    lim = np.where(cal_ref == 0, ref_len, len(B))
    cal_pos[dec] = (gr["cals"].random(int(dec.sum())) * lim[dec]).astype(np.int64)
    strand = np.full(total, 3, dtype=np.int64)
    cal_pos, cal_ref, strand, decoy = _shuffle_rows(gr["cals"], counts, cal_pos, cal_ref, strand,
                                                    dec.astype(np.uint8))
    sc = Scoring(2, -3, 5, 2, 32)
    b = _vector_batch([A, B], mat, lens, counts, cal_pos, cal_ref, strand, sc,
                      from_b.astype(np.int64), src_pos, rev.astype(np.int64), "two_references")
    b.cal_decoy = decoy
    return b


def random_small_batch(seed: int, n_refs: int = 2, ref_len=(40, 400), n_reads: int = 50,
                       read_len=(1, 60), max_cals: int = 4, band: int = 8,
                       scoring: Optional[Scoring] = None, strand_choices=(1, 2, 3),
                       homopolymer: bool = False) -> Batch:
    """Small mixed batch for parity and edge cases: ragged read lengths, CALs near
    both reference ends, mixed strand masks, optional homopolymer sequences."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 99, seed])))
    refs = []
    for _ in range(n_refs):
        n = int(rng.integers(ref_len[0], ref_len[1] + 1))
        refs.append(np.zeros(n, np.uint8) if homopolymer else uniform_genome(rng, n))
    reads, cals = [], []
    for _ in range(n_reads):
        L = int(rng.integers(read_len[0], read_len[1] + 1))
        k = int(rng.integers(0, n_refs))
        ref = refs[k]
        if homopolymer:
            rd = np.zeros(L, np.uint8)
        elif rng.random() < 0.7 and len(ref) > L:
            p = int(rng.integers(0, len(ref) - L + 1))
            rd = _substitute(rng, ref[p:p + L].copy(), 0.05)
            if rng.random() < 0.5:
                rd = (3 - rd[::-1]).astype(np.uint8)
        else:
            rd = uniform_genome(rng, L)
        reads.append(rd)
        nc = int(rng.integers(0, max_cals + 1))
        lst = []
        for _ in range(nc):
            kk = int(rng.integers(0, n_refs))
            m = len(refs[kk])
            choice = rng.random()
            if choice < 0.2:
                p = int(rng.integers(0, min(m, 5)))           # near the start
            elif choice < 0.4:
                p = int(rng.integers(max(0, m - 5), m))       # near the end
            else:
                p = int(rng.integers(0, m))
            lst.append((p, kk, int(rng.choice(strand_choices))))
        cals.append(lst)
    sc = scoring or Scoring(2, -3, 5, 2, band)
    sc = dataclasses.replace(sc, band=band) if scoring is None else sc
    return _pack_batch(refs, reads, cals, sc, None, None, None, f"small{seed}")


# --------------------------------------------------------------------------- serving

def served_references(scale: float = 1.0):
    """Two resident references (3.2 Gbp and 2.7 Gbp at scale 1), random with 5%
    planted repeats."""
    codes, offs, lens = served_reference_pack(scale)
    return [codes[int(o):int(o) + int(n)] for o, n in zip(offs, lens)]


def served_reference_pack(scale: float = 1.0, progress=None):
    """The two served references drawn straight into one concatenated code array
    (each at a 16-aligned offset), as (codes, offsets, lengths): the same codes
    as ``served_references`` without a second copy.  ``progress(msg)`` is called
    after each reference."""
    g = seed_streams(5)
    lens = np.array([int(3.2e9 * scale), int(2.7e9 * scale)], dtype=np.int64)
    offs, total = aligned_offsets(lens)
    codes = np.zeros(total, dtype=np.uint8)
    for k, n in enumerate(lens):
        genome = codes[int(offs[k]):int(offs[k]) + int(n)]
        uniform_genome(g["reference"], int(n), out=genome)
        plant_repeats(g["repeats"], genome, 0.05 if scale >= 0.01 else 0.0)
        if progress:
            progress(f"served reference {k}: {int(n):,} bases drawn")
    return codes, offs, lens


def long_reference(n_reads: int = 600, long_len: int = (1 << 32) + 3_000_005, patch: int = 4096,
                   read_len=(75, 250), band: int = 32) -> Batch:
    """Reads on a reference longer than 2^32 bases, at the positions where 64-bit
    reference coordinates matter: around 2^31 and 2^32, near both ends, and in
    between.  Reference 0 is a short random sequence, so the long one (reference
    1) starts past word 0.  The long reference is all code 0 except random
    patches of ``patch`` bases around those loci: the array is allocated lazily,
    so only the patches take host memory.  Reads (length uniform in
    ``read_len``, 1% substitutions, either strand) come from the patches; each
    has its true locus plus 1..5 decoys in other patches (either reference),
    with both strands requested.  ``ref_patches`` lists the stretches that hold
    random codes (everything else is code 0)."""
    g = seed_streams(9)
    short = uniform_genome(g["reference"], 10_000)
    loci = [0, 1 << 30, (1 << 31) - patch // 2, (1 << 31) + patch, 3_000_000_000, (1 << 32) - patch // 2,
            (1 << 32) + patch, long_len - patch]
    lens = np.array([len(short), long_len], dtype=np.int64)
    offs, total = aligned_offsets(lens)
    ref_codes = np.zeros(total, dtype=np.uint8)  # lazily zero: untouched pages take no memory
    ref_codes[offs[0]:offs[0] + lens[0]] = short
    patches = [(0, 0, len(short))]
    for a in loci:
        a = int(min(max(a, 0), long_len - patch))
        ref_codes[offs[1] + a:offs[1] + a + patch] = uniform_genome(g["reference"], patch)
        patches.append((1, a, patch))
    rr, re_ = g["reads"], g["errors"]
    L = rr.integers(read_len[0], read_len[1] + 1, n_reads)
    mat = np.zeros((n_reads, int(L.max())), dtype=np.uint8)
    src = rr.integers(0, len(patches), n_reads)
    true_ref = np.zeros(n_reads, np.int64)
    true_pos = np.zeros(n_reads, np.int64)
    rev = rr.integers(0, 2, n_reads)
    for i in range(n_reads):
        k, a, n = patches[src[i]]
        start = a + int(rr.integers(0, n - L[i] + 1))
        seq = ref_codes[offs[k] + start:offs[k] + start + L[i]].copy()
        seq = _substitute(re_, seq, 0.01)
        if rev[i]:
            seq = (3 - seq)[::-1]
        mat[i, :L[i]] = seq
        true_ref[i], true_pos[i] = k, start
    counts = 1 + g["cals"].integers(1, 6, n_reads)
    cal_pos, cal_ref = [], []
    for i in range(n_reads):
        cal_pos.append(true_pos[i])
        cal_ref.append(true_ref[i])
        for _ in range(counts[i] - 1):
            k, a, n = patches[int(g["cals"].integers(0, len(patches)))]
            cal_pos.append(a + int(g["cals"].integers(0, max(1, n - L[i]))))
            cal_ref.append(k)
    cal_pos = np.array(cal_pos, np.int64)
    cal_ref = np.array(cal_ref, np.int64)
    strand = np.full(len(cal_pos), 3, np.int64)
    b = _vector_batch([np.zeros(1, np.uint8)], mat, L.astype(np.int64), counts, cal_pos, cal_ref, strand,
                      Scoring(2, -3, 5, 2, band), true_ref, true_pos, rev.astype(np.int64), "long_reference")
    b.ref_codes, b.ref_off, b.ref_len = ref_codes, offs, lens
    b.ref_patches = patches  # (reference, start, length) of every stretch that is not all code 0
    return b


def served_arrivals(rate_per_s: float, n_requests: int, seed: int = 0):
    """Poisson arrival times (seconds) and request sizes, log-uniform on [1, 10000] reads."""
    g = seed_streams(5, 100 + seed)
    gaps = g["arrivals"].exponential(1.0 / rate_per_s, n_requests)
    t = np.cumsum(gaps)
    sizes = np.floor(np.exp(g["arrivals"].uniform(0.0, math.log(10001.0), n_requests))).astype(np.int64)
    sizes = np.clip(sizes, 1, 10000)
    return t, sizes


def served_request(refs, n_reads: int, seed: int, band: int = 32, ref_pack=None) -> Batch:
    """One served request: reads of length U{75..250} with U{1..32} CALs on random
    references (the first CAL is the true locus).  ``ref_pack`` = (codes, offsets,
    lengths) of the concatenated references, shared instead of copied."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED + 5, 7, seed])))
    lens = rng.integers(75, 251, n_reads).astype(np.int64)
    src = rng.integers(0, len(refs), n_reads)
    mat = np.zeros((n_reads, int(lens.max())), np.uint8)
    pos = np.zeros(n_reads, np.int64)
    rev = np.zeros(n_reads, bool)
    for k in range(len(refs)):
        idx = np.nonzero(src == k)[0]
        if len(idx) == 0:
            continue
        mm, pp, vv = _sample_reads_matrix(rng, rng, refs[k], lens[idx], 0.01, 0.001)
        mat[idx, :mm.shape[1]] = mm
        pos[idx] = pp
        rev[idx] = vv
    counts = rng.integers(1, 33, n_reads).astype(np.int64)
    total = int(counts.sum())
    cal_ref = rng.integers(0, len(refs), total).astype(np.int64)
    lim = np.array([len(r) for r in refs], dtype=np.int64)[cal_ref]
    cal_pos = (rng.random(total) * lim).astype(np.int64)
    starts = np.zeros(n_reads, np.int64)
    np.cumsum(counts[:-1], out=starts[1:])
    cal_pos[starts] = pos
    cal_ref[starts] = src
    strand = np.full(total, 3, np.int64)
    sc = Scoring(2, -3, 5, 2, band)
    b = _vector_batch([], mat, lens, counts, cal_pos, cal_ref, strand, sc,
                      src.astype(np.int64), pos, rev.astype(np.int64), f"request{seed}")
    if ref_pack is None:
        ref_pack = concat_aligned(list(refs))
    b.ref_codes, b.ref_off, b.ref_len = ref_pack[0], ref_pack[1], np.asarray(ref_pack[2], np.int64)
    return b


def with_duplicate_cals(batch: Batch, seed: int = 0, mean_copies: float = 4.0, jitter_frac: float = 0.3,
                        max_jitter: int = 3, split_strands: bool = True) -> Batch:
    """The CAL stream a seed index hands to the CAL Filter (section 3.3): every
    CAL of ``batch`` arrives several times, once per seed that hit it (1 +
    Poisson(mean_copies - 1) copies), a fraction of the copies shifted by a few
    bases (seeds on the far side of an indel), and with ``split_strands`` a
    both-strand CAL may arrive as separate forward and reverse copies.  The
    copies of a read are shuffled.  References and reads are unchanged."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 77, seed])))
    n = batch.n_cals
    copies = 1 + rng.poisson(max(mean_copies - 1.0, 0.0), n)
    src = np.repeat(np.arange(n), copies)
    pos = batch.cal_pos[src].copy()
    shift = rng.random(len(src)) < jitter_frac
    first = np.zeros(len(src), dtype=bool)
    first[np.cumsum(copies) - copies] = True
    shift &= ~first  # the first copy keeps the CAL itself
    delta = rng.integers(1, max_jitter + 1, len(src)) * rng.choice([-1, 1], len(src))
    ref_len = batch.ref_len[batch.cal_ref[src].astype(np.int64)]
    pos = np.where(shift, np.clip(pos + delta, 0, ref_len - 1), pos)
    strand = batch.strand[src].copy()
    if split_strands:
        both = (strand == 3) & ~first
        pick = rng.integers(1, 4, len(src)).astype(np.uint8)
        strand = np.where(both, pick, strand).astype(np.uint8)
    ref = batch.cal_ref[src]
    # shuffle within each read
    r_of = np.repeat(np.arange(batch.n_reads), np.diff(batch.cal_ptr))[src]
    order = np.lexsort((rng.random(len(src)), r_of))
    counts = np.bincount(r_of, minlength=batch.n_reads).astype(np.int64)
    ptr = np.zeros(batch.n_reads + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return dataclasses.replace(batch, cal_ptr=ptr, cal_pos=pos[order].astype(np.int64),
                               cal_ref=ref[order].astype(np.int16), strand=strand[order],
                               name=batch.name + "+dupcals")


def seeding_batch(n_reads: int = 2000, ref_len: int = 2_000_000, read_len=(100, 100), n_refs: int = 1,
                  seed: int = 0, sub_rate: float = 0.01, indel_rate: float = 0.001) -> Batch:
    """Reads for the seeding path (no CALs: the seed index finds them).  Each
    reference is random with 5% planted repeats (the chromosome-scale recipe);
    reads are sampled uniformly over the references with the sequencer error
    model, half from the reverse strand; the true locus is kept."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 55, seed])))
    refs = []
    for k in range(n_refs):
        n = int(ref_len) - 37 * k  # lengths that are not multiples of 16
        g = uniform_genome(rng, n)
        plant_repeats(rng, g, 0.05)
        refs.append(g)
    lens = rng.integers(read_len[0], read_len[1] + 1, n_reads)
    which = rng.integers(0, n_refs, n_reads)
    reads = [None] * n_reads
    true_pos = np.zeros(n_reads, np.int64)
    true_rev = np.zeros(n_reads, bool)
    for k in range(n_refs):
        idx = np.nonzero(which == k)[0]
        if len(idx) == 0:
            continue
        rd, pos, rev = _sample_reads(rng, rng, refs[k], lens[idx], sub_rate, indel_rate)
        for j, r in enumerate(idx):
            reads[r] = rd[j]
        true_pos[idx] = pos
        true_rev[idx] = rev
    sc = Scoring(2, -3, 5, 2, 32)
    return _pack_batch(refs, reads, [[] for _ in range(n_reads)], sc, which.astype(np.int16), true_pos,
                       true_rev, f"seeding{seed}")

"""CPU model of the two-slots-per-lane traceback's number layout, against the oracle.

The traceback kernel that traces two slots per lane keeps every value of window
column j in a 16-bit half as 16 * (V + beta + j * c) + tag, with c = -mismatch
and beta = max(c, gap_open + gap_extend, gap_extend).  The column offset makes
every substitution plus c non-negative (one byte-permutation table per column),
the bias keeps every operand of the packed half-precision three-way maximum in
[0, 0x7BFF], where it orders bit patterns as integers, and the 4 tag bits carry
the cell's choices (bits 3:2: H from zero, the diagonal, F or E, in that order
on equal values; bit 1: F opened from H above; bit 0: E opened from H on the
left).  This model runs that arithmetic on the CPU, one slot at a time: 16-bit
wrapping adds, a three-way maximum that asserts each operand lies in the ordered
domain, the cell codes read from the tag bits alone, the end-cell check and the
walk back.  Every traced slot must give the oracle's start and CIGAR.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1805_00106_amd import workloads as wl

M16 = 0xFFFF


def _fits(sc, max_read_len, wcap):
    c = -sc.mismatch
    goe = sc.gap_open + sc.gap_extend
    beta = max(c, goe, sc.gap_extend)
    if 16 * (sc.match + c) + 8 > 255:
        return None
    if (sc.match * max_read_len + beta + (wcap - 1) * c + 1) * 16 > 0x7BFF:
        return None
    return beta


def _hmax3(a, b, cc):
    for x in (a, b, cc):
        assert 0 <= x <= 0x7BFF, f"three-way maximum operand {x:#x} outside [0, 0x7BFF]"
    return max(a, b, cc)


def _add(a, k):
    return (a + k) & M16


def _trace_slot(q, w, ie, je, sc, beta):
    """The kernel's arithmetic on one slot's rectangle: rows 0..ie of the oriented
    read q, columns 0..je of the window w.  Returns (end value, start_i, start_j,
    CIGAR entries) or None if the end value disagrees with nothing to compare."""
    c0 = -sc.mismatch
    goe, ge = sc.gap_open + sc.gap_extend, sc.gap_extend
    sx, sm = 8, 16 * (sc.match + c0) + 8
    kue, kuf, kee, kfe = 16 * (c0 - goe) + 1, 6 - 16 * goe, 16 * (c0 - ge), -16 * ge
    rows, cols = ie + 1, je + 1
    Hc = np.zeros((rows, cols), np.int64)     # clean H (tag bits cleared)
    Ev = np.zeros((rows, cols), np.int64)     # E entering each cell
    Fv = np.zeros((rows, cols), np.int64)     # F entering each cell
    code = np.zeros((rows, cols), np.int64)
    for j in range(cols):
        zj = 16 * (beta + j * c0) + 12
        for i in range(rows):
            s = sm if q[i] == w[j] else sx
            hd = (16 * (beta - c0) if j == 0 else
                  16 * (beta + (j - 1) * c0) if i == 0 else Hc[i - 1, j - 1])
            diag = _add(hd, s)
            if j == 0:
                e = 16 * beta + 12
            else:
                e = _hmax3(_add(Ev[i, j - 1] & ~1 & M16, kee), _add(Hc[i, j - 1], kue), zj)
            if i == 0:
                f = zj
            else:
                f = _hmax3(_add(Fv[i - 1, j] & ~2 & M16, kfe), _add(Hc[i - 1, j], kuf), zj)
            ht = _hmax3(diag, e, f)
            Ev[i, j], Fv[i, j] = e, f
            Hc[i, j] = ht & ~15 & M16
            code[i, j] = (ht & 12) | (e & 1) | (f & 2)
    endval = (int(Hc[ie, je]) >> 4) - beta - je * c0
    # the walk back from the end cell (the kernel's rules)
    ops = []

    def emit(op):
        if ops and ops[-1][1] == op:
            ops[-1][0] += 1
        else:
            ops.append([1, op])

    tail = len(q) - 1 - ie
    if tail > 0:
        ops.append([tail, 4])
    i, j, state = ie, je, 0
    start_i = start_j = 0
    cd = int(code[i, j])
    while True:
        if state == 0:
            src = cd >> 2
            if src == 2:
                emit(7 if q[i] == w[j] else 8)
                start_i, start_j = i, j
                if i == 0 or j == 0:
                    break
                cd = int(code[i - 1, j - 1])
                if (cd >> 2) == 3:
                    break
                i, j = i - 1, j - 1
            elif src == 1:
                state = 1
            elif src == 0:
                state = 2
            else:
                raise AssertionError("the walk reached a cell with H = 0")
        elif state == 1:
            emit(1)
            assert i > 0
            opened = (cd >> 1) & 1
            i -= 1
            state = 0 if opened else 1
            cd = int(code[i, j])
        else:
            emit(2)
            assert j > 0
            opened = cd & 1
            j -= 1
            state = 0 if opened else 2
            cd = int(code[i, j])
    if start_i > 0:
        if ops and ops[-1][1] == 4:
            ops[-1][0] += start_i
        else:
            ops.append([start_i, 4])
    cigar = [(n << 4) | op for n, op in reversed(ops)]
    return endval, start_i, start_j, cigar


def _check_batch(b, max_read_len):
    sc = b.scoring
    wcap = max_read_len + 2 * sc.band
    beta = _fits(sc, max_read_len, wcap)
    assert beta is not None
    s, r, e, _ = orc.align_batch(b, n_threads=4)
    slots = np.flatnonzero(s > 0)
    rs, qs, nops, cig = orc.traceback(b, s, r, e, slots, cap=64, max_read_len=max_read_len)
    owner = np.repeat(np.arange(b.n_reads), np.diff(b.cal_ptr))
    checked = 0
    for t, slot in enumerate(slots):
        if nops[t] <= 0:
            continue
        cal, h = slot >> 1, slot & 1
        rd = b.read(int(owner[cal]))
        q = rd if h == 0 else (3 - rd)[::-1]
        ref = b.reference(int(b.cal_ref[cal]))
        ws = max(0, int(b.cal_pos[cal]) - sc.band)
        we = min(len(ref), int(b.cal_pos[cal]) + len(rd) + sc.band)
        w = ref[ws:we]
        endval, si, sj, cigar = _trace_slot(q, w, int(e[slot]), int(r[slot]) - ws, sc, beta)
        assert endval == s[slot], (slot, endval, s[slot])
        assert (si, ws + sj) == (int(qs[t]), int(rs[t])), (slot, si, sj, qs[t], rs[t])
        assert cigar == [int(x) for x in cig[t, :nops[t]]], (slot, cigar, cig[t, :nops[t]])
        checked += 1
    return checked


@pytest.mark.parametrize("seed", range(4))
def test_pair_layout_matches_oracle_traceback(seed):
    b = wl.random_small_batch(80 + seed, n_reads=40, read_len=(1, 60), band=10)
    assert _check_batch(b, 60) > 50


@pytest.mark.parametrize("scoring", [(2, -3, 5, 2), (1, -1, 1, 1), (3, -4, 6, 1), (1, -9, 0, 1), (5, -10, 12, 3)])
def test_pair_layout_other_scorings(scoring):
    """Scorings inside the layout's bounds (16 * (match - mismatch) + 8 <= 255),
    homopolymers (ties everywhere) and mixed reads."""
    for seed, homo in ((90, True), (91, False)):
        b = wl.random_small_batch(seed, n_reads=30, read_len=(1, 50), band=8, homopolymer=homo)
        b = dataclasses.replace(b, scoring=wl.Scoring(*scoring, 8))
        assert _check_batch(b, 50) > 20


def test_pair_layout_bounds():
    """The layout's admission rule: the byte table and the 16-bit range."""
    assert _fits(wl.Scoring(2, -3, 5, 2, 32), 100, 164) is not None
    assert _fits(wl.Scoring(2, -3, 5, 2, 64), 250, 378) is not None
    assert _fits(wl.Scoring(2, -20, 5, 2, 32), 100, 164) is None      # 16 * 22 + 8 > 255
    assert _fits(wl.Scoring(2, -3, 5, 2, 200), 1024, 1424) is None    # values past 0x7BFF

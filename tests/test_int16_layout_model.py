"""CPU model of the int16 scoring sweep's number layout, against the oracle.

The int16 kernels hold every value as (V + beta) * 2^K + tag(column) in a
16-bit half and take two three-way maxima per row from the packed
half-precision maximum, which orders int16 bit patterns like integers only on
[0, 0x7BFF] (with the wall patterns [0x8000, 0xFBFF] below them).  This model
runs the same sweep on the CPU, lane by lane (numpy over the 64 lanes of a
tile): 16-bit wrapping adds and subtracts, the signed 16-bit maximum, and a
three-way maximum that asserts every operand lies in that domain before
ranking it.  It uses the layout rules the library states (the widest K of 6, 5,
4 with (beta + top + 1 + 49 * gap_extend) * 2^K <= 0x7BFF, beta = max(|mismatch|,
gap_open + gap_extend + 1, 256 / 2^K + gap_extend), chosen per tile from its
longest read), row r of a strip offset by r * gap_extend * 2^K (so that F moves
down a row with no gap-extend step), strips of R rows handed over column by
column at offset 0, the tile folds (offsets removed) and re-bases, padding rows
and wall columns, and compares every slot with the oracle.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1805_00106_amd import workloads as wl

M16 = 0xFFFF


ROW_OFFSET_ROWS = 49   # a strip holds at most 50 rows: row r of a strip carries r * gap_extend


def _layout(match, mismatch, goe, ge, top):
    for k in (6, 5, 4):
        u = 1 << k
        # the padding rows' substitution (-256) on the row handed over as H - GF
        beta = max(-mismatch, goe + 1, (256 + u - 1) // u + ge)
        if (beta + top + 1 + ROW_OFFSET_ROWS * ge) * u <= 0x7BFF:
            return k, beta
    return None


def _s16(x):
    x = np.asarray(x, np.int64) & M16
    return np.where(x >= 0x8000, x - 0x10000, x)


def _imax(a, b):
    return np.where(_s16(a) >= _s16(b), a, b) & M16


def _rank(v):
    return np.where(v >= 0x8000, 0, v + 1)


def _hmax3(a, b, c):
    ops = [np.asarray(x, np.int64) & M16 for x in (a, b, c)]
    for x in ops:
        ok = (x <= 0x7BFF) | ((x >= 0x8000) & (x <= 0xFBFF))
        assert ok.all(), f"three-way maximum operand outside the ordered domain: {x[~ok][:4]}"
    out = ops[0]
    for x in ops[1:]:
        out = np.where(_rank(x) > _rank(out), x, out)
    return out


def _tile(reads, wins, sc, R):
    """One tile: reads[l] (oriented codes), wins[l] (window codes) per lane.
    Returns (score, col, row) per lane with the kernel's tie rule."""
    n = len(reads)
    L = np.array([len(q) for q in reads])
    W = np.array([len(w) for w in wins])
    Lmax, Wmax = int(L.max()), int(W.max())
    goe, ge = sc.gap_open + sc.gap_extend, sc.gap_extend
    K, beta = _layout(sc.match, sc.mismatch, goe, ge, sc.match * Lmax)
    U, B = 1 << K, beta << K
    GOE_E, GE_E, GO_F, GF = goe * U + 1, ge * U + 1, (goe - ge) * U, ge * U
    # a diagonal move goes one row down: the substitution carries the row step GF
    SM, SX = (sc.match * U - 1 + GF) & M16, (sc.mismatch * U - 1 + GF) & M16
    q = np.full((n, Lmax), -1, np.int64)
    for l, rd in enumerate(reads):
        q[l, :len(rd)] = rd
    w = np.full((n, Wmax), -1, np.int64)
    for l, wd in enumerate(wins):
        w[l, :len(wd)] = wd
    best = np.zeros(n, np.int64)   # key: V << 32 | (0xFFFF - col) << 16 | (0xFFFF - row)
    scr_h = np.zeros((Wmax, n), np.int64)
    scr_f = np.zeros((Wmax, n), np.int64)
    nstrips = (Lmax + R - 1) // R
    for s in range(nstrips):
        r0 = s * R
        # strip row r carries + r * GF (so F needs no gap-extend step); the rows
        # above the strip are handed over as H - GF and F at offset 0
        off = np.arange(R, dtype=np.int64)[:, None] * GF
        Hl = np.full((R, n), U + B, np.int64) + off
        E = np.full((R, n), U + B - 1, np.int64) + off
        M = np.zeros((R, n), np.int64)
        hup_prev = np.full(n, U + B - GF, np.int64)
        for tb in range(0, Wmax, U):
            for c in range(tb, min(tb + U, Wmax)):
                zt = U - 1 - (c - tb) + B
                if s == 0:
                    hup = np.full(n, zt - GF, np.int64)
                    F = np.full(n, (zt - GO_F - GF) & M16, np.int64)
                else:
                    hup, F = scr_h[c].copy(), scr_f[c].copy()

                def sub(r):
                    i = r0 + r
                    if i >= Lmax:
                        return np.full(n, 0xFF00, np.int64)
                    qi = q[:, i]
                    v = np.where(qi == w[:, c], SM, SX)
                    v = np.where(c >= W, 0x8000, v)          # wall column
                    return np.where(qi < 0, 0xFF00, v)       # padding row
                t = (hup_prev + sub(0)) & M16
                hup_prev = hup
                for r in range(R):
                    tn = (Hl[r] + sub(r + 1)) & M16 if r + 1 < R else None
                    H = _hmax3(t, E[r], F)
                    t = tn
                    e2, u = (E[r] - GE_E) & M16, (H - GOE_E) & M16
                    F = _imax(F, (H - GO_F) & M16)
                    E[r] = _hmax3(e2, u, zt - 1 + r * GF)
                    M[r] = _imax(M[r], H)
                    Hl[r] = H
                scr_h[c], scr_f[c] = (Hl[R - 1] - R * GF) & M16, (F - R * GF) & M16
            # fold: best value per lane, its smallest column (largest tag), then smallest row
            M = (M - off) & M16
            mx = M.max(axis=0)
            V = (mx >> K) - beta
            col = tb + (U - 1) - (mx & (U - 1))
            row = r0 + np.argmax(M == mx[None, :], axis=0)
            key = np.where(V > 0, (V << 32) | ((0xFFFF - col) << 16) | (0xFFFF - row), 0)
            best = np.maximum(best, key)
            M[:] = 0
            Hl = (Hl + U) & M16
            E = (E + U) & M16
            hup_prev = (hup_prev + U) & M16
    V = best >> 32
    col = 0xFFFF - ((best >> 16) & 0xFFFF)
    row = 0xFFFF - (best & 0xFFFF)
    return V, np.where(V > 0, col, -1), np.where(V > 0, row, -1)


def _model(batch, R):
    """Both strands of every CAL through the model, tiles of up to 64 CALs."""
    sc = batch.scoring
    n = batch.n_cals
    score = np.full(2 * n, -1, np.int64)
    ref_end = np.full(2 * n, -1, np.int64)
    read_end = np.full(2 * n, -1, np.int64)
    owner = np.repeat(np.arange(batch.n_reads), np.diff(batch.cal_ptr))
    for h in (0, 1):
        tasks = [c for c in range(n) if (batch.strand[c] >> h) & 1]
        for a in range(0, len(tasks), 64):
            chunk = tasks[a:a + 64]
            reads, wins, ws = [], [], []
            for c in chunk:
                rd = batch.read(int(owner[c])).astype(np.int64)
                if h:
                    rd = 3 - rd[::-1]
                k = int(batch.cal_ref[c])
                ref = batch.reference(k)
                p = int(batch.cal_pos[c])
                lo, hi = max(0, p - sc.band), min(len(ref), p + len(rd) + sc.band)
                reads.append(rd)
                wins.append(ref[lo:hi].astype(np.int64))
                ws.append(lo)
            V, col, row = _tile(reads, wins, sc, R)
            for j, c in enumerate(chunk):
                score[2 * c + h] = V[j]
                ref_end[2 * c + h] = ws[j] + col[j] if V[j] > 0 else -1
                read_end[2 * c + h] = row[j]
    return score, ref_end, read_end


CASES = [
    # scoring, read lengths, strip rows: K 6 at the top of its range
    # ((8 + 388 + 1 + 98) * 64 = 31680), K 5 from one base more, K 4 with beta from
    # the mismatch, beta from the gap terms, a large gap extension (row offsets of
    # up to 49 * 29) at the top of K 4, beta from the padding rows at the top of
    # K 6, several strips per read
    ((2, -3, 5, 2), (185, 194), 50),
    ((2, -3, 5, 2), (190, 195), 50),
    ((2, -500, 5, 2), (240, 250), 50),
    ((1, -1, 300, 2), (40, 80), 24),
    ((3, -1, 10, 29), (150, 170), 50),
    ((3, -1, 1, 1), (100, 146), 34),
    ((2, -3, 5, 2), (1, 60), 24),
]


def test_int16_layout_rule():
    """Tag width and bias from the rule, at its edges; no int16 layout for a gap
    extension whose row offsets leave no room."""
    assert _layout(2, -3, 7, 2, 2 * 194) == (6, 8)
    assert _layout(2, -3, 7, 2, 2 * 195) == (5, 10)
    assert _layout(2, -500, 7, 2, 500) == (4, 500)
    assert _layout(1, -1, 302, 2, 80) == (6, 303)
    assert _layout(3, -1, 39, 29, 510) == (4, 45)
    assert _layout(3, -1, 2, 1, 3 * 146) == (6, 5)
    assert _layout(3, -1, 2, 1, 3 * 147) == (5, 9)
    assert _layout(1, -1, 400, 100, 80) is None


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-L{c[1][1]}-R{c[2]}" for c in CASES])
def test_int16_layout_model_matches_oracle(case):
    (m, x, go, ge), lens, R = case
    for seed, homo in ((31, True), (32, False)):
        b = wl.random_small_batch(seed, n_reads=6, read_len=lens, ref_len=(300, 700), band=12,
                                  max_cals=2, homopolymer=homo)
        b = dataclasses.replace(b, scoring=wl.Scoring(m, x, go, ge, 12))
        if homo:
            # full windows on both strands: the largest values the layout must hold
            b = dataclasses.replace(b, cal_pos=np.full_like(b.cal_pos, 12), strand=np.full_like(b.strand, 3))
        s, r, e = _model(b, R)
        es, er, ee, _ = orc.align_batch(b)
        req = np.repeat(b.strand, 2) & np.tile([1, 2], b.n_cals) > 0
        np.testing.assert_array_equal(s[req], es[req])
        np.testing.assert_array_equal(r[req], er[req])
        np.testing.assert_array_equal(e[req], ee[req])
        if homo:
            assert int(es.max()) == m * int(b.read_len[np.diff(b.cal_ptr) > 0].max())

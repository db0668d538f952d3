"""Brute-force local alignment by enumerating every edit transcript.

TEST INFRASTRUCTURE ONLY.  This pins the C oracle with a definition that shares
nothing with Gotoh's recurrences: the local alignment score of a read q against
a window w is the maximum, over every pair of non-empty substrings q[a..b] and
w[c..d] and every edit transcript aligning them end to end, of

    sum of pair scores  (match if the bases agree, mismatch otherwise)
  - sum over maximal runs of k consecutive read-only (or window-only) columns
    of (gap_open + k * gap_extend),

and 0 for the empty alignment (affine gap model, section 3.5 of the paper).  A
run of read-only columns next to a run of window-only columns counts as two
gaps.  The reported end is the last aligned cell (b, d): among optimal
alignments the smallest window end d, then the smallest read end b; both are
-1 when the best score is 0.

Every transcript is listed explicitly, and the scores of all inputs of one shape
are evaluated together with numpy, so it stays usable up to about 6 x 8 bases.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np

_NEG = np.iinfo(np.int64).min // 4


@functools.lru_cache(maxsize=None)
def transcripts(m: int, n: int):
    """Every transcript aligning m read bases with n window bases.

    Returns a list of (pair_index, n_gap_runs, gap_length) where pair_index holds
    the flat indices u*n + v of the aligned (read u, window v) pairs.
    """
    out = []

    def rec(u, v, ops):
        if u == m and v == n:
            pairs, runs, glen = [], 0, 0
            uu = vv = 0
            prev = None
            for op in ops:
                if op == "P":
                    pairs.append(uu * n + vv)
                    uu += 1
                    vv += 1
                else:
                    if op != prev:
                        runs += 1
                    glen += 1
                    if op == "Q":
                        uu += 1
                    else:
                        vv += 1
                prev = op
            out.append((np.array(pairs, dtype=np.int64), runs, glen))
            return
        if u < m and v < n:
            rec(u + 1, v + 1, ops + ("P",))
        if u < m:
            rec(u + 1, v, ops + ("Q",))
        if v < n:
            rec(u, v + 1, ops + ("W",))

    rec(0, 0, ())
    return out


def local_batch(Q: np.ndarray, Wm: np.ndarray, match=2, mismatch=-3, gap_open=5, gap_extend=2, final_row=False):
    """Brute-force local alignment of N pairs of equal shape.

    Q: [N, m] read codes, Wm: [N, n] window codes.  With final_row, only
    alignments whose last read base is the read's last base count (the V1
    array's output: the best cell of the final row).
    Returns (score, ref_end, read_end) int64 arrays of length N.
    """
    Q = np.asarray(Q, dtype=np.int64)
    Wm = np.asarray(Wm, dtype=np.int64)
    N, m = Q.shape
    n = Wm.shape[1]
    S = np.where(Q[:, :, None] == Wm[:, None, :], match, mismatch).astype(np.int64)
    # best global-alignment score of any substring pair ending at each cell (b, d)
    Hend = np.full((N, m, n), _NEG, dtype=np.int64)
    for mm in range(1, m + 1):
        for nn in range(1, n + 1):
            starts = [(a, c) for a in range(m - mm + 1) for c in range(n - nn + 1)]
            B = np.stack([S[:, a:a + mm, c:c + nn].reshape(N, mm * nn) for a, c in starts], axis=1)
            G = np.full((N, len(starts)), _NEG, dtype=np.int64)
            for idx, runs, glen in transcripts(mm, nn):
                val = B[:, :, idx].sum(axis=-1) - (runs * gap_open + glen * gap_extend)
                np.maximum(G, val, out=G)
            for p, (a, c) in enumerate(starts):
                b, d = a + mm - 1, c + nn - 1
                np.maximum(Hend[:, b, d], G[:, p], out=Hend[:, b, d])
    if final_row:
        Hend[:, :m - 1, :] = _NEG
    flat = Hend.reshape(N, m * n)
    best = np.maximum(flat.max(axis=1), 0)
    score = best.copy()
    ref_end = np.full(N, -1, dtype=np.int64)
    read_end = np.full(N, -1, dtype=np.int64)
    pos = best > 0
    if pos.any():
        hit = (Hend == best[:, None, None]) & pos[:, None, None]
        # order cells by (window end d, then read end b)
        order = hit.transpose(0, 2, 1).reshape(N, n * m)
        first = np.argmax(order, axis=1)
        d = first // m
        b = first % m
        ref_end[pos] = d[pos]
        read_end[pos] = b[pos]
    return score, ref_end, read_end


def all_strings(length: int) -> np.ndarray:
    """Every ACGT code string of the given length, as an [4**length, length] array."""
    if length == 0:
        return np.zeros((1, 0), dtype=np.uint8)
    return np.array(list(itertools.product(range(4), repeat=length)), dtype=np.uint8)


def exhaustive(m: int, n: int, **scoring):
    """Brute force over every pair of strings of lengths (m, n)."""
    qs = all_strings(m)
    ws = all_strings(n)
    Q = np.repeat(qs, len(ws), axis=0)
    Wm = np.tile(ws, (len(qs), 1))
    s, r, e = local_batch(Q, Wm, **scoring)
    return Q, Wm, s, r, e


def longest_common_substring(q, w):
    """Length and end cell (smallest window end, then smallest read end) of the longest
    common substring, by direct substring search."""
    q = list(map(int, q))
    w = list(map(int, w))
    best = (0, -1, -1)
    for k in range(min(len(q), len(w)), 0, -1):
        found = None
        for d in range(k - 1, len(w)):
            sub = w[d - k + 1:d + 1]
            for b in range(k - 1, len(q)):
                if q[b - k + 1:b + 1] == sub:
                    found = (k, d, b)
                    break
            if found:
                break
        if found:
            best = found
            break
    return best

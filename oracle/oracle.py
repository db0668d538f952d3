"""ctypes wrapper of the C oracle (sw_oracle.c).  Test infrastructure only.

All sequences are numpy uint8 code arrays (A, C, G, T = 0, 1, 2, 3).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

MAX_READ_LEN = 1024

_lib = None


class _Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32),
                ("band", ctypes.c_int32), ("final_row", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=False)
        _lib = ctypes.CDLL(path)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _sc(match, mismatch, gap_open, gap_extend, band=0, final_row=False):
    return _Scoring(int(match), int(mismatch), int(gap_open), int(gap_extend), int(band), int(bool(final_row)))


def gotoh_pairs(qs, ws, match=2, mismatch=-3, gap_open=5, gap_extend=2, final_row=False):
    """Score a list of (q, w) code arrays.  Returns (score, ref_end, read_end) int64 arrays."""
    n = len(qs)
    ql = np.array([len(q) for q in qs], dtype=np.int64)
    wl = np.array([len(w) for w in ws], dtype=np.int64)
    qo = np.zeros(n, np.int64)
    wo = np.zeros(n, np.int64)
    if n:
        np.cumsum(ql[:-1], out=qo[1:])
        np.cumsum(wl[:-1], out=wo[1:])
    qc = np.ascontiguousarray(np.concatenate(qs) if n else np.zeros(0, np.uint8), dtype=np.uint8)
    wc = np.ascontiguousarray(np.concatenate(ws) if n else np.zeros(0, np.uint8), dtype=np.uint8)
    score = np.zeros(n, np.int64)
    re = np.zeros(n, np.int64)
    qe = np.zeros(n, np.int64)
    sc = _sc(match, mismatch, gap_open, gap_extend, 0, final_row)
    lib().oracle_gotoh_many(_p(qc), _p(qo), _p(ql), _p(wc), _p(wo), _p(wl), ctypes.c_int64(n),
                            ctypes.byref(sc), _p(score), _p(re), _p(qe))
    return score, re, qe


def gotoh(q, w, **kw):
    s, r, e = gotoh_pairs([np.asarray(q, np.uint8)], [np.asarray(w, np.uint8)], **kw)
    return int(s[0]), int(r[0]), int(e[0])


def align_batch(batch, n_threads: int = 1, max_read_len: int = MAX_READ_LEN, final_row: bool = False):
    """Oracle of the batch entry point on a workloads.Batch.  Returns
    (score int32[2n], ref_end int64[2n], read_end int16[2n], n_errors)."""
    sc = batch.scoring
    n = batch.n_cals
    score = np.zeros(2 * n, np.int32)
    ref_end = np.zeros(2 * n, np.int64)
    read_end = np.zeros(2 * n, np.int16)
    arrs = dict(
        read_codes=np.ascontiguousarray(batch.read_codes, np.uint8),
        read_off=np.ascontiguousarray(batch.read_off, np.int64),
        read_len=np.ascontiguousarray(batch.read_len, np.int32),
        ref_codes=np.ascontiguousarray(batch.ref_codes, np.uint8),
        ref_off=np.ascontiguousarray(batch.ref_off, np.int64),
        ref_len=np.ascontiguousarray(batch.ref_len, np.int64),
        cal_ptr=np.ascontiguousarray(batch.cal_ptr, np.int64),
        cal_pos=np.ascontiguousarray(batch.cal_pos, np.int64),
        cal_ref=np.ascontiguousarray(batch.cal_ref, np.int16),
        strand=np.ascontiguousarray(batch.strand, np.uint8),
    )
    s = _sc(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band, final_row)
    f = lib().oracle_align_batch
    f.restype = ctypes.c_int64
    errs = f(_p(arrs["read_codes"]), _p(arrs["read_off"]), _p(arrs["read_len"]),
             ctypes.c_int32(batch.n_reads), _p(arrs["ref_codes"]), _p(arrs["ref_off"]),
             _p(arrs["ref_len"]), ctypes.c_int32(batch.n_refs), _p(arrs["cal_ptr"]),
             _p(arrs["cal_pos"]), _p(arrs["cal_ref"]), _p(arrs["strand"]), ctypes.c_int64(n),
             ctypes.byref(s), ctypes.c_int32(max_read_len), _p(score), _p(ref_end), _p(read_end),
             ctypes.c_int32(n_threads))
    return score, ref_end, read_end, int(errs)


CIGAR_CHARS = {1: "I", 2: "D", 4: "S", 7: "=", 8: "X"}


def cigar_string(ops):
    """Text form of (length << 4) | op entries."""
    return "".join(f"{int(v) >> 4}{CIGAR_CHARS[int(v) & 15]}" for v in ops)


def traceback(batch, score, ref_end, read_end, slots, cap=64, max_read_len: int = MAX_READ_LEN):
    """Start and CIGAR of each slot in `slots` (see oracle_traceback).  Returns
    (ref_start int64[n], read_start int16[n], n_ops int32[n], cigar uint32[n, cap])."""
    sc = batch.scoring
    slots = np.ascontiguousarray(slots, np.int64)
    n = len(slots)
    score = np.ascontiguousarray(score, np.int32)
    ref_end = np.ascontiguousarray(ref_end, np.int64)
    read_end = np.ascontiguousarray(read_end, np.int16)
    rs = np.zeros(n, np.int64)
    qs = np.zeros(n, np.int16)
    nops = np.zeros(n, np.int32)
    cig = np.zeros(max(n, 1) * cap, np.uint32)
    arrs = [np.ascontiguousarray(batch.read_codes, np.uint8), np.ascontiguousarray(batch.read_off, np.int64),
            np.ascontiguousarray(batch.read_len, np.int32), np.ascontiguousarray(batch.ref_codes, np.uint8),
            np.ascontiguousarray(batch.ref_off, np.int64), np.ascontiguousarray(batch.ref_len, np.int64),
            np.ascontiguousarray(batch.cal_ptr, np.int64), np.ascontiguousarray(batch.cal_pos, np.int64),
            np.ascontiguousarray(batch.cal_ref, np.int16)]
    s_ = _sc(sc.match, sc.mismatch, sc.gap_open, sc.gap_extend, sc.band)
    lib().oracle_traceback(_p(arrs[0]), _p(arrs[1]), _p(arrs[2]), ctypes.c_int32(batch.n_reads), _p(arrs[3]),
                           _p(arrs[4]), _p(arrs[5]), ctypes.c_int32(batch.n_refs), _p(arrs[6]), _p(arrs[7]),
                           _p(arrs[8]), ctypes.c_int64(batch.n_cals), ctypes.byref(s_),
                           ctypes.c_int32(max_read_len), _p(score), _p(ref_end), _p(read_end), _p(slots),
                           ctypes.c_int64(n), ctypes.c_int32(cap), _p(rs), _p(qs), _p(nops), _p(cig))
    return rs, qs, nops, cig[:n * cap].reshape(n, cap)


def cal_filter(cal_ptr, cal_pos, cal_ref, strand, n_reads, bucket_bits=0):
    """Duplicate-CAL filter (oracle_cal_filter).  Returns (out_ptr, out_pos, out_ref, out_strand, cal_map)."""
    cal_ptr = np.ascontiguousarray(cal_ptr, np.int64)
    cal_pos = np.ascontiguousarray(cal_pos, np.int64)
    cal_ref = np.ascontiguousarray(cal_ref, np.int16)
    strand = np.ascontiguousarray(strand, np.uint8)
    n = len(cal_pos)
    op = np.zeros(n_reads + 1, np.int64)
    opos = np.zeros(max(n, 1), np.int64)
    oref = np.zeros(max(n, 1), np.int16)
    ost = np.zeros(max(n, 1), np.uint8)
    cmap = np.zeros(max(n, 1), np.int64)
    f = lib().oracle_cal_filter
    f.restype = ctypes.c_int64
    m = f(_p(cal_ptr), _p(cal_pos), _p(cal_ref), _p(strand), ctypes.c_int32(n_reads), ctypes.c_int32(bucket_bits),
          _p(op), _p(opos), _p(oref), _p(ost), _p(cmap))
    return op, opos[:m], oref[:m], ost[:m], cmap[:n]


def find_cals(batch, seed_len=22, stride=1, max_cals_per_seed=0):
    """Seeds of every read looked up in the reference (oracle_find_cals).  Returns
    (cal_ptr, cal_pos, cal_ref, strand) for the reads of `batch`."""
    arrs = [np.ascontiguousarray(batch.ref_codes, np.uint8), np.ascontiguousarray(batch.ref_off, np.int64),
            np.ascontiguousarray(batch.ref_len, np.int64), np.ascontiguousarray(batch.read_codes, np.uint8),
            np.ascontiguousarray(batch.read_off, np.int64), np.ascontiguousarray(batch.read_len, np.int32)]
    ptr = np.zeros(batch.n_reads + 1, np.int64)
    f = lib().oracle_find_cals
    f.restype = ctypes.c_int64
    args = lambda cap, pos, ref, st: (_p(arrs[0]), _p(arrs[1]), _p(arrs[2]), ctypes.c_int32(batch.n_refs),
                                      _p(arrs[3]), _p(arrs[4]), _p(arrs[5]), ctypes.c_int32(batch.n_reads),
                                      ctypes.c_int32(seed_len), ctypes.c_int32(stride),
                                      ctypes.c_int32(max_cals_per_seed), _p(ptr), _p(pos), _p(ref), _p(st),
                                      ctypes.c_int64(cap))
    cap = 4 * max(batch.n_reads, 1)
    while True:
        pos = np.zeros(cap, np.int64)
        ref = np.zeros(cap, np.int16)
        st = np.zeros(cap, np.uint8)
        n = f(*args(cap, pos, ref, st))
        if n <= cap:
            return ptr, pos[:n], ref[:n], st[:n]
        cap = int(n)


def reduce_best(cal_ptr, cal_ref, n_reads, n_refs, score):
    cal_ptr = np.ascontiguousarray(cal_ptr, np.int64)
    cal_ref = np.ascontiguousarray(cal_ref, np.int16)
    score = np.ascontiguousarray(score, np.int32)
    bs = np.zeros(n_reads * n_refs, np.int32)
    bl = np.zeros(n_reads * n_refs, np.int64)
    nt = np.zeros(n_reads * n_refs, np.int32)
    lib().oracle_reduce_best(_p(cal_ptr), _p(cal_ref), ctypes.c_int32(n_reads), ctypes.c_int32(n_refs),
                             _p(score), _p(bs), _p(bl), _p(nt))
    return bs.reshape(n_reads, n_refs), bl.reshape(n_reads, n_refs), nt.reshape(n_reads, n_refs)


def topk(cal_ptr, n_reads, score, k):
    cal_ptr = np.ascontiguousarray(cal_ptr, np.int64)
    score = np.ascontiguousarray(score, np.int32)
    ts = np.zeros(n_reads * k, np.int32)
    tl = np.zeros(n_reads * k, np.int64)
    lib().oracle_topk(_p(cal_ptr), ctypes.c_int32(n_reads), _p(score), ctypes.c_int32(k), _p(ts), _p(tl))
    return ts.reshape(n_reads, k), tl.reshape(n_reads, k)


def tied_flags(cal_ptr, n_reads, score):
    cal_ptr = np.ascontiguousarray(cal_ptr, np.int64)
    score = np.ascontiguousarray(score, np.int32)
    fl = np.zeros(len(score), np.uint8)
    lib().oracle_tied_flags(_p(cal_ptr), ctypes.c_int32(n_reads), _p(score), _p(fl))
    return fl


def classify(best_score, threshold):
    best_score = np.ascontiguousarray(best_score, np.int32)
    n_reads, n_refs = best_score.shape
    cls = np.zeros(n_reads, np.int32)
    lib().oracle_classify(_p(best_score), ctypes.c_int32(n_reads), ctypes.c_int32(n_refs),
                          ctypes.c_int32(threshold), _p(cls))
    return cls


# --------------------------------------------------------------- sequence helpers
_LETTERS = "ACGT"


def encode(s: str) -> np.ndarray:
    """Bases to codes with the paper's order A, C, G, T = 0..3 (Fig. 3)."""
    return np.array([_LETTERS.index(ch) for ch in s], dtype=np.uint8)


def decode(codes) -> str:
    return "".join(_LETTERS[int(c)] for c in codes)


def reverse_complement(codes) -> np.ndarray:
    """Reverse complement (section 3.1): complement is 3 - code under A,C,G,T = 0..3."""
    codes = np.asarray(codes, np.uint8)
    return (3 - codes[::-1]).astype(np.uint8)


def bits_msb_first(codes) -> str:
    """Two bits per base, most significant bit first, as the index figure prints seeds."""
    return "".join(format(int(c), "02b") for c in codes)

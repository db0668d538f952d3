"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad host-visible arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sw_align.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sw_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def sw():
    import paper_1805_00106_amd as sw
    sw.lib()
    return sw


def test_header_declares_entry_points():
    names = _declared_functions()
    for n in ("sw_align_batch", "sw_workspace_bytes", "sw_reduce_best", "sw_classify", "sw_pack_2bit",
              "sw_topk", "sw_tied_flags", "sw_traceback", "sw_traceback_workspace_bytes",
              "sw_ctx_create", "sw_align_batch_ctx", "sw_strerror", "sw_alu_peak", "sw_check_half_max",
              "sw_cal_filter", "sw_index_build", "sw_find_cals", "sw_server_create", "sw_server_submit"):
        assert n in names


def test_library_exports_every_declared_symbol(sw):
    L = sw.lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_covers_codes(sw):
    L = sw.lib()
    for code in range(0, -11, -1):
        assert L.sw_strerror(code).decode() != "unknown error"


def _refset(sw, n_refs=1, length=1000):
    offs = (ctypes.c_int64 * n_refs)(*[0] * n_refs)
    lens = (ctypes.c_int64 * n_refs)(*[length] * n_refs)
    return sw._RefSetC(ctypes.c_void_p(16), ctypes.cast(offs, ctypes.c_void_p), ctypes.cast(lens, ctypes.c_void_p),
                       n_refs), (offs, lens)


def _call(sw, sc, refs=None, n_cals=4, workspace=None, n_reads=2):
    L = sw.lib()
    p = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    if refs is None:
        refs, keep = _refset(sw)
    return L.sw_align_batch(p, p, p, n_reads, ctypes.byref(refs), p, p, p, p, n_cals,
                            ctypes.byref(sc) if sc is not None else None, p, p, p, workspace, 0, None)


@pytest.mark.parametrize("field,value,code", [
    ("match", 0, -2), ("mismatch", 1, -2), ("gap_open", -1, -2), ("gap_extend", 0, -2), ("band", -1, -2),
    ("band", 5000, -2), ("precision", 7, -1), ("kernel", 9, -1), ("max_read_len", 5000, -3),
    ("max_read_len", -3, -1), ("mode", 2, -1), ("mode", -1, -1),
])
def test_scoring_validation(sw, field, value, code):
    sc = sw.Scoring.make(max_read_len=100)
    setattr(sc, field, value)
    assert _call(sw, sc) == code


def test_int32_range_includes_row_offsets(sw):
    """match * max_read_len + 49 * gap_extend <= 2^19 - 2 (the int32 sweep's row offsets)."""
    for (m, ge, mrl), code in (((511, 20, 1024), -5), ((511, 21, 1024), -2), ((1, 10699, 1), -5),
                               ((1, 10700, 1), -2)):
        sc = sw.Scoring.make(m, -1, 0, ge, 8, sw.PREC_INT32, max_read_len=mrl)
        assert _call(sw, sc) == code, (m, ge, mrl)


def test_null_scoring_is_invalid(sw):
    assert _call(sw, None) == -1


def test_int16_bound_rejected_when_requested(sw):
    sc = sw.Scoring.make(precision=sw.PREC_INT16, max_read_len=300)   # 2 * 300 > 510
    assert _call(sw, sc) == -4
    sc = sw.Scoring.make(precision=sw.PREC_INT16, max_read_len=255)
    assert _call(sw, sc) == -5                                         # passes bound, then no workspace
    # the one-CAL-per-lane sweep offsets row r of a strip by r * gap_extend * 2^K:
    # (beta + match * L + 1 + 49 * gap_extend) * 16 must stay below 0x7C00 (K = 4),
    # beta = max(|mismatch|, gap_open + gap_extend + 1, 16 + gap_extend)
    for (m, x, go, ge, mrl), code in (((3, -1, 10, 29, 170), -5),     # (45 + 510 + 1 + 1421) * 16 = 31632
                                      ((3, -1, 10, 30, 170), -4),     # (46 + 510 + 1 + 1470) * 16 = 32432
                                      ((1, -1, 300, 2, 80), -5),
                                      ((1, -1, 300, 100, 80), -4)):   # 49 * 100 of row offsets
        sc = sw.Scoring.make(m, x, go, ge, 8, sw.PREC_INT16, max_read_len=mrl)
        assert _call(sw, sc) == code, (m, x, go, ge, mrl)


def test_reference_set_validation(sw):
    sc = sw.Scoring.make(max_read_len=100)
    refs, keep = _refset(sw, n_refs=65)
    assert _call(sw, sc, refs=refs) == -8
    refs, keep = _refset(sw, n_refs=1, length=0)
    assert _call(sw, sc, refs=refs) == -1


def test_counts_and_workspace_validation(sw):
    sc = sw.Scoring.make(max_read_len=100)
    assert _call(sw, sc, n_cals=-1) == -1
    assert _call(sw, sc, n_reads=-1) == -1
    assert _call(sw, sc, n_cals=10) == -5        # no workspace
    assert _call(sw, sc, n_cals=0) == 0          # nothing to do


def test_reduce_and_classify_validation(sw):
    L = sw.lib()
    p = ctypes.c_void_p(16)
    assert L.sw_reduce_best(p, p, -1, 1, 1, p, p, p, p, None) == -1
    assert L.sw_reduce_best(p, p, 1, 0, 1, p, p, p, p, None) == -1
    assert L.sw_reduce_best(p, p, 1, 65, 1, p, p, p, p, None) == -8
    assert L.sw_reduce_best(p, p, 1, 1, -1, p, p, p, p, None) == -1
    assert L.sw_reduce_best(p, None, 1, 1, 1, p, p, p, p, None) == -1
    assert L.sw_classify(p, 1, 0, 0, p, None) == -1
    assert L.sw_pack_2bit(p, -1, p, None) == -1


def test_topk_and_tied_validation(sw):
    L = sw.lib()
    p = ctypes.c_void_p(16)
    assert L.sw_topk(p, -1, 1, p, 1, p, p, None) == -1
    assert L.sw_topk(p, 1, 1, p, 0, p, p, None) == -1
    assert L.sw_topk(p, 1, 1, p, sw.MAX_TOPK + 1, p, p, None) == -1
    assert L.sw_topk(None, 1, 1, p, 1, p, p, None) == -1
    assert L.sw_topk(p, 1, -1, p, 1, p, p, None) == -1
    assert L.sw_topk(p, 0, 1, p, 1, p, p, None) == 0
    assert L.sw_tied_flags(p, -1, 1, p, p, None) == -1
    assert L.sw_tied_flags(p, 1, 1, None, p, None) == -1
    assert L.sw_tied_flags(p, 1, -1, p, p, None) == -1
    assert L.sw_tied_flags(p, 0, 1, p, p, None) == 0


def test_cigar_text(sw):
    ops = [(3 << 4) | 4, (10 << 4) | 7, (1 << 4) | 8, (5 << 4) | 7, (2 << 4) | 2, (4 << 4) | 7]
    assert sw.cigar_text(ops, len(ops)) == "3S10=1X5=2D4="
    assert sw.cigar_text(ops, len(ops), extended=False) == "3S16M2D4M"


def test_traceback_validation(sw):
    L = sw.lib()
    p = ctypes.c_void_p(16)
    sc = sw.Scoring.make(max_read_len=100)
    refs, keep = _refset(sw)
    args = lambda n_slots, cap, scp: (p, p, p, 1, ctypes.byref(refs), p, p, p, 1, scp, p, p, p, p, n_slots, cap,
                                      p, p, p, p, None, 0, None)
    assert L.sw_traceback(*args(1, 0, ctypes.byref(sc))) == -1
    assert L.sw_traceback(*args(-1, 4, ctypes.byref(sc))) == -1
    assert L.sw_traceback(*args(1, 4, None)) == -1
    assert L.sw_traceback(*args(0, 4, ctypes.byref(sc))) == 0
    bad = sw.Scoring.make(max_read_len=100, match=0)
    assert L.sw_traceback(*args(1, 4, ctypes.byref(bad))) == -2


def test_cal_filter_validation(sw):
    L = sw.lib()
    p = ctypes.c_void_p(16)
    call = lambda n_reads, n_cals, bits, ws, nb: L.sw_cal_filter(p, p, p, p, n_reads, n_cals, bits, p, p, p, p, p,
                                                                 ws, nb, None)
    assert call(-1, 1, 0, p, 1 << 30) == -1
    assert call(1, -1, 0, p, 1 << 30) == -1
    assert call(1, 1, -1, p, 1 << 30) == -1
    assert call(1, 1, 41, p, 1 << 30) == -1
    assert call(1, 1, 0, None, 0) == -5
    assert call(10, 1, 0, p, 8) == -5
    assert L.sw_cal_filter_workspace_bytes(1000) >= 8 * 1001


def test_alu_peak_validation(sw):
    L = sw.lib()
    v = ctypes.c_double()
    assert L.sw_alu_peak(8, 1 << 10, ctypes.byref(v), None) == -1
    assert L.sw_alu_peak(16, 4, ctypes.byref(v), None) == -1
    assert L.sw_alu_peak(32, 1 << 10, None, None) == -1
    assert L.sw_check_half_max(None, None) == -1


def test_ctx_capacity_validation(sw):
    """Task positions are int32 in the batched planner (two tasks per CAL in int32
    precision): a capacity whose task count leaves int32 is rejected before any
    HIP call."""
    L = sw.lib()
    h = ctypes.c_void_p()
    for max_cals in (-1, (2**31 - 1) // 2 + 1, 1 << 40):
        o = sw._CtxOpts(0, 16, max_cals, 1, 0, None)
        assert L.sw_ctx_create(ctypes.byref(o), ctypes.byref(h)) == -1
    o = sw._CtxOpts(-1, 16, 16, 1, 0, None)
    assert L.sw_ctx_create(ctypes.byref(o), ctypes.byref(h)) == -1


def test_binding_rejects_malformed_tensors(sw):
    """The binding checks dtype, device, contiguity and element counts of every
    tensor before any library call (on this host, CPU tensors fail the device
    check first)."""
    import torch
    t = torch.zeros(4, dtype=torch.int64)
    with pytest.raises(ValueError):
        sw._dev(t, torch.int64, what="cal_pos")
    db = sw.DeviceBatch(torch.zeros(4, dtype=torch.int32), torch.zeros(2, dtype=torch.int64),
                        torch.zeros(2, dtype=torch.int32), torch.zeros(3, dtype=torch.int64),
                        torch.zeros(3, dtype=torch.int32), torch.zeros(3, dtype=torch.int16),
                        torch.zeros(3, dtype=torch.uint8))
    with pytest.raises(ValueError):
        sw._check_batch(db)


@pytest.mark.parametrize("field,value", [("max_steps_in_flight", -1), ("max_steps_in_flight", 4),
                                         ("max_step_chunks", 0), ("max_step_chunks", 4097),
                                         ("max_step_reads", 0), ("memory_budget", 1 << 19)])
def test_server_create_rejects_bad_options(sw, field, value):
    """The server's options are checked before any device call."""
    sc = sw.Scoring.make(2, -3, 5, 2, 8, sw.PREC_AUTO, max_read_len=128)
    opts = sw._ServerOpts(0, sc, 1 << 24, 1024, 1 << 16, 64, 0, 0)
    setattr(opts, field, value)
    h = ctypes.c_void_p()
    assert sw.lib().sw_server_create(ctypes.byref(opts), ctypes.byref(h)) == -1  # SW_ERR_INVALID_ARG
    assert not h.value

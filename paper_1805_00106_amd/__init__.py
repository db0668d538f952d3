"""MI355X (gfx950) affine-gap Smith-Waterman CAL scorer: Python binding.

The binding only marshals arguments: every step of the scoring path runs in the
HIP kernels of ``libswalign.so`` (C ABI, include/sw_align.h).  PyTorch provides
device memory and streams.  Importing this module fails loudly when the built
library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch  # load torch's HIP runtime before the library so both share it

__all__ = [
    "lib", "Scoring", "RefSet", "DeviceBatch", "pack_2bit", "workspace_bytes", "align_batch", "align_batch_noalloc",
    "reduce_best", "topk", "tied_flags", "classify", "error_count", "traceback", "cigar_text", "cal_filter", "SeedIndex", "alu_peak", "check_half_max", "SwError", "Context", "Outputs", "Server", "Request",
    "PREC_AUTO", "PREC_INT16", "PREC_INT32", "KERNEL_AUTO", "KERNEL_INTER", "KERNEL_INTRA",
    "MODE_LOCAL", "MODE_FINAL_ROW", "MAX_READ_LEN", "MAX_REFS", "MAX_TOPK",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswalign.so")

PREC_AUTO, PREC_INT16, PREC_INT32 = 0, 1, 2
KERNEL_AUTO, KERNEL_INTER, KERNEL_INTRA = 0, 1, 2
MODE_LOCAL, MODE_FINAL_ROW = 0, 1
MAX_READ_LEN = 1024
MAX_TOPK = 64
MAX_REFS = 64

_lib = None


class SwError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().sw_strerror(code).decode()
        if code == -7:
            msg += f" (hipError {lib().sw_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")


class Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32), ("band", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("max_read_len", ctypes.c_int32), ("mode", ctypes.c_int32)]

    @classmethod
    def make(cls, match=2, mismatch=-3, gap_open=5, gap_extend=2, band=32, precision=PREC_AUTO,
             kernel=KERNEL_AUTO, max_read_len=0, mode=MODE_LOCAL):
        return cls(match, mismatch, gap_open, gap_extend, band, precision, kernel, max_read_len, mode)


class _RefSetC(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("word_offset", ctypes.c_void_p), ("length", ctypes.c_void_p),
                ("n_refs", ctypes.c_int32)]


class _IndexOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("seed_len", ctypes.c_int32), ("addr_bits", ctypes.c_int32)]


class _FindOpts(ctypes.Structure):
    _fields_ = [("stride", ctypes.c_int32), ("max_cals_per_seed", ctypes.c_int32), ("max_read_len", ctypes.c_int32)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("scoring", Scoring), ("memory_budget", ctypes.c_size_t),
                ("max_step_reads", ctypes.c_int32), ("max_step_cals", ctypes.c_int64),
                ("max_step_chunks", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("max_steps_in_flight", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("step_reads", ctypes.c_int64), ("step_cals", ctypes.c_int64),
                ("pending", ctypes.c_int64), ("in_flight_requests", ctypes.c_int64),
                ("arena_used", ctypes.c_int64), ("arena_size", ctypes.c_int64),
                ("steps_launched_early", ctypes.c_int64)]


class _CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_reads", ctypes.c_int32), ("max_cals", ctypes.c_int64),
                ("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.sw_strerror.restype = ctypes.c_char_p
        L.sw_strerror.argtypes = [ctypes.c_int]
        L.sw_version.restype = ctypes.c_char_p
        L.sw_last_hip_error.restype = ctypes.c_int
        L.sw_pack_2bit.argtypes = [vp, i64, vp, vp]
        L.sw_workspace_bytes.restype = sz
        L.sw_workspace_bytes.argtypes = [i32, i64, ctypes.POINTER(Scoring)]
        L.sw_align_batch.argtypes = [vp, vp, vp, i32, ctypes.POINTER(_RefSetC), vp, vp, vp, vp, i64,
                                     ctypes.POINTER(Scoring), vp, vp, vp, vp, sz, vp]
        L.sw_align_batch_noalloc.argtypes = [vp, vp, vp, i32, ctypes.POINTER(_RefSetC), vp, vp, vp, vp, i64,
                                             ctypes.POINTER(Scoring), vp, vp, vp, vp]
        L.sw_error_count.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.sw_reduce_best.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, vp, vp]
        L.sw_classify.argtypes = [vp, i32, i32, i32, vp, vp]
        L.sw_topk.argtypes = [vp, i32, i64, vp, i32, vp, vp, vp]
        L.sw_alu_peak.argtypes = [i32, i64, ctypes.POINTER(ctypes.c_double), vp]
        L.sw_check_half_max.argtypes = [ctypes.POINTER(ctypes.c_int64), vp]
        L.sw_traceback.argtypes = [vp, vp, vp, i32, ctypes.POINTER(_RefSetC), vp, vp, vp, i64,
                                   ctypes.POINTER(Scoring), vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, vp,
                                   ctypes.c_size_t, vp]
        L.sw_index_build.argtypes = [ctypes.POINTER(_RefSetC), ctypes.POINTER(_IndexOpts), ctypes.POINTER(vp), vp]
        L.sw_index_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.sw_index_destroy.argtypes = [vp]
        L.sw_find_cals.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(_FindOpts), vp, vp, vp, vp, i64,
                                   ctypes.POINTER(i64), vp]
        L.sw_cal_filter.argtypes = [vp, vp, vp, vp, i32, i64, i32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.sw_cal_filter_workspace_bytes.argtypes = [i32]
        L.sw_cal_filter_workspace_bytes.restype = ctypes.c_size_t
        L.sw_traceback_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Scoring)]
        L.sw_traceback_workspace_bytes.restype = ctypes.c_size_t
        L.sw_tied_flags.argtypes = [vp, i32, i64, vp, vp, vp]
        L.sw_ctx_create.argtypes = [ctypes.POINTER(_CtxOpts), ctypes.POINTER(vp)]
        L.sw_ctx_destroy.argtypes = [vp]
        L.sw_align_batch_ctx.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(_RefSetC), vp, vp, vp, vp, i64,
                                         ctypes.POINTER(Scoring), vp, vp, vp, vp]
        L.sw_ctx_error_count.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.sw_ctx_last_plan.restype = ctypes.c_char_p
        L.sw_ctx_last_plan.argtypes = [vp]
        L.sw_server_create.argtypes = [ctypes.POINTER(_ServerOpts), ctypes.POINTER(vp)]
        L.sw_server_set_refs.argtypes = [vp, ctypes.POINTER(_RefSetC)]
        L.sw_server_submit.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp,
                                       ctypes.POINTER(i64)]
        L.sw_server_wait.argtypes = [vp, i64, i32, ctypes.POINTER(i32)]
        L.sw_server_request_info.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.sw_server_release.argtypes = [vp, i64]
        L.sw_server_stats.argtypes = [vp, ctypes.POINTER(_ServerStats)]
        L.sw_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != 0:
        raise SwError(rc, where)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if t.numel() == 0:  # torch reports no address for an empty tensor: use its storage's
        p = t.untyped_storage().data_ptr()
        return ctypes.c_void_p(p) if p else None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype, numel: Optional[int] = None, what: str = "tensor") -> torch.Tensor:
    """A device tensor the C ABI may read or write through its address: on the
    GPU, of the stated dtype, contiguous and (when given) of exactly `numel`
    elements.  Raises ValueError otherwise, before any library call."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch.Tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{what}: must be on the GPU, is on {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{what}: dtype must be {dtype}, is {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: must hold {numel} elements, holds {t.numel()}")
    return t


def _check_batch(db: "DeviceBatch"):
    """Every array of a batch, against the counts the C ABI is given."""
    n, m = db.n_reads, db.n_cals
    _dev(db.reads2bit, torch.int32, what="reads2bit")
    _dev(db.read_word_off, torch.int64, n, "read_word_off")
    _dev(db.read_len, torch.int32, n, "read_len")
    _dev(db.cal_ptr, torch.int64, n + 1, "cal_ptr")
    _dev(db.cal_pos, torch.int64, m, "cal_pos")
    _dev(db.cal_ref, torch.int16, m, "cal_ref")
    _dev(db.strand, torch.uint8, m, "strand")


def _check_outputs(out: "Outputs", n_cals: int):
    _dev(out.score, torch.int32, 2 * n_cals, "score")
    _dev(out.ref_end, torch.int64, 2 * n_cals, "ref_end")
    _dev(out.read_end, torch.int16, 2 * n_cals, "read_end")


def pack_2bit(codes: torch.Tensor, stream=None) -> torch.Tensor:
    """Pack a device uint8 code tensor (A,C,G,T = 0..3) into uint32 words."""
    _dev(codes, torch.uint8)
    n = codes.numel()
    words = torch.empty((n + 15) // 16, dtype=torch.int32, device=codes.device)
    _check(lib().sw_pack_2bit(_ptr(codes), n, _ptr(words), _stream(stream)), "sw_pack_2bit")
    return words


class RefSet:
    """References resident in device memory (2-bit packed)."""

    def __init__(self, words: torch.Tensor, word_offset, length):
        _dev(words, torch.int32, what="reference words")
        if len(word_offset) != len(length) or not 1 <= len(length) <= MAX_REFS:
            raise ValueError("word_offset and length must name the same 1..MAX_REFS references")
        for o, n in zip(word_offset, length):
            if int(o) < 0 or int(n) < 1 or int(o) + (int(n) + 15) // 16 > words.numel():
                raise ValueError(f"reference at word {int(o)} of {int(n)} bases lies outside the "
                                 f"{words.numel()} packed words")
        self.words = words
        self.word_offset = (ctypes.c_int64 * len(word_offset))(*[int(x) for x in word_offset])
        self.length = (ctypes.c_int64 * len(length))(*[int(x) for x in length])
        self.n_refs = len(length)
        self._c = _RefSetC(words.data_ptr(), ctypes.cast(self.word_offset, ctypes.c_void_p),
                           ctypes.cast(self.length, ctypes.c_void_p), self.n_refs)

    @classmethod
    def from_codes(cls, codes: torch.Tensor, code_offset, length, stream=None):
        """Pack concatenated reference codes (each reference at a 16-aligned offset) on the device."""
        words = pack_2bit(codes, stream)
        return cls(words, [int(o) // 16 for o in code_offset], list(length))

    @property
    def c(self):
        return ctypes.byref(self._c)


class DeviceBatch:
    """Device tensors of one batch in the library's layout."""

    def __init__(self, reads2bit, read_word_off, read_len, cal_ptr, cal_pos, cal_ref, strand):
        self.reads2bit = reads2bit
        self.read_word_off = read_word_off
        self.read_len = read_len
        self.cal_ptr = cal_ptr
        self.cal_pos = cal_pos
        self.cal_ref = cal_ref
        self.strand = strand

    @property
    def n_reads(self):
        return int(self.read_len.numel())

    @property
    def n_cals(self):
        return int(self.cal_pos.numel())

    @classmethod
    def upload(cls, batch, device="cuda", stream=None):
        """From a workloads.Batch (host codes, each read at a 16-aligned offset)."""
        t = lambda a, dt: _nonnull(torch.from_numpy(a).to(device=device, dtype=dt).contiguous())
        codes = t(batch.read_codes, torch.uint8)
        words = pack_2bit(codes, stream)
        return cls(words, t(batch.read_off // 16, torch.int64), t(batch.read_len, torch.int32),
                   t(batch.cal_ptr, torch.int64), t(batch.cal_pos, torch.int64), t(batch.cal_ref, torch.int16),
                   t(batch.strand, torch.uint8))


def workspace_bytes(n_reads: int, n_cals: int, sc: Scoring) -> int:
    return int(lib().sw_workspace_bytes(n_reads, n_cals, ctypes.byref(sc)))


def _nonnull(t: torch.Tensor) -> torch.Tensor:
    """An empty tensor still gets a storage address: the C ABI rejects null
    pointers, and nothing is read through the address of an empty array."""
    if t.numel() > 0:
        return t
    return torch.empty(1, dtype=t.dtype, device=t.device)[:0]


class Outputs:
    def __init__(self, n_cals, device="cuda"):
        self.score = _nonnull(torch.empty(2 * n_cals, dtype=torch.int32, device=device))
        self.ref_end = _nonnull(torch.empty(2 * n_cals, dtype=torch.int64, device=device))
        self.read_end = _nonnull(torch.empty(2 * n_cals, dtype=torch.int16, device=device))


def align_batch(db: DeviceBatch, refs: RefSet, sc: Scoring, out: Optional[Outputs] = None,
                workspace: Optional[torch.Tensor] = None, stream=None) -> Outputs:
    """sw_align_batch on device tensors; returns (score, ref_end, read_end) tensors."""
    _check_batch(db)
    n = db.n_cals
    if out is None:
        out = Outputs(n, db.cal_pos.device)
    _check_outputs(out, n)
    need = workspace_bytes(db.n_reads, n, sc)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=db.cal_pos.device)
    _dev(workspace, torch.uint8, what="workspace")
    rc = lib().sw_align_batch(_ptr(db.reads2bit), _ptr(db.read_word_off), _ptr(db.read_len), db.n_reads,
                              refs.c, _ptr(db.cal_ptr), _ptr(db.cal_pos), _ptr(db.cal_ref), _ptr(db.strand), n,
                              ctypes.byref(sc), _ptr(out.score), _ptr(out.ref_end), _ptr(out.read_end),
                              _ptr(workspace), workspace.numel(), _stream(stream))
    _check(rc, "sw_align_batch")
    return out


NOALLOC_SCRATCH_BYTES = 128 << 20


def align_batch_noalloc(db: DeviceBatch, refs: RefSet, sc: Scoring, out: Outputs, stream=None) -> Outputs:
    """sw_align_batch_noalloc: the plain scoring call with its scratch in the
    library's static device array (no allocation in the library; the caller
    brings the outputs).  Calls that overlap on one device race."""
    _check_batch(db)
    _check_outputs(out, db.n_cals)
    rc = lib().sw_align_batch_noalloc(_ptr(db.reads2bit), _ptr(db.read_word_off), _ptr(db.read_len), db.n_reads,
                                      refs.c, _ptr(db.cal_ptr), _ptr(db.cal_pos), _ptr(db.cal_ref), _ptr(db.strand),
                                      db.n_cals, ctypes.byref(sc), _ptr(out.score), _ptr(out.ref_end),
                                      _ptr(out.read_end), _stream(stream))
    _check(rc, "sw_align_batch_noalloc")
    return out


def reduce_best(db: DeviceBatch, n_refs: int, score: torch.Tensor, stream=None):
    _check_batch(db)
    _dev(score, torch.int32, 2 * db.n_cals, "score")
    n = db.n_reads
    dev = score.device
    bs = torch.empty(n * n_refs, dtype=torch.int32, device=dev)
    bl = torch.empty(n * n_refs, dtype=torch.int64, device=dev)
    nt = torch.empty(n * n_refs, dtype=torch.int32, device=dev)
    _check(lib().sw_reduce_best(_ptr(db.cal_ptr), _ptr(db.cal_ref), n, n_refs, db.n_cals, _ptr(score), _ptr(bs), _ptr(bl),
                                _ptr(nt), _stream(stream)), "sw_reduce_best")
    return bs.view(n, n_refs), bl.view(n, n_refs), nt.view(n, n_refs)


def alu_peak(bits: int = 16, iters: int = 1 << 19, stream=None) -> float:
    """Measured sustained integer lane-ops per second of the current device (sw_alu_peak)."""
    v = ctypes.c_double(0.0)
    _check(lib().sw_alu_peak(bits, iters, ctypes.byref(v), _stream(stream)), "sw_alu_peak")
    return v.value


def check_half_max(stream=None) -> int:
    """Halves where the packed half-precision maximum breaks the order the int16
    kernels rely on, over every pair of operands (sw_check_half_max); 0 expected."""
    v = ctypes.c_int64(-1)
    _check(lib().sw_check_half_max(ctypes.byref(v), _stream(stream)), "sw_check_half_max")
    return v.value


def topk(db: DeviceBatch, score: torch.Tensor, k: int, stream=None):
    """The k best slots of each read (score, slot), highest score first; -1 past the valid slots."""
    _check_batch(db)
    _dev(score, torch.int32, 2 * db.n_cals, "score")
    n = db.n_reads
    ts = torch.empty(n * k, dtype=torch.int32, device=score.device)
    tl = torch.empty(n * k, dtype=torch.int64, device=score.device)
    _check(lib().sw_topk(_ptr(db.cal_ptr), n, db.n_cals, _ptr(score), k, _ptr(ts), _ptr(tl), _stream(stream)),
           "sw_topk")
    return ts.view(n, k), tl.view(n, k)


def tied_flags(db: DeviceBatch, score: torch.Tensor, stream=None) -> torch.Tensor:
    """1 for every slot whose score equals its read's best score, else 0."""
    _check_batch(db)
    _dev(score, torch.int32, 2 * db.n_cals, "score")
    fl = torch.empty(score.numel(), dtype=torch.uint8, device=score.device)
    _check(lib().sw_tied_flags(_ptr(db.cal_ptr), db.n_reads, db.n_cals, _ptr(score), _ptr(fl), _stream(stream)),
           "sw_tied_flags")
    return fl


def traceback(db: DeviceBatch, refs: "RefSet", sc: Scoring, out: "Outputs", slots: torch.Tensor, cap: int = 64,
              stream=None):
    """Start position and CIGAR of each slot in `slots` (int64 device tensor, -1 to skip), from
    the outputs `out` of a scoring call on the same batch.  Returns (ref_start, read_start,
    n_ops, cigar[n, cap]); entries are (length << 4) | op with BAM op codes."""
    _check_batch(db)
    _check_outputs(out, db.n_cals)
    slots = slots.to(device=out.score.device, dtype=torch.int64).contiguous()
    n = slots.numel()
    dev = out.score.device
    rs = torch.empty(n, dtype=torch.int64, device=dev)
    qs = torch.empty(n, dtype=torch.int16, device=dev)
    nops = torch.empty(n, dtype=torch.int32, device=dev)
    cig = torch.zeros(max(n, 1) * cap, dtype=torch.int32, device=dev)
    nb = lib().sw_traceback_workspace_bytes(n, db.n_cals, ctypes.byref(sc))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    _check(lib().sw_traceback(_ptr(db.reads2bit), _ptr(db.read_word_off), _ptr(db.read_len), db.n_reads, refs.c,
                              _ptr(db.cal_ptr), _ptr(db.cal_pos), _ptr(db.cal_ref), db.n_cals, ctypes.byref(sc),
                              _ptr(out.score), _ptr(out.ref_end), _ptr(out.read_end), _ptr(slots), n, cap,
                              _ptr(rs), _ptr(qs), _ptr(nops), _ptr(cig), _ptr(ws), nb, _stream(stream)),
           "sw_traceback")
    return rs, qs, nops, cig[:n * cap].view(n, cap)


def cal_filter(db: DeviceBatch, bucket_bits: int = 0, stream=None, workspace: Optional[torch.Tensor] = None):
    """CAL Filter on device: a DeviceBatch with each read's duplicate CALs folded
    into one (same reads), and cal_map (input CAL -> kept CAL).  Synchronises the
    stream once to read the number of kept CALs."""
    _check_batch(db)
    dev = db.cal_pos.device
    n = db.n_cals
    out_ptr = torch.empty(db.n_reads + 1, dtype=torch.int64, device=dev)
    out_pos = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    out_ref = torch.empty(max(n, 1), dtype=torch.int16, device=dev)
    out_strand = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    cal_map = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    nb = lib().sw_cal_filter_workspace_bytes(db.n_reads)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    _check(lib().sw_cal_filter(_ptr(db.cal_ptr), _ptr(db.cal_pos), _ptr(db.cal_ref), _ptr(db.strand), db.n_reads,
                               n, bucket_bits, _ptr(out_ptr), _ptr(out_pos), _ptr(out_ref), _ptr(out_strand),
                               _ptr(cal_map), _ptr(workspace), nb, _stream(stream)), "sw_cal_filter")
    if stream is not None:
        stream.synchronize()
    m = int(out_ptr[-1].item())
    kept = DeviceBatch(db.reads2bit, db.read_word_off, db.read_len, out_ptr, out_pos[:m], out_ref[:m],
                       out_strand[:m])
    return kept, cal_map[:n]


class SeedIndex:
    """Seed index of a resident reference set (sw_index_*): pointer table + CAL
    table in device memory; find() turns reads into the CSR CAL lists that
    cal_filter and align_batch take."""

    def __init__(self, refs: "RefSet", seed_len: int = 22, addr_bits: int = 0, device: int = 0, stream=None):
        self._h = ctypes.c_void_p()
        self.seed_len = seed_len
        self._cap_hint = 0  # CALs found by the last call: the next call's first guess
        o = _IndexOpts(device, seed_len, addr_bits)
        _check(lib().sw_index_build(refs.c, ctypes.byref(o), ctypes.byref(self._h), _stream(stream)),
               "sw_index_build")

    def info(self):
        n, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sw_index_info(self._h, ctypes.byref(n), ctypes.byref(b)), "sw_index_info")
        return {"entries": n.value, "device_bytes": b.value}

    def find(self, db: DeviceBatch, stride: int = 1, max_cals_per_seed: int = 0, max_read_len: int = 0,
             capacity: Optional[int] = None, stream=None) -> DeviceBatch:
        """CALs of the reads of `db` (its own CAL arrays are ignored)."""
        n = db.n_reads
        _dev(db.reads2bit, torch.int32, what="reads2bit")
        _dev(db.read_word_off, torch.int64, n, "read_word_off")
        _dev(db.read_len, torch.int32, n, "read_len")
        dev = db.read_len.device
        o = _FindOpts(stride, max_cals_per_seed, max_read_len)
        ptr = torch.empty(db.n_reads + 1, dtype=torch.int64, device=dev)
        cap = capacity if capacity is not None else max(16 * max(db.n_reads, 1), self._cap_hint)
        for _ in range(2):
            pos = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
            ref = torch.empty(max(cap, 1), dtype=torch.int16, device=dev)
            st = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
            n = ctypes.c_int64()
            rc = lib().sw_find_cals(self._h, _ptr(db.reads2bit), _ptr(db.read_word_off), _ptr(db.read_len),
                                    db.n_reads, ctypes.byref(o), _ptr(ptr), _ptr(pos), _ptr(ref), _ptr(st), cap,
                                    ctypes.byref(n), _stream(stream))
            if rc == -5 and n.value > cap:
                cap = n.value
                continue
            _check(rc, "sw_find_cals")
            m = n.value
            self._cap_hint = max(self._cap_hint, m + m // 8)
            return DeviceBatch(db.reads2bit, db.read_word_off, db.read_len, ptr, pos[:m], ref[:m], st[:m])
        raise SwError(-5, "sw_find_cals")

    def close(self):
        if self._h:
            lib().sw_index_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_OP_TEXT = {1: "I", 2: "D", 4: "S", 7: "=", 8: "X"}


def cigar_text(entries, n_ops: int, extended: bool = True) -> str:
    """SAM text of one CIGAR row; extended=False folds '=' and 'X' into 'M'."""
    out = []
    for v in list(entries)[:max(n_ops, 0)]:
        v = int(v) & 0xFFFFFFFF
        op = _OP_TEXT[v & 15]
        if not extended and op in "=X":
            op = "M"
        if out and out[-1][1] == op:
            out[-1][0] += v >> 4
        else:
            out.append([v >> 4, op])
    return "".join(f"{n}{op}" for n, op in out)


def classify(best_score: torch.Tensor, threshold: int, stream=None) -> torch.Tensor:
    if best_score.dim() != 2:
        raise ValueError("best_score must be [n_reads, n_refs]")
    best_score = _dev(best_score.contiguous(), torch.int32, what="best_score")
    n, k = best_score.shape
    cls = torch.empty(n, dtype=torch.int32, device=best_score.device)
    _check(lib().sw_classify(_ptr(best_score.contiguous()), n, k, threshold, _ptr(cls), _stream(stream)),
           "sw_classify")
    return cls


class Context:
    """Batched execution context (sw_ctx_*): length-binned persistent work queue,
    HIP graphs per call shape and an autotuned binning plan.  Same outputs as
    align_batch, bit for bit."""

    def __init__(self, max_reads: int, max_cals: int, device: int = 0, use_graph: bool = True,
                 autotune: bool = True, tune_cache: Optional[str] = None):
        self._h = ctypes.c_void_p()
        self._cache = tune_cache.encode() if tune_cache else None
        opts = _CtxOpts(device, max_reads, max_cals, int(use_graph), int(autotune), self._cache)
        _check(lib().sw_ctx_create(ctypes.byref(opts), ctypes.byref(self._h)), "sw_ctx_create")

    def close(self):
        if self._h:
            lib().sw_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def align(self, db: DeviceBatch, refs: RefSet, sc: Scoring, out: Optional[Outputs] = None, stream=None):
        _check_batch(db)
        if out is None:
            out = Outputs(db.n_cals, db.cal_pos.device)
        _check_outputs(out, db.n_cals)
        rc = lib().sw_align_batch_ctx(self._h, _ptr(db.reads2bit), _ptr(db.read_word_off), _ptr(db.read_len),
                                      db.n_reads, refs.c, _ptr(db.cal_ptr), _ptr(db.cal_pos), _ptr(db.cal_ref),
                                      _ptr(db.strand), db.n_cals, ctypes.byref(sc), _ptr(out.score),
                                      _ptr(out.ref_end), _ptr(out.read_end), _stream(stream))
        _check(rc, "sw_align_batch_ctx")
        return out

    def error_count(self) -> int:
        v = ctypes.c_int64(0)
        _check(lib().sw_ctx_error_count(self._h, ctypes.byref(v)), "sw_ctx_error_count")
        return int(v.value)

    def last_plan(self) -> str:
        return lib().sw_ctx_last_plan(self._h).decode()


class Request:
    """Host outputs of one served request (filled when it completes)."""

    def __init__(self, rid, n_reads, n_cals, n_refs, keep):
        import numpy as np
        self.id = rid
        self.score = np.full(2 * n_cals, -7, np.int32)
        self.ref_end = np.full(2 * n_cals, -7, np.int64)
        self.read_end = np.full(2 * n_cals, -7, np.int16)
        self.best_score = np.full(n_reads * n_refs, -7, np.int32)
        self.best_slot = np.full(n_reads * n_refs, -7, np.int64)
        self.n_tied = np.full(n_reads * n_refs, -7, np.int32)
        self.keep = keep
        self.n_reads, self.n_refs = n_reads, n_refs


class Server:
    """Served scoring (sw_server_*): resident references, admission by the
    footprint in a pinned device-mapped staging arena, continuous batching of
    admitted requests, per-request timestamps."""

    def __init__(self, scoring: Scoring, memory_budget: int = 1 << 30, max_step_reads: int = 65536,
                 max_step_cals: int = 1 << 20, max_step_chunks: int = 512, device: int = 0, autotune: bool = False,
                 max_steps_in_flight: int = 0):
        self._h = ctypes.c_void_p()
        opts = _ServerOpts(device, scoring, memory_budget, max_step_reads, max_step_cals, max_step_chunks,
                           int(autotune), max_steps_in_flight)
        _check(lib().sw_server_create(ctypes.byref(opts), ctypes.byref(self._h)), "sw_server_create")
        self.n_refs = 0
        self.requests = {}

    def set_refs(self, refs: "RefSet"):
        self._refs = refs
        self.n_refs = refs.n_refs
        _check(lib().sw_server_set_refs(self._h, refs.c), "sw_server_set_refs")

    def prepare(self, read_codes, read_code_off, read_len, cal_ptr, cal_pos, cal_ref, strand) -> Request:
        """Contiguous inputs and freshly allocated host outputs for one submission."""
        import numpy as np
        a = [np.ascontiguousarray(read_codes, np.uint8), np.ascontiguousarray(read_code_off, np.int64),
             np.ascontiguousarray(read_len, np.int32), np.ascontiguousarray(cal_ptr, np.int64),
             np.ascontiguousarray(cal_pos, np.int64), np.ascontiguousarray(cal_ref, np.int16),
             np.ascontiguousarray(strand, np.uint8)]
        req = Request(0, len(a[2]), len(a[4]), self.n_refs, a)
        p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
        req.args = (p(a[0]), len(a[0]), p(a[1]), p(a[2]), req.n_reads, p(a[3]), p(a[4]), p(a[5]), p(a[6]),
                    len(a[4]), p(req.score), p(req.ref_end), p(req.read_end), p(req.best_score), p(req.best_slot),
                    p(req.n_tied))
        return req

    def submit_prepared(self, req: Request) -> Request:
        rid = ctypes.c_int64(0)
        _check(lib().sw_server_submit(self._h, *req.args, ctypes.byref(rid)), "sw_server_submit")
        req.id = int(rid.value)
        self.requests[req.id] = req
        return req

    def submit(self, read_codes, read_code_off, read_len, cal_ptr, cal_pos, cal_ref, strand) -> Request:
        return self.submit_prepared(self.prepare(read_codes, read_code_off, read_len, cal_ptr, cal_pos, cal_ref,
                                                 strand))

    def prepare_batch(self, batch) -> Request:
        return self.prepare(batch.read_codes, batch.read_off, batch.read_len, batch.cal_ptr, batch.cal_pos,
                            batch.cal_ref, batch.strand)

    def submit_batch(self, batch) -> Request:
        return self.submit_prepared(self.prepare_batch(batch))

    def wait(self, req: Request, timeout_ms: int = -1) -> bool:
        done = ctypes.c_int32(0)
        _check(lib().sw_server_wait(self._h, req.id, timeout_ms, ctypes.byref(done)), "sw_server_wait")
        return bool(done.value)

    def info(self, req: Request):
        st = ctypes.c_int32(0)
        t = [ctypes.c_double(0) for _ in range(3)]
        _check(lib().sw_server_request_info(self._h, req.id, ctypes.byref(st), *[ctypes.byref(x) for x in t]),
               "sw_server_request_info")
        return int(st.value), t[0].value, t[1].value, t[2].value

    def release(self, req: Request):
        _check(lib().sw_server_release(self._h, req.id), "sw_server_release")
        self.requests.pop(req.id, None)

    def stats(self):
        st = _ServerStats()
        _check(lib().sw_server_stats(self._h, ctypes.byref(st)), "sw_server_stats")
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if self._h:
            lib().sw_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def error_count(reset: bool = False) -> int:
    v = ctypes.c_int64(0)
    _check(lib().sw_error_count(ctypes.byref(v), int(reset)), "sw_error_count")
    return int(v.value)

"""Thin Python binding of libsalo.so (argument marshalling only).

Every alignment step runs in the library's gfx950 kernels; this module only
turns torch tensors and streams into the pointers and sizes of the C ABI
(include/salo.h) and raises on a non-OK status.  There is no fallback: if
the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsalo.so")

MODE_AUTO, MODE_PLAIN, MODE_PERSISTENT = 0, 1, 2
_MODES = {"auto": MODE_AUTO, "plain": MODE_PLAIN, "persistent": MODE_PERSISTENT}


class SaloError(RuntimeError):
    """A non-OK status from the library."""

    def __init__(self, status: int, message: str):
        super().__init__("salo status %d: %s" % (status, message))
        self.status = status


class Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("force_int32", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("no_f16", ctypes.c_int32), ("split_waves", ctypes.c_int32)]


class Bin(ctypes.Structure):
    _fields_ = [("m_hi", ctypes.c_int32), ("packed", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("cols", ctypes.c_int32)]


_lock = threading.Lock()
_lib = None


def load(path: str | None = None):
    """Load libsalo.so (built by paper_2301_09310_amd.build)."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or os.environ.get("SALO_LIB") or LIB_PATH
        if not os.path.exists(p):
            raise ImportError("libsalo.so not found at %s; build it with "
                              "`python -m paper_2301_09310_amd.build`" % p)
        lib = ctypes.CDLL(p)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.salo_align_batch.argtypes = [vp, vp, vp, vp, i64, Scoring, vp, vp, vp, vp]
        lib.salo_align_batch.restype = i32
        lib.salo_align_batch_ex.argtypes = [vp, vp, vp, vp, i64, Scoring, vp, vp, vp,
                                            vp, ctypes.POINTER(Options)]
        lib.salo_align_batch_ex.restype = i32
        lib.salo_reserve.argtypes = [i64, vp]
        lib.salo_reserve.restype = i32
        lib.salo_error_count.argtypes = [vp, ctypes.POINTER(i64)]
        lib.salo_error_count.restype = i32
        lib.salo_last_error.argtypes = []
        lib.salo_last_error.restype = ctypes.c_char_p
        lib.salo_release.argtypes = []
        lib.salo_release.restype = None
        lib.salo_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_float)]
        lib.salo_last_timing.restype = i32
        lib.salo_set_bins.argtypes = [ctypes.POINTER(Bin), i32]
        lib.salo_set_bins.restype = i32
        lib.salo_get_bins.argtypes = [ctypes.POINTER(Bin), i32, ctypes.POINTER(i32)]
        lib.salo_get_bins.restype = i32
        lib.salo_version.argtypes = []
        lib.salo_version.restype = i32
        lib.salo_align_starts.argtypes = [vp, vp, vp, vp, vp, vp, i64, Scoring, vp, vp, vp, vp,
                                          vp, vp, ctypes.POINTER(Options)]
        lib.salo_align_starts.restype = i32
        lib.salo_pack_bases.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp, vp]
        lib.salo_align_batch_n.argtypes = [vp, vp, vp, vp, vp, vp, i64, Scoring, vp, vp, vp,
                                           vp, ctypes.POINTER(Options)]
        lib.salo_align_batch_n.restype = i32
        lib.salo_pack_bases.restype = i32
        lib.salo_align_batch_banded.argtypes = [vp, vp, vp, vp, i64, Scoring, i32, vp, vp, vp,
                                                vp, ctypes.POINTER(Options)]
        lib.salo_align_batch_banded.restype = i32
        lib.salo_align_trace.argtypes = [vp, vp, vp, vp, i64, Scoring, vp, vp, vp, vp, vp, vp,
                                         vp, vp, vp, i64, vp, ctypes.POINTER(Options)]
        lib.salo_align_trace.restype = i32
        lib.salo_align_batch_noalloc.argtypes = [vp, vp, vp, vp, i64, Scoring, vp, vp, vp, vp]
        lib.salo_align_batch_noalloc.restype = i32
        lib.salo_align_batch_tagged.argtypes = [vp, vp, vp, vp, i64, Scoring, vp, vp, vp, vp, vp,
                                                vp, ctypes.POINTER(Options)]
        lib.salo_align_batch_tagged.restype = i32
        lib.salo_host_alloc.argtypes = [i64, ctypes.POINTER(vp)]
        lib.salo_host_alloc.restype = i32
        lib.salo_host_free.argtypes = [vp]
        lib.salo_host_free.restype = i32
        if path is None:
            _lib = lib
        return lib


def _check(lib, st: int):
    if st != 0:
        raise SaloError(st, lib.salo_last_error().decode())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_options(mode="auto", lanes=0, cols=0, force_int32=False, waves_per_cu=0,
                 timing=False, no_f16=False, split_waves=0):
    o = Options()
    o.split_waves = int(split_waves)
    o.timing = 1 if timing else 0
    o.no_f16 = 1 if no_f16 else 0
    o.mode = _MODES[mode] if isinstance(mode, str) else int(mode)
    o.lanes, o.cols = int(lanes), int(cols)
    o.force_int32 = 1 if force_int32 else 0
    o.waves_per_cu = int(waves_per_cu)
    return o


def _mask_arg(mask, name):
    import torch
    if mask is None:
        return None
    if not mask.is_cuda or mask.dtype not in (torch.int32, torch.uint32) or \
            not mask.is_contiguous():
        raise ValueError("%s must be a contiguous 32-bit CUDA tensor" % name)
    return mask.data_ptr()


def align_batch(q_seqs, q_offsets, t_seqs, t_offsets, scoring=(1, -4, 6, 1),
                out=None, stream=None, q_nmask=None, t_nmask=None, **options):
    """Align every pair on the GPU.

    q_seqs/t_seqs: uint8 CUDA tensors (2-bit packed); q_offsets/t_offsets:
    int64 CUDA tensors of n_pairs+1 entries.  Returns (score, q_end, t_end)
    int32 CUDA tensors (or fills `out`, a triple of such tensors).
    q_nmask / t_nmask: optional int32 CUDA tensors, one bit per base marking
    N (salo_align_batch_n).  With no options and no masks the call goes
    to salo_align_batch itself, else to salo_align_batch_ex.  Keyword
    options: mode ('auto' | 'plain' | 'persistent'), lanes, cols, split_waves,
    force_int32, no_f16, waves_per_cu, timing.
    """
    import torch
    lib = load()
    n = q_offsets.numel() - 1
    if t_offsets.numel() - 1 != n:
        raise ValueError("offset arrays differ in length")
    for name, t, dt in (("q_seqs", q_seqs, torch.uint8), ("t_seqs", t_seqs, torch.uint8),
                        ("q_offsets", q_offsets, torch.int64),
                        ("t_offsets", t_offsets, torch.int64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dt))
    if out is None:
        dev = q_offsets.device
        out = tuple(torch.empty(max(n, 0), dtype=torch.int32, device=dev) for _ in range(3))
    sc = Scoring(*[int(x) for x in scoring])
    opts = make_options(**options)
    qm, tm = _mask_arg(q_nmask, "q_nmask"), _mask_arg(t_nmask, "t_nmask")
    if qm is None and tm is None and not options:
        # default options: the plain entry point of the ABI
        st = lib.salo_align_batch(q_seqs.data_ptr(), q_offsets.data_ptr(), t_seqs.data_ptr(),
                                  t_offsets.data_ptr(), n, sc, out[0].data_ptr(),
                                  out[1].data_ptr(), out[2].data_ptr(), _stream_handle(stream))
    elif qm is None and tm is None:
        st = lib.salo_align_batch_ex(q_seqs.data_ptr(), q_offsets.data_ptr(), t_seqs.data_ptr(),
                                     t_offsets.data_ptr(), n, sc, out[0].data_ptr(),
                                     out[1].data_ptr(), out[2].data_ptr(),
                                     _stream_handle(stream), ctypes.byref(opts))
    else:
        st = lib.salo_align_batch_n(q_seqs.data_ptr(), qm, q_offsets.data_ptr(),
                                    t_seqs.data_ptr(), tm, t_offsets.data_ptr(), n, sc,
                                    out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                                    _stream_handle(stream), ctypes.byref(opts))
    _check(lib, st)
    return out


def align_batch_noalloc(q_seqs, q_offsets, t_seqs, t_offsets, scoring=(1, -4, 6, 1),
                        out=None, stream=None):
    """salo_align_batch_noalloc: align_batch with the library's fixed
    scratch instead of an allocated workspace (at most 4,194,304 pairs;
    targets above 12,288 bases get -1).  `out` (a triple of int32 CUDA
    tensors) is allocated here when not given."""
    import torch
    lib = load()
    _check_inputs(q_seqs, q_offsets, t_seqs, t_offsets)
    n = q_offsets.numel() - 1
    if out is None:
        out = tuple(torch.empty(max(n, 0), dtype=torch.int32, device=q_offsets.device)
                    for _ in range(3))
    st = lib.salo_align_batch_noalloc(q_seqs.data_ptr(), q_offsets.data_ptr(),
                                      t_seqs.data_ptr(), t_offsets.data_ptr(), n,
                                      Scoring(*[int(x) for x in scoring]), out[0].data_ptr(),
                                      out[1].data_ptr(), out[2].data_ptr(),
                                      _stream_handle(stream))
    _check(lib, st)
    return out


def align_batch_tagged(q_seqs, q_offsets, t_seqs, t_offsets, scoring, out_ptrs, pair_tag,
                       tag_done_ptr, stream=None, **options):
    """salo_align_batch_tagged: align_batch whose pair p adds 1 to the host
    counter tag_done[pair_tag[p]] once its outputs are written.  out_ptrs:
    three addresses of int32 [n_pairs] outputs (device memory or
    host_alloc memory); pair_tag: int32 CUDA tensor [n_pairs];
    tag_done_ptr: address of host_alloc memory holding the counters."""
    import torch
    lib = load()
    n = _check_inputs(q_seqs, q_offsets, t_seqs, t_offsets)
    if not pair_tag.is_cuda or pair_tag.dtype != torch.int32 or pair_tag.numel() < n:
        raise ValueError("pair_tag must be an int32 CUDA tensor of n_pairs entries")
    opts = make_options(**options)
    st = lib.salo_align_batch_tagged(q_seqs.data_ptr(), q_offsets.data_ptr(), t_seqs.data_ptr(),
                                     t_offsets.data_ptr(), n, Scoring(*[int(x) for x in scoring]),
                                     out_ptrs[0], out_ptrs[1], out_ptrs[2], pair_tag.data_ptr(),
                                     tag_done_ptr, _stream_handle(stream), ctypes.byref(opts))
    _check(lib, st)


class HostBuffer:
    """Host memory from salo_host_alloc (coherent for host and device), as a
    numpy array of `count` elements of `dtype`; freed by free() or when
    collected."""

    def __init__(self, count: int, dtype):
        import numpy as np
        lib = load()
        self.dtype = np.dtype(dtype)
        self.nbytes = max(int(count) * self.dtype.itemsize, 4)
        p = ctypes.c_void_p(0)
        _check(lib, lib.salo_host_alloc(self.nbytes, ctypes.byref(p)))
        self.ptr = int(p.value)
        buf = (ctypes.c_uint8 * self.nbytes).from_address(self.ptr)
        self.array = np.frombuffer(buf, dtype=self.dtype, count=int(count))

    def free(self):
        if self.ptr:
            self.array = None
            load().salo_host_free(ctypes.c_void_p(self.ptr))
            self.ptr = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _check_inputs(q_seqs, q_offsets, t_seqs, t_offsets):
    import torch
    n = q_offsets.numel() - 1
    if t_offsets.numel() - 1 != n:
        raise ValueError("offset arrays differ in length")
    for name, t, dt in (("q_seqs", q_seqs, torch.uint8), ("t_seqs", t_seqs, torch.uint8),
                        ("q_offsets", q_offsets, torch.int64),
                        ("t_offsets", t_offsets, torch.int64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dt))
    return n


def align_banded(q_seqs, q_offsets, t_seqs, t_offsets, band: int, scoring=(1, -4, 6, 1),
                 out=None, stream=None, **options):
    """Banded alignment (salo_align_batch_banded): Eq. 1 over the cells with
    |i - j| <= band.  Arguments and result as align_batch; options as
    align_batch (mode 'plain' is not supported)."""
    import torch
    lib = load()
    n = _check_inputs(q_seqs, q_offsets, t_seqs, t_offsets)
    if out is None:
        dev = q_offsets.device
        out = tuple(torch.empty(max(n, 0), dtype=torch.int32, device=dev) for _ in range(3))
    sc = Scoring(*[int(x) for x in scoring])
    opts = make_options(**options)
    st = lib.salo_align_batch_banded(q_seqs.data_ptr(), q_offsets.data_ptr(), t_seqs.data_ptr(),
                                     t_offsets.data_ptr(), n, sc, int(band), out[0].data_ptr(),
                                     out[1].data_ptr(), out[2].data_ptr(),
                                     _stream_handle(stream), ctypes.byref(opts))
    _check(lib, st)
    return out


CIGAR_OPS = {7: "=", 8: "X", 1: "I", 2: "D"}


def cigar_offsets(q_offsets, t_offsets):
    """Device int64 offsets giving each pair room for m + n CIGAR runs."""
    import torch
    cap = (q_offsets[1:] - q_offsets[:-1]) + (t_offsets[1:] - t_offsets[:-1])
    off = torch.zeros(cap.numel() + 1, dtype=torch.int64, device=q_offsets.device)
    torch.cumsum(cap, 0, out=off[1:])
    return off


def align_trace(q_seqs, q_offsets, t_seqs, t_offsets, answers, starts, scoring=(1, -4, 6, 1),
                cig_off=None, workspace=None, workspace_bytes=1 << 30, stream=None, out=None,
                **options):
    """CIGAR of every pair's best alignment (salo_align_trace).
    answers: (score, q_end, t_end) of align_batch; starts: (q_start,
    t_start) of align_starts.  Returns (cig_off, cig, cig_len): int64
    offsets, uint32 runs (as int32 storage), int32 run counts, all CUDA.
    workspace: a CUDA uint8 tensor (allocated with workspace_bytes if None).
    out: (cig, cig_len) to fill; with cig_off and workspace also given, the
    call allocates nothing and does not synchronise (graph capture)."""
    import torch
    lib = load()
    n = _check_inputs(q_seqs, q_offsets, t_seqs, t_offsets)
    arrs = (answers[0], starts[0], answers[1], starts[1], answers[2])
    for t in arrs:
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous() or t.numel() != n:
            raise ValueError("answers and starts must be contiguous int32 CUDA tensors")
    dev = q_offsets.device
    # buffers made here are made, and their contents computed, on the
    # launch stream, after the work the current stream has queued (which
    # produced the inputs); each is marked as used by that stream, so the
    # caching allocator cannot hand it to other work while the kernel runs
    launch = stream if stream is not None else torch.cuda.current_stream(dev)
    made = []
    if launch != torch.cuda.current_stream(dev):
        launch.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(launch):
        if cig_off is None:
            cig_off = cigar_offsets(q_offsets, t_offsets)
            made.append(cig_off)
        if out is None:
            total = int(cig_off[-1].item()) if n > 0 else 0
            cig = torch.zeros(max(total, 1), dtype=torch.int32, device=dev)
            cig_len = torch.empty(max(n, 0), dtype=torch.int32, device=dev)
            made += [cig, cig_len]
        else:
            cig, cig_len = out
            if cig.dtype != torch.int32 or cig_len.dtype != torch.int32 or \
                    not cig.is_contiguous() or cig_len.numel() != n:
                raise ValueError("out must be (int32 cig, int32 cig_len of n_pairs) CUDA "
                                 "tensors")
        if workspace is None:
            workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=dev)
            made.append(workspace)
    sc = Scoring(*[int(x) for x in scoring])
    opts = make_options(**options)
    st = lib.salo_align_trace(q_seqs.data_ptr(), q_offsets.data_ptr(), t_seqs.data_ptr(),
                              t_offsets.data_ptr(), n, sc, *(x.data_ptr() for x in arrs),
                              cig_off.data_ptr(), cig.data_ptr(), cig_len.data_ptr(),
                              workspace.data_ptr(), workspace.numel(), _stream_handle(launch),
                              ctypes.byref(opts))
    _check(lib, st)
    if launch != torch.cuda.current_stream(dev):
        for t in made:
            t.record_stream(launch)
    return cig_off, cig, cig_len


def align_starts(q_seqs, q_offsets, t_seqs, t_offsets, answers, scoring=(1, -4, 6, 1),
                 out=None, stream=None, q_nmask=None, t_nmask=None, **options):
    """Start positions of the align call's answers (salo_align_starts).
    answers: the (score, q_end, t_end) int32 CUDA tensors of align_batch on
    the same inputs and scoring.  Returns (q_start, t_start) int32 CUDA
    tensors (or fills `out`, a pair)."""
    import torch
    lib = load()
    n = q_offsets.numel() - 1
    for name, t in zip(("score", "q_end", "t_end"), answers):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous() or t.numel() != n:
            raise ValueError("%s must be a contiguous int32 CUDA tensor of n_pairs" % name)
    if out is None:
        dev = q_offsets.device
        out = tuple(torch.empty(max(n, 0), dtype=torch.int32, device=dev) for _ in range(2))
    sc = Scoring(*[int(x) for x in scoring])
    opts = make_options(**options)
    st = lib.salo_align_starts(q_seqs.data_ptr(), _mask_arg(q_nmask, "q_nmask"),
                               q_offsets.data_ptr(), t_seqs.data_ptr(),
                               _mask_arg(t_nmask, "t_nmask"), t_offsets.data_ptr(), n, sc,
                               answers[0].data_ptr(),
                               answers[1].data_ptr(), answers[2].data_ptr(), out[0].data_ptr(),
                               out[1].data_ptr(), _stream_handle(stream), ctypes.byref(opts))
    _check(lib, st)
    return out


def align_batch_raw(q_ptr, q_off_ptr, t_ptr, t_off_ptr, n_pairs, scoring, s_ptr, qe_ptr,
                    te_ptr, stream_handle=None, options=None):
    """Direct pass-through of salo_align_batch_ex with raw addresses;
    returns the status code (no exception)."""
    lib = load()
    opts = options if options is not None else make_options()
    return lib.salo_align_batch_ex(q_ptr, q_off_ptr, t_ptr, t_off_ptr, int(n_pairs),
                                   Scoring(*[int(x) for x in scoring]), s_ptr, qe_ptr, te_ptr,
                                   stream_handle, ctypes.byref(opts))


def last_timing(stream=None):
    """(plan_ms, dp_ms) of the last call made with timing=True on `stream`."""
    lib = load()
    a, b = ctypes.c_float(0), ctypes.c_float(0)
    _check(lib, lib.salo_last_timing(_stream_handle(stream), ctypes.byref(a), ctypes.byref(b)))
    return float(a.value), float(b.value)


def set_bins(bins):
    """Install a bin table: a list of (m_hi, packed, lanes[, cols]) (cols:
    query columns per lane, 8/16/32, 0 or absent for 16); None restores the
    built-in table."""
    lib = load()
    if bins is None:
        _check(lib, lib.salo_set_bins(None, 0))
        return
    arr = (Bin * len(bins))(*[Bin(int(b[0]), int(b[1]), int(b[2]),
                                  int(b[3]) if len(b) > 3 else 0) for b in bins])
    _check(lib, lib.salo_set_bins(arr, len(bins)))


def get_bins():
    """The current bin table as (m_hi, packed, lanes, cols) tuples."""
    lib = load()
    arr = (Bin * 16)()
    n = ctypes.c_int32(0)
    _check(lib, lib.salo_get_bins(arr, 16, ctypes.byref(n)))
    return [(arr[i].m_hi, arr[i].packed, arr[i].lanes, arr[i].cols or 16)
            for i in range(n.value)]


def load_tune_table(path: str, key: str = "bins") -> None:
    """Install a bin table of an autotuner JSON file: `bins` (throughput,
    the built-in default) or `serve_bins` (latency, for served streams).
    The table applies to every later call in this process."""
    import json
    with open(path) as f:
        t = json.load(f)
    set_bins([(b["m_hi"], b["packed"], b["lanes"], b.get("cols", 0)) for b in t[key]])


def pack_bases(chars, offsets=None, revcomp: bool = False, out=None, invalid=None,
               stream=None, n_mask=None):
    """Pack character reads on the GPU (salo_pack_bases).  chars: uint8
    CUDA tensor; offsets: int64 CUDA tensor (sequence CSR, needed for
    revcomp).  Returns the packed uint8 CUDA tensor of ceil(n/16)*4 bytes
    (or fills `out`).  `invalid`, if given, is an int64 CUDA tensor of one
    element to which the number of invalid bases is added.  `n_mask`, if
    given, is an int32 CUDA tensor of ceil(n/32) words that receives the N
    bits (N and n then count as bases)."""
    import torch
    lib = load()
    if not chars.is_cuda or chars.dtype != torch.uint8 or not chars.is_contiguous():
        raise ValueError("chars must be a contiguous uint8 CUDA tensor")
    n = chars.numel()
    nbytes = ((n + 15) // 16) * 4
    if out is None:
        out = torch.empty(max(nbytes, 4), dtype=torch.uint8, device=chars.device)
    if out.numel() < nbytes:
        raise ValueError("out holds %d bytes, %d needed" % (out.numel(), nbytes))
    n_seqs = 0
    off_ptr = None
    if offsets is not None:
        if not offsets.is_cuda or offsets.dtype != torch.int64 or not offsets.is_contiguous():
            raise ValueError("offsets must be a contiguous int64 CUDA tensor")
        n_seqs = offsets.numel() - 1
        off_ptr = offsets.data_ptr()
    inv_ptr = None
    if invalid is not None:
        if not invalid.is_cuda or invalid.dtype != torch.int64:
            raise ValueError("invalid must be an int64 CUDA tensor")
        inv_ptr = invalid.data_ptr()
    nm_ptr = None
    if n_mask is not None:
        if n_mask.numel() < (n + 31) // 32:
            raise ValueError("n_mask holds %d words, %d needed" % (n_mask.numel(),
                                                                  (n + 31) // 32))
        nm_ptr = _mask_arg(n_mask, "n_mask")
    st = lib.salo_pack_bases(chars.data_ptr() if n else None, n, off_ptr, n_seqs,
                             1 if revcomp else 0, out.data_ptr(), nm_ptr, inv_ptr,
                             _stream_handle(stream))
    _check(lib, st)
    return out


def reserve(max_pairs: int, stream=None):
    lib = load()
    _check(lib, lib.salo_reserve(int(max_pairs), _stream_handle(stream)))


def error_count(stream=None) -> int:
    lib = load()
    v = ctypes.c_int64(0)
    _check(lib, lib.salo_error_count(_stream_handle(stream), ctypes.byref(v)))
    return int(v.value)


def last_error() -> str:
    return load().salo_last_error().decode()


def release():
    load().salo_release()


def version() -> int:
    return int(load().salo_version())


def to_device(batch, device="cuda"):
    """Copy a packed inputs.Batch to device tensors (q, q_off, t, t_off)."""
    import torch
    return (torch.from_numpy(batch.q_seqs).to(device),
            torch.from_numpy(batch.q_offsets).to(device),
            torch.from_numpy(batch.t_seqs).to(device),
            torch.from_numpy(batch.t_offsets).to(device))

"""MI355X decoder for the absolute-offset LZ77 block format (AXP1).

Thin ctypes binding of `libaceapex.so` (the C ABI in include/aceapex.h):
argument marshalling only.  Every step of a decode runs in the library's HIP
kernels; PyTorch supplies device memory and the stream.  There is no CPU
fallback: without the built library every call raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaceapex.so")
_lib = None

AX_OK, AX_E_ARG, AX_E_CORRUPT, AX_E_UNSUPPORTED, AX_E_CAPACITY = 0, -1, -2, -3, -4
AX_E_HIP, AX_E_RANGE, AX_E_DEVICE, AX_E_NOMEM = -5, -6, -7, -8
COPY_PERIODIC, COPY_SERIAL = 0, 1

EXPORTS = [
    "aceapex_strerror", "aceapex_last_error", "aceapex_encode_params_default", "aceapex_encode_bound",
    "aceapex_encode", "aceapex_read_info", "aceapex_decoder_create", "aceapex_decoder_destroy",
    "aceapex_decoder_info", "aceapex_decoder_workspace", "aceapex_decode_all", "aceapex_decode_all_static",
    "aceapex_decoder_stage_ms",
    "aceapex_decoder_set_timing", "aceapex_decoder_status", "aceapex_decoder_set_option",
    "aceapex_workspace_status", "aceapex_batch_create", "aceapex_batch_destroy", "aceapex_batch_workspace",
    "aceapex_batch_set_option", "aceapex_batch_set_timing", "aceapex_batch_stage_ms", "aceapex_decode_batch",
    "aceapex_decoder_build_index", "aceapex_closure_blocks", "aceapex_range_plan_create", "aceapex_range_plan_destroy",
    "aceapex_range_plan_workspace", "aceapex_range_plan_last", "aceapex_decode_ranges", "aceapex_decode_range",
    "aceapex_range_workspace", "aceapex_decoder_streams", "aceapex_decoder_tokens",
    "aceapex_closure_sizes",
]
OPT_BULK_ROUNDS, OPT_FILL_ROUNDS, OPT_FILL_TAIL, OPT_TAIL_CHUNKS, OPT_GRAPH, OPT_ROUND0_TILE = 1, 2, 3, 4, 5, 6
OPT_TAIL_MODE, OPT_JUMP_PASSES, OPT_RANGE_JUMP_TOKENS = 7, 8, 9
TAIL_JUMP, TAIL_CHASE = 0, 1
STATIC_SCRATCH_BYTES = 128 << 20  # AX_STATIC_SCRATCH_BYTES


class AceapexError(RuntimeError):
    def __init__(self, code, what):
        lib = _load()
        detail = lib.aceapex_last_error().decode(errors="replace")
        super().__init__(f"{what}: {lib.aceapex_strerror(code).decode()} ({code}) {detail}")
        self.code = code


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64)


class EncodeParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "block_size", "min_match", "no_rep", "depth_cap", "hash_bits", "chain_depth",
        "rans_min_syms_per_lane", "off_cost_q", "window_log", "threads")] + [
        ("progress", PROGRESS_FN), ("progress_user", ctypes.c_void_p)]


class EncodeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_bytes", "n_blocks", "comp_bytes", "n_commands", "n_matches", "n_rep", "n_match_bytes",
        "n_lit_bytes", "n_src_bytes", "n_off_bytes", "n_len_bytes")] + [
        ("max_depth", ctypes.c_uint32), ("passes", ctypes.c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_bytes", "n_blocks", "archive_bytes", "header_bytes", "payload_bytes", "n_matches", "xxh3")] + [
        (n, ctypes.c_uint32) for n in ("block_size", "min_match", "flags", "depth_cap")]


class Job(ctypes.Structure):
    _fields_ = [("dec", ctypes.c_void_p), ("d_out", ctypes.c_void_p), ("out_cap", ctypes.c_uint64)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, vp, u64, u32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    u8p = P(ctypes.c_uint8)
    L.aceapex_strerror.argtypes = [ctypes.c_int]
    L.aceapex_strerror.restype = ctypes.c_char_p
    L.aceapex_last_error.argtypes = []
    L.aceapex_last_error.restype = ctypes.c_char_p
    L.aceapex_encode_params_default.argtypes = [P(EncodeParams)]
    L.aceapex_encode_params_default.restype = None
    L.aceapex_encode_bound.argtypes = [u64, P(EncodeParams), P(u64)]
    L.aceapex_encode.argtypes = [u8p, u64, P(EncodeParams), u8p, u64, P(u64), P(EncodeStats)]
    L.aceapex_read_info.argtypes = [u8p, u64, P(Info)]
    L.aceapex_decoder_create.argtypes = [u8p, u64, vp, u64, P(vp)]
    L.aceapex_decoder_destroy.argtypes = [vp]
    L.aceapex_decoder_destroy.restype = None
    L.aceapex_decoder_info.argtypes = [vp, P(Info)]
    L.aceapex_decoder_workspace.argtypes = [vp, P(u64)]
    L.aceapex_decode_all.argtypes = [vp, vp, u64, vp, u64, ctypes.c_int, vp]
    L.aceapex_decode_all_static.argtypes = [vp, vp, u64, ctypes.c_int, vp]
    L.aceapex_decoder_stage_ms.argtypes = [vp] + [P(ctypes.c_float)] * 4
    L.aceapex_decoder_set_timing.argtypes = [vp, ctypes.c_int]
    L.aceapex_decoder_status.argtypes = [vp, vp, vp, P(ctypes.c_int32), P(u64)]
    L.aceapex_decoder_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int64]
    L.aceapex_workspace_status.argtypes = [vp, vp, P(ctypes.c_int32), P(u64)]
    L.aceapex_batch_create.argtypes = [P(Job), ctypes.c_uint32, P(vp)]
    L.aceapex_batch_destroy.argtypes = [vp]
    L.aceapex_batch_destroy.restype = None
    L.aceapex_batch_workspace.argtypes = [vp, P(u64)]
    L.aceapex_batch_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int64]
    L.aceapex_batch_set_timing.argtypes = [vp, ctypes.c_int]
    L.aceapex_batch_stage_ms.argtypes = [vp] + [P(ctypes.c_float)] * 4
    L.aceapex_decode_batch.argtypes = [vp, vp, u64, ctypes.c_int, vp]
    u64p = P(u64)
    L.aceapex_decoder_build_index.argtypes = [vp, vp, u64, vp]
    L.aceapex_closure_blocks.argtypes = [vp, ctypes.c_uint32, u64p, u64p, u64p, u64, u64p, u64p, ctypes.c_uint32]
    L.aceapex_closure_sizes.argtypes = [vp, ctypes.c_uint32, u64p, u64p, u64p, u64p, ctypes.c_uint32]
    L.aceapex_range_plan_create.argtypes = [vp, u64, u64, P(vp)]
    L.aceapex_range_plan_destroy.argtypes = [vp]
    L.aceapex_range_plan_destroy.restype = None
    L.aceapex_range_plan_workspace.argtypes = [vp, u64p]
    L.aceapex_range_plan_last.argtypes = [vp, u64p, u64p]
    L.aceapex_decode_ranges.argtypes = [vp, ctypes.c_uint32, u64p, u64p, P(vp), u64p, vp, u64, ctypes.c_int, vp]
    L.aceapex_decode_range.argtypes = [vp, u64, u64, vp, u64, vp, u64, vp]
    L.aceapex_range_workspace.argtypes = [vp, u64, u64, u64p]
    L.aceapex_decoder_streams.argtypes = [vp, u64, u64, vp, u64, vp, u8p, u64, P(ctypes.c_uint32)]
    L.aceapex_decoder_tokens.argtypes = [vp, u64, u64, u64p, u64p, P(ctypes.c_uint32)]
    _lib = L
    return L


def lib():
    return _load()


def _check(rc, what):
    if rc != AX_OK:
        raise AceapexError(rc, what)


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def encode_params(**kw):
    p = EncodeParams()
    _load().aceapex_encode_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, int(v))
    return p


def encode(data, stats=False, progress=None, **kw):
    """Host encode (aceapex_encode).  Returns the archive as a uint8 array.
    progress(bytes_done, bytes_total), if given, runs after each segment."""
    a = np.ascontiguousarray(np.frombuffer(data, np.uint8) if isinstance(data, (bytes, bytearray)) else data,
                             dtype=np.uint8)
    p = encode_params(**kw)
    cb = PROGRESS_FN(lambda _u, done, total: progress(done, total)) if progress else None
    if cb:
        p.progress = cb
    bound = ctypes.c_uint64()
    _check(_load().aceapex_encode_bound(a.size, ctypes.byref(p), ctypes.byref(bound)), "encode_bound")
    out = np.empty(bound.value, np.uint8)
    n = ctypes.c_uint64()
    st = EncodeStats()
    _check(_load().aceapex_encode(_u8(a), a.size, ctypes.byref(p), _u8(out), out.size, ctypes.byref(n),
                                  ctypes.byref(st)), "encode")
    arc = out[: n.value].copy()
    return (arc, st) if stats else arc


def read_info(prefix):
    a = np.ascontiguousarray(prefix[:64] if not isinstance(prefix, (bytes, bytearray)) else
                             np.frombuffer(bytes(prefix[:64]), np.uint8), dtype=np.uint8)
    inf = Info()
    _check(_load().aceapex_read_info(_u8(a), a.size, ctypes.byref(inf)), "read_info")
    return inf


def _stream_ptr(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Decoder:
    """A decoder for one archive resident in device memory.

    h_archive: host bytes holding at least the header and index.
    d_archive: torch.uint8 CUDA tensor holding the whole archive.
    """

    def __init__(self, h_archive, d_archive):
        import torch

        h = np.ascontiguousarray(h_archive, dtype=np.uint8)
        self.info = read_info(h)
        if h.size < self.info.header_bytes:
            raise ValueError("host copy must hold the header and index")
        if d_archive.dtype != torch.uint8 or not d_archive.is_cuda:
            raise ValueError("d_archive must be a CUDA uint8 tensor")
        self._d_archive = d_archive  # keep alive
        self._h = ctypes.c_void_p()
        _check(_load().aceapex_decoder_create(_u8(h), int(self.info.header_bytes), ctypes.c_void_p(d_archive.data_ptr()),
                                              d_archive.numel(), ctypes.byref(self._h)), "decoder_create")
        ws = ctypes.c_uint64()
        _check(_load().aceapex_decoder_workspace(self._h, ctypes.byref(ws)), "decoder_workspace")
        self.workspace_bytes = ws.value
        self._work = None
        self.device = d_archive.device

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.aceapex_decoder_destroy(self._h)
            self._h = None

    def workspace(self):
        import torch

        if self._work is None:
            self._work = torch.empty(max(256, self.workspace_bytes), dtype=torch.uint8, device=self.device)
        return self._work

    def set_option(self, option, value):
        _check(_load().aceapex_decoder_set_option(self._h, int(option), int(value)), "set_option")

    def set_bulk_rounds(self, rounds):
        self.set_option(OPT_BULK_ROUNDS, rounds)

    def set_timing(self, on=True):
        _check(_load().aceapex_decoder_set_timing(self._h, int(bool(on))), "set_timing")

    def decode_all(self, out=None, copy_mode=COPY_PERIODIC, stream=None, work=None):
        """Enqueue a full decode; returns the output tensor (async)."""
        import torch

        n = int(self.info.n_bytes)
        if out is None:
            out = torch.empty(max(16, n), dtype=torch.uint8, device=self.device)
        w = self.workspace() if work is None else work
        _check(_load().aceapex_decode_all(self._h, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                          ctypes.c_void_p(w.data_ptr()), w.numel(), int(copy_mode),
                                          _stream_ptr(stream)), "decode_all")
        return out[:n] if out.numel() != n else out

    def decode_all_static(self, out, copy_mode=COPY_PERIODIC, stream=None):
        """Enqueue a full decode whose workspace is the library's static
        device scratch (aceapex_decode_all_static: allocates nothing)."""
        _check(_load().aceapex_decode_all_static(self._h, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                                 int(copy_mode), _stream_ptr(stream)), "decode_all_static")
        return out

    def static_status(self, stream=None):
        """Device status of the last aceapex_decode_all_static on the current device."""
        err = ctypes.c_int32()
        bad = ctypes.c_uint64()
        _check(_load().aceapex_decoder_status(self._h, None, _stream_ptr(stream), ctypes.byref(err),
                                              ctypes.byref(bad)), "decoder_status")
        return err.value, bad.value

    def status(self, stream=None, work=None):
        err = ctypes.c_int32()
        bad = ctypes.c_uint64()
        w = self.workspace() if work is None else work
        _check(_load().aceapex_decoder_status(self._h, ctypes.c_void_p(w.data_ptr()), _stream_ptr(stream),
                                              ctypes.byref(err), ctypes.byref(bad)), "decoder_status")
        return err.value, bad.value

    def build_index(self, stream=None, work=None):
        """Token index for range closures (device parse pass; synchronous)."""
        w = self.workspace() if work is None else work
        _check(_load().aceapex_decoder_build_index(self._h, ctypes.c_void_p(w.data_ptr()), w.numel(),
                                                   _stream_ptr(stream)), "build_index")

    def range_workspace(self, off, length):
        """Device workspace bytes aceapex_decode_range needs for [off, off+length)."""
        b = ctypes.c_uint64()
        _check(_load().aceapex_range_workspace(self._h, int(off), int(length), ctypes.byref(b)), "range_workspace")
        return b.value

    def decode_range(self, off, length, out, work, stream=None):
        """Enqueue the decode of one byte range into `out` (a CUDA uint8
        tensor of at least `length` bytes); `work` holds at least
        range_workspace(off, length) bytes."""
        _check(_load().aceapex_decode_range(self._h, int(off), int(length), ctypes.c_void_p(out.data_ptr()),
                                            out.numel(), ctypes.c_void_p(work.data_ptr()), work.numel(),
                                            _stream_ptr(stream)), "decode_range")
        return out

    def streams(self, first, count=1, stream=None, work=None):
        """The entropy stage alone: the decoded LIT, LEN, OFF and CMD streams
        of blocks [first, first + count), one dict per block (synchronous)."""
        w = self.workspace() if work is None else work
        B, mm = int(self.info.block_size), int(self.info.min_match)
        cap = int(count) * (5 * B + 10 * (B // mm + 1) + 16)
        buf = np.zeros(max(1, cap), np.uint8)
        n = np.zeros(max(1, 4 * int(count)), np.uint32)
        _check(_load().aceapex_decoder_streams(self._h, int(first), int(count), ctypes.c_void_p(w.data_ptr()),
                                               w.numel(), _stream_ptr(stream), _u8(buf), cap,
                                               n.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))), "decoder_streams")
        out, at = [], 0
        for i in range(int(count)):
            blk = {}
            for k, name in enumerate(("lit", "len", "off", "cmd")):
                m = int(n[4 * i + k])
                blk[name] = buf[at: at + m].copy()
                at += m
            out.append(blk)
        return out

    def tokens(self, first, count):
        """Matches [first, first + count) of the device parse (build_index
        first): (src, dst, len) arrays."""
        src = np.zeros(max(1, int(count)), np.uint64)
        dst = np.zeros(max(1, int(count)), np.uint64)
        ln = np.zeros(max(1, int(count)), np.uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        _check(_load().aceapex_decoder_tokens(self._h, int(first), int(count), src.ctypes.data_as(u64p),
                                              dst.ctypes.data_as(u64p),
                                              ln.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))), "decoder_tokens")
        c = int(count)
        return src[:c], dst[:c], ln[:c]

    def closure_sizes(self, offs, lens, threads=0):
        """Closure size of each range on its own: (blocks, matches) arrays."""
        o = np.ascontiguousarray(offs, dtype=np.uint64)
        ln = np.ascontiguousarray(lens, dtype=np.uint64)
        nb = np.zeros(max(1, o.size), np.uint64)
        nt = np.zeros(max(1, o.size), np.uint64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        _check(_load().aceapex_closure_sizes(self._h, o.size, o.ctypes.data_as(u64p), ln.ctypes.data_as(u64p),
                                             nb.ctypes.data_as(u64p), nt.ctypes.data_as(u64p), threads),
               "closure_sizes")
        return nb[: o.size], nt[: o.size]

    def closure_blocks(self, offs, lens, threads=0, want_blocks=True):
        """Union source closure of ranges: (ascending block array, match count)."""
        o = np.ascontiguousarray(offs, dtype=np.uint64)
        ln = np.ascontiguousarray(lens, dtype=np.uint64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        nb, nt = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_load().aceapex_closure_blocks(self._h, o.size, o.ctypes.data_as(u64p), ln.ctypes.data_as(u64p), None, 0,
                                              ctypes.byref(nb), ctypes.byref(nt), threads), "closure_blocks")
        if not want_blocks:
            return None, nt.value, nb.value
        blocks = np.zeros(max(1, nb.value), np.uint64)
        _check(_load().aceapex_closure_blocks(self._h, o.size, o.ctypes.data_as(u64p), ln.ctypes.data_as(u64p),
                                              blocks.ctypes.data_as(u64p), blocks.size, ctypes.byref(nb),
                                              ctypes.byref(nt), threads), "closure_blocks")
        return blocks[: nb.value], nt.value, nb.value

    def stage_ms(self, remainder=False):
        """(entropy, parse, copy) ms of the last timed decode, summed over
        windows; remainder=True appends the copy's deep-remainder part."""
        a, p, c, r = ctypes.c_float(), ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        _check(_load().aceapex_decoder_stage_ms(self._h, ctypes.byref(a), ctypes.byref(p), ctypes.byref(c),
                                                ctypes.byref(r)), "stage_ms")
        return (a.value, p.value, c.value, r.value) if remainder else (a.value, p.value, c.value)


def workspace_status(work, stream=None):
    err = ctypes.c_int32()
    bad = ctypes.c_uint64()
    _check(_load().aceapex_workspace_status(ctypes.c_void_p(work.data_ptr()), _stream_ptr(stream), ctypes.byref(err),
                                            ctypes.byref(bad)), "workspace_status")
    return err.value, bad.value


class Batch:
    """Many whole archives decoded by one plan (aceapex_decode_batch).

    decoders: list of Decoder; outs: list of CUDA uint8 tensors (one per
    decoder, at least its decoded size)."""

    def __init__(self, decoders, outs):
        n = len(decoders)
        jobs = (Job * max(1, n))()
        for i, (d, o) in enumerate(zip(decoders, outs)):
            if o.numel() < d.info.n_bytes:
                raise ValueError("output tensor smaller than the decoded size")
            jobs[i].dec, jobs[i].d_out, jobs[i].out_cap = d._h, o.data_ptr(), o.numel()
        self._decoders, self._outs = list(decoders), list(outs)  # keep alive
        self._h = ctypes.c_void_p()
        _check(_load().aceapex_batch_create(jobs, n, ctypes.byref(self._h)), "batch_create")
        ws = ctypes.c_uint64()
        _check(_load().aceapex_batch_workspace(self._h, ctypes.byref(ws)), "batch_workspace")
        self.workspace_bytes = ws.value
        self.device = outs[0].device if outs else None
        self._work = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.aceapex_batch_destroy(self._h)
            self._h = None

    def workspace(self):
        import torch

        if self._work is None:
            self._work = torch.empty(max(256, self.workspace_bytes), dtype=torch.uint8, device=self.device)
        return self._work

    def set_option(self, option, value):
        _check(_load().aceapex_batch_set_option(self._h, int(option), int(value)), "batch_set_option")

    def set_timing(self, on=True):
        _check(_load().aceapex_batch_set_timing(self._h, int(bool(on))), "batch_set_timing")

    def stage_ms(self, remainder=False):
        a, p, c, r = ctypes.c_float(), ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        _check(_load().aceapex_batch_stage_ms(self._h, ctypes.byref(a), ctypes.byref(p), ctypes.byref(c),
                                              ctypes.byref(r)), "batch_stage_ms")
        return (a.value, p.value, c.value, r.value) if remainder else (a.value, p.value, c.value)

    def decode(self, copy_mode=COPY_PERIODIC, stream=None, work=None):
        w = self.workspace() if work is None else work
        _check(_load().aceapex_decode_batch(self._h, ctypes.c_void_p(w.data_ptr()), w.numel(), int(copy_mode),
                                            _stream_ptr(stream)), "decode_batch")
        return self._outs

    def decode_all_static(self, out, copy_mode=COPY_PERIODIC, stream=None):
        """Enqueue a full decode whose workspace is the library's static
        device scratch (aceapex_decode_all_static: allocates nothing)."""
        _check(_load().aceapex_decode_all_static(self._h, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                                 int(copy_mode), _stream_ptr(stream)), "decode_all_static")
        return out

    def static_status(self, stream=None):
        """Device status of the last aceapex_decode_all_static on the current device."""
        err = ctypes.c_int32()
        bad = ctypes.c_uint64()
        _check(_load().aceapex_decoder_status(self._h, None, _stream_ptr(stream), ctypes.byref(err),
                                              ctypes.byref(bad)), "decoder_status")
        return err.value, bad.value

    def status(self, stream=None, work=None):
        return workspace_status(self.workspace() if work is None else work, stream)


class RangePlan:
    """Reusable range decode (aceapex_decode_ranges) for one decoder."""

    def __init__(self, decoder, max_blocks=4096, max_tokens=1 << 20):
        self.decoder = decoder
        self._h = ctypes.c_void_p()
        _check(_load().aceapex_range_plan_create(decoder._h, int(max_blocks), int(max_tokens), ctypes.byref(self._h)),
               "range_plan_create")
        ws = ctypes.c_uint64()
        _check(_load().aceapex_range_plan_workspace(self._h, ctypes.byref(ws)), "range_plan_workspace")
        self.workspace_bytes = ws.value
        self.max_blocks, self.max_tokens = int(max_blocks), int(max_tokens)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.aceapex_range_plan_destroy(self._h)
            self._h = None

    def last(self):
        b, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_load().aceapex_range_plan_last(self._h, ctypes.byref(b), ctypes.byref(t)), "range_plan_last")
        return b.value, t.value

    def decode(self, offs, lens, outs, work, copy_mode=COPY_PERIODIC, stream=None):
        """Enqueue the decode of ranges; outs: CUDA uint8 tensors (at least
        len bytes each).  Raises AceapexError(AX_E_CAPACITY) when the closure
        exceeds the limits or an output is too small."""
        n = len(offs)
        o = np.ascontiguousarray(offs, dtype=np.uint64)
        ln = np.ascontiguousarray(lens, dtype=np.uint64)
        caps = np.ascontiguousarray([t.numel() for t in outs], dtype=np.uint64)
        ptrs = (ctypes.c_void_p * max(1, n))(*[t.data_ptr() for t in outs])
        u64p = ctypes.POINTER(ctypes.c_uint64)
        rc = _load().aceapex_decode_ranges(self._h, n, o.ctypes.data_as(u64p), ln.ctypes.data_as(u64p), ptrs,
                                           caps.ctypes.data_as(u64p), ctypes.c_void_p(work.data_ptr()),
                                           work.numel(), int(copy_mode), _stream_ptr(stream))
        _check(rc, "decode_ranges")

"""ctypes binding of the ORACLE (`axo.c`) — test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product never does.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

OK, E_ARG, E_CORRUPT, E_NOMEM, E_CHECKSUM = 0, -1, -2, -3, -4


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "block_size", "min_match", "no_rep", "depth_cap", "hash_bits", "chain_depth",
        "rans_min_syms_per_lane", "off_cost_q", "window_log")]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_bytes", "n_blocks", "comp_bytes", "n_commands", "n_lit_cmds", "n_matches", "n_rep",
        "n_escapes", "n_match_bytes", "n_lit_bytes", "n_forced_bytes")] + [
        ("max_depth", ctypes.c_uint32), ("passes", ctypes.c_uint32)]


class Cmd(ctypes.Structure):
    _fields_ = [("dst", ctypes.c_uint64), ("src", ctypes.c_uint64), ("len", ctypes.c_uint32),
                ("lit_pos", ctypes.c_uint32), ("kind", ctypes.c_uint8), ("rep", ctypes.c_uint8),
                ("pad", ctypes.c_uint8 * 6)]


CMD_DTYPE = np.dtype([("dst", "<u8"), ("src", "<u8"), ("len", "<u4"), ("lit_pos", "<u4"),
                      ("kind", "u1"), ("rep", "u1"), ("pad", "u1", 6)])


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_bytes", "n_blocks", "xxh3", "payload_bytes", "n_matches", "archive_bytes")] + [
        (n, ctypes.c_uint32) for n in ("block_size", "min_match", "flags", "depth_cap")]


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libaxo.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        u8p, u32p, u64p = P(ctypes.c_uint8), P(ctypes.c_uint32), P(ctypes.c_uint64)
        L.axo_params_default.argtypes = [P(Params)]
        L.axo_encode.argtypes = [u8p, ctypes.c_uint64, P(Params), P(u8p), u64p, P(Stats)]
        L.axo_encode_ex.argtypes = [u8p, ctypes.c_uint64, P(Params), P(u8p), u64p, P(Stats), u8p]
        L.axo_assemble.argtypes = [u8p, ctypes.c_uint64, P(Cmd), ctypes.c_uint64, P(Params), P(u8p), u64p]
        L.axo_free.argtypes = [ctypes.c_void_p]
        L.axo_read_info.argtypes = [u8p, ctypes.c_uint64, P(Info)]
        L.axo_decode.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
        L.axo_block_streams.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, u8p, u32p, u8p, u32p,
                                        ctypes.c_uint32, u8p, u32p, ctypes.c_uint32, u8p, u32p]
        L.axo_block_parse.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, P(Cmd), ctypes.c_uint64, u64p]
        L.axo_depths.argtypes = [u8p, ctypes.c_uint64, u32p, ctypes.c_uint64, u32p]
        L.axo_parse_all.argtypes = [u8p, ctypes.c_uint64, P(P(Cmd)), u64p]
        L.axo_block_levels.argtypes = [u8p, ctypes.c_uint64, u32p, u32p, u32p, u32p]
        L.axo_closure.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u8p, u64p]
        L.axo_stream_encode.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                        P(u8p), u32p]
        L.axo_stream_decode.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32, u32p, u32p]
        L.axo_leb_put.argtypes = [ctypes.c_uint64, u8p]
        L.axo_leb_put.restype = ctypes.c_uint32
        L.axo_leb_get.argtypes = [u8p, ctypes.c_uint32, u64p, u32p]
        L.axo_copy_serial.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.axo_copy_periodic.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        _lib = L
    return _lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _arr(x):
    a = np.ascontiguousarray(np.frombuffer(x, dtype=np.uint8) if isinstance(x, (bytes, bytearray)) else x,
                             dtype=np.uint8)
    return a


def params(**kw):
    p = Params()
    lib().axo_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, int(v))
    return p


def _take(ptr, n):
    out = np.ctypeslib.as_array(ptr, shape=(int(n),)).copy() if n else np.zeros(0, np.uint8)
    lib().axo_free(ptr)
    return out


def encode(data, **kw):
    """Encode bytes/uint8 array; returns (archive uint8 array, Stats)."""
    a = _arr(data)
    p = params(**kw)
    out = ctypes.POINTER(ctypes.c_uint8)()
    n = ctypes.c_uint64()
    st = Stats()
    rc = lib().axo_encode(_u8(a), a.size, ctypes.byref(p), ctypes.byref(out), ctypes.byref(n), ctypes.byref(st))
    if rc:
        raise OracleError(rc, "encode")
    return _take(out, n.value), st


def encode_forced(data, **kw):
    """Encode and also return the forced-literal mask of the depth cap."""
    a = _arr(data)
    p = params(**kw)
    out = ctypes.POINTER(ctypes.c_uint8)()
    n = ctypes.c_uint64()
    st = Stats()
    forced = np.zeros(max(1, a.size), np.uint8)
    rc = lib().axo_encode_ex(_u8(a), a.size, ctypes.byref(p), ctypes.byref(out), ctypes.byref(n),
                             ctypes.byref(st), _u8(forced))
    if rc:
        raise OracleError(rc, "encode")
    return _take(out, n.value), st, forced[: a.size]


def assemble(data, cmds, **kw):
    """Container from data + explicit commands: a list of (kind, dst, len, src,
    rep) tuples, or an array of CMD_DTYPE records in output order."""
    a = _arr(data)
    if isinstance(cmds, np.ndarray):
        arr = np.ascontiguousarray(cmds, dtype=CMD_DTYPE)
        ptr, count = arr.ctypes.data_as(ctypes.POINTER(Cmd)), arr.size
    else:
        arr = (Cmd * max(1, len(cmds)))()
        for i, (kind, dst, ln, src, rep) in enumerate(cmds):
            arr[i].kind, arr[i].dst, arr[i].len, arr[i].src, arr[i].rep = kind, dst, ln, src, rep
        ptr, count = arr, len(cmds)
    p = params(**kw)
    out = ctypes.POINTER(ctypes.c_uint8)()
    n = ctypes.c_uint64()
    rc = lib().axo_assemble(_u8(a), a.size, ptr, count, ctypes.byref(p), ctypes.byref(out), ctypes.byref(n))
    if rc:
        raise OracleError(rc, "assemble")
    return _take(out, n.value)


def info(arc):
    a = _arr(arc)
    inf = Info()
    rc = lib().axo_read_info(_u8(a), a.size, ctypes.byref(inf))
    if rc:
        raise OracleError(rc, "read_info")
    return inf


def decode(arc, copy_mode=0, verify=True, n_bytes=None):
    a = _arr(arc)
    n = info(a).n_bytes if n_bytes is None else n_bytes
    out = np.empty(max(1, int(n)), dtype=np.uint8)
    rc = lib().axo_decode(_u8(a), a.size, _u8(out), int(n), int(copy_mode), int(bool(verify)))
    if rc:
        raise OracleError(rc, "decode")
    return out[: int(n)]


def decode_rc(arc, copy_mode=0, verify=True):
    """Return code of a decode attempt (for corruption tests)."""
    a = _arr(arc)
    inf = Info()
    rc = lib().axo_read_info(_u8(a), a.size, ctypes.byref(inf))
    if rc:
        return rc
    if inf.n_bytes > (1 << 32):
        return E_ARG
    out = np.empty(max(1, int(inf.n_bytes)), dtype=np.uint8)
    return lib().axo_decode(_u8(a), a.size, _u8(out), int(inf.n_bytes), int(copy_mode), int(bool(verify)))


def block_streams(arc, block):
    a = _arr(arc)
    B = info(a).block_size
    bufs = [np.zeros(B, np.uint8), np.zeros(10 * B, np.uint8), np.zeros(10 * B, np.uint8), np.zeros(B, np.uint8)]
    ns = [ctypes.c_uint32() for _ in range(4)]
    rc = lib().axo_block_streams(_u8(a), a.size, block, _u8(bufs[0]), ctypes.byref(ns[0]), _u8(bufs[1]),
                                 ctypes.byref(ns[1]), 10 * B, _u8(bufs[2]), ctypes.byref(ns[2]), 10 * B,
                                 _u8(bufs[3]), ctypes.byref(ns[3]))
    if rc:
        raise OracleError(rc, "block_streams")
    return {k: bufs[i][: ns[i].value].copy() for i, k in enumerate(("lit", "len", "off", "cmd"))}


def block_parse(arc, block):
    a = _arr(arc)
    B = info(a).block_size
    out = np.zeros(B, dtype=CMD_DTYPE)
    n = ctypes.c_uint64()
    rc = lib().axo_block_parse(_u8(a), a.size, block, out.ctypes.data_as(ctypes.POINTER(Cmd)), B, ctypes.byref(n))
    if rc:
        raise OracleError(rc, "block_parse")
    return out[: n.value]


def parse_all(arc):
    """Every command of the archive in output order, as CMD_DTYPE records."""
    a = _arr(arc)
    ptr = ctypes.POINTER(Cmd)()
    n = ctypes.c_uint64()
    rc = lib().axo_parse_all(_u8(a), a.size, ctypes.byref(ptr), ctypes.byref(n))
    if rc:
        raise OracleError(rc, "parse_all")
    if not n.value:
        lib().axo_free(ptr)
        return np.zeros(0, CMD_DTYPE)
    raw = ctypes.cast(ptr, ctypes.POINTER(ctypes.c_uint8))
    out = np.ctypeslib.as_array(raw, shape=(n.value * CMD_DTYPE.itemsize,)).copy().view(CMD_DTYPE)
    lib().axo_free(ptr)
    return out


def depths(arc):
    a = _arr(arc)
    m = info(a).n_matches
    d = np.zeros(max(1, m), dtype=np.uint32)
    mx = ctypes.c_uint32()
    rc = lib().axo_depths(_u8(a), a.size, d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), m, ctypes.byref(mx))
    if rc:
        raise OracleError(rc, "depths")
    return d[:m], mx.value


def block_levels(arc, per_block=False):
    """Maxima of the raw and match-sourced block levels; with per_block=True
    also the level of every block: (raw_max, msrc_max, raw[], msrc[])."""
    a = _arr(arc)
    r, m = ctypes.c_uint32(), ctypes.c_uint32()
    nb = info(a).n_blocks
    raw = np.zeros(max(1, nb), np.uint32)
    msrc = np.zeros(max(1, nb), np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    rc = lib().axo_block_levels(_u8(a), a.size, ctypes.byref(r), ctypes.byref(m), raw.ctypes.data_as(u32p),
                                msrc.ctypes.data_as(u32p))
    if rc:
        raise OracleError(rc, "block_levels")
    if per_block:
        return r.value, m.value, raw[:nb], msrc[:nb]
    return r.value, m.value


def closure(arc, off, n):
    a = _arr(arc)
    nb = info(a).n_blocks
    mask = np.zeros(max(1, nb), dtype=np.uint8)
    k = ctypes.c_uint64()
    rc = lib().axo_closure(_u8(a), a.size, off, n, _u8(mask), ctypes.byref(k))
    if rc:
        raise OracleError(rc, "closure")
    return mask[:nb], k.value


def stream_encode(sym, min_syms_per_lane=128, force_rans=False, lanes_log2=-1):
    a = _arr(sym)
    out = ctypes.POINTER(ctypes.c_uint8)()
    n = ctypes.c_uint32()
    rc = lib().axo_stream_encode(_u8(a), a.size, min_syms_per_lane, int(force_rans), lanes_log2,
                                 ctypes.byref(out), ctypes.byref(n))
    if rc:
        raise OracleError(rc, "stream_encode")
    return _take(out, n.value)


def stream_decode(rec, cap):
    a = _arr(rec)
    out = np.zeros(max(1, cap), np.uint8)
    n, used = ctypes.c_uint32(), ctypes.c_uint32()
    rc = lib().axo_stream_decode(_u8(a), a.size, _u8(out), cap, ctypes.byref(n), ctypes.byref(used))
    return rc, out[: n.value].copy(), used.value


def leb_put(v):
    buf = (ctypes.c_uint8 * 10)()
    n = lib().axo_leb_put(v, buf)
    return bytes(buf[:n])


def leb_get(b):
    a = _arr(b)
    v, used = ctypes.c_uint64(), ctypes.c_uint32()
    rc = lib().axo_leb_get(_u8(a), a.size, ctypes.byref(v), ctypes.byref(used))
    return rc, v.value, used.value


def copy(buf, dst, src, ln, periodic):
    a = np.array(buf, dtype=np.uint8)
    (lib().axo_copy_periodic if periodic else lib().axo_copy_serial)(_u8(a), dst, src, ln)
    return a

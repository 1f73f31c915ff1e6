"""Seeded synthetic inputs (DNA, English-like text, batch plans, request traces).

Input generation only: none of the codec's arithmetic lives here, so the
oracle side and the product side may both use it.  The C generator
(`axsynth.c`) is built into `libaxsynth.so` next to this file.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libaxsynth.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.axs_dna.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64]
        lib.axs_text.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64]
        lib.axs_dna_segmented.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        lib.axs_batch_plan.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u64p, u8p]
        lib.axs_trace.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p, u64p]
        lib.axs_splitmix64.argtypes = [u64p]
        lib.axs_splitmix64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def dna(n, seed):
    """Synthetic DNA: n bytes over {A,C,G,T,a,c,g,t,N}."""
    out = np.empty(int(n), dtype=np.uint8)
    if _load().axs_dna(_u8(out), int(n), int(seed)) != 0:
        raise MemoryError("axs_dna")
    return out


def dna_segmented(n, seed, seg=256 << 20, threads=16):
    """Large synthetic DNA: independent segments of `seg` bytes, in parallel."""
    out = np.empty(int(n), dtype=np.uint8)
    if _load().axs_dna_segmented(_u8(out), int(n), int(seed), int(seg), int(threads)) != 0:
        raise MemoryError("axs_dna_segmented")
    return out


def text(n, seed):
    """Synthetic English-like text: n bytes."""
    out = np.empty(int(n), dtype=np.uint8)
    if _load().axs_text(_u8(out), int(n), int(seed)) != 0:
        raise MemoryError("axs_text")
    return out


def batch_plan(count, seed):
    """Sizes (bytes) and kinds (0 DNA, 1 text) of a batch of archives."""
    sizes = np.empty(int(count), dtype=np.uint64)
    kinds = np.empty(int(count), dtype=np.uint8)
    _load().axs_batch_plan(int(count), int(seed), _u64(sizes), _u8(kinds))
    return sizes, kinds


def trace(count, seed, n, block, rate, len_min, len_max):
    """Open-loop Poisson request trace: (arrival_ns, offset, length) arrays."""
    arr = np.empty(int(count), dtype=np.uint64)
    off = np.empty(int(count), dtype=np.uint64)
    ln = np.empty(int(count), dtype=np.uint64)
    _load().axs_trace(int(count), int(seed), int(n), int(block), float(rate), int(len_min), int(len_max),
                      _u64(arr), _u64(off), _u64(ln))
    return arr, off, ln


def splitmix64(state, count):
    """First `count` outputs of SplitMix64 from `state`."""
    st = ctypes.c_uint64(state)
    return [_load().axs_splitmix64(ctypes.byref(st)) for _ in range(count)]


# Workloads: (generator, n_bytes, seed)
CONFIGS = {
    1: ("dna", 4 * 1024 * 1024, 1),
    2: ("dna", 15500 * 16384, 2),
    3: ("text", 209715200, 3),
}


def config_input(k, n=None):
    kind, size, seed = CONFIGS[k]
    size = size if n is None else n
    return dna(size, seed) if kind == "dna" else text(size, seed)

"""Seeded synthetic inputs (DNA, English-like text, protein-like sequences,
FASTQ-like reads, batch plans, request traces).

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
        lib.axs_protein.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64]
        lib.axs_reads.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64]
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


def dna_segmented(n, seed, seg=256 << 20, threads=16, progress=None):
    """Multi-GiB synthetic DNA: consecutive segments of `seg` bytes, segment i
    an independent dna() stream seeded seed + i * 0x9E3779B97F4A7C15 (mod
    2^64), so planted copies source within their segment and a single
    segment equals dna(n, seed).  Segments are generated on `threads` threads;
    progress(bytes_done, n), if given, runs as segments finish."""
    import concurrent.futures as cf

    n = int(n)
    out = np.empty(n, dtype=np.uint8)
    lib = _load()

    def one(i):
        a = i * seg
        part = out[a: min(n, a + seg)]
        if lib.axs_dna(_u8(part), part.size, (int(seed) + i * 0x9E3779B97F4A7C15) & (2**64 - 1)) != 0:
            raise MemoryError("axs_dna")
        return part.size

    done = 0
    with cf.ThreadPoolExecutor(max_workers=max(1, int(threads))) as pool:
        for size in cf.as_completed([pool.submit(one, i) for i in range((n + seg - 1) // seg)]):
            done += size.result()
            if progress:
                progress(done, n)
    return out


def text(n, seed):
    """Synthetic English-like text: n bytes."""
    out = np.empty(int(n), dtype=np.uint8)
    if _load().axs_text(_u8(out), int(n), int(seed)) != 0:
        raise MemoryError("axs_text")
    return out


def protein(n, seed):
    """Synthetic protein-like sequences, one per line: n bytes."""
    out = np.empty(int(n), dtype=np.uint8)
    if _load().axs_protein(_u8(out), int(n), int(seed)) != 0:
        raise MemoryError("axs_protein")
    return out


def reads(n, seed):
    """Synthetic FASTQ-like 100-base reads of a synthetic genome: n bytes."""
    out = np.empty(int(n), dtype=np.uint8)
    if _load().axs_reads(_u8(out), int(n), int(seed)) != 0:
        raise MemoryError("axs_reads")
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


# Named workloads: (generator, n_bytes, seed)
WORKLOADS = {
    "dna4": ("dna", 4 * 1024 * 1024, 1),
    "dna254": ("dna", 15500 * 16384, 2),
    "text200": ("text", 209715200, 3),
    "protein254": ("protein", 15500 * 16384, 6),
    "reads254": ("reads", 15500 * 16384, 7),
}
GENERATORS = {"dna": dna, "text": text, "protein": protein, "reads": reads}


def workload_input(name, n=None):
    kind, size, seed = WORKLOADS[name]
    size = size if n is None else n
    return GENERATORS[kind](size, seed)

"""CPU checks of the product library: it loads, exports every symbol the C
header declares, and its host encoder writes exactly the oracle's container
for the same parameters (byte parity, so every later GPU parity case can use
either encoder's archive)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
import paper_2608_10188_amd as ax

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "aceapex.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aceapex_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ax.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(ax.EXPORTS) | set(names)


def _declared_arity():
    with open(os.path.join(ROOT, "include", "aceapex.h")) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(aceapex_\w+)\s*\(([^;{]*?)\)\s*;", text, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_argument_counts_match_header():
    """Every ctypes prototype has exactly the parameters the header declares."""
    lib = ax.lib()
    arity = _declared_arity()
    assert len(arity) >= 20
    for name, n in arity.items():
        fn = getattr(lib, name)
        assert fn.argtypes is not None, name
        assert len(fn.argtypes) == n, (name, len(fn.argtypes), n)


def test_strerror_and_params():
    lib = ax.lib()
    assert lib.aceapex_strerror(ax.AX_E_CORRUPT) == b"corrupt archive"
    p = ax.encode_params()
    assert (p.block_size, p.min_match, p.chain_depth, p.off_cost_q) == (16384, 4, 32, 6)


@pytest.mark.parametrize("kind", ["dna", "text"])
@pytest.mark.parametrize("kw", [{}, {"no_rep": 1}, {"min_match": 6}, {"block_size": 4096},
                                {"depth_cap": 2}, {"window_log": 16}, {"chain_depth": 4}])
def test_library_encoder_matches_oracle_bytes(kind, kw):
    x = synth.dna(700000, 31) if kind == "dna" else synth.text(700000, 32)
    want, _ = oracle.encode(x, **kw)
    for threads in (1, 3):
        got = ax.encode(x, threads=threads, **kw)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("kw", [{}, {"window_log": 20}])
def test_library_encoder_parallel_chains_match_oracle(kw):
    """Inputs above 4 Mi positions per thread build their hash chains in
    parallel parts stitched together; the archive must not change."""
    x = synth.dna(13 << 20, 33)
    want, _ = oracle.encode(x, **kw)
    assert np.array_equal(ax.encode(x, threads=3, **kw), want)


@pytest.mark.parametrize("x", [b"", b"z", b"abc" * 7000, bytes(range(256)) * 100])
def test_library_encoder_matches_oracle_edge(x):
    want, _ = oracle.encode(x)
    assert np.array_equal(ax.encode(x), want)


def test_library_read_info():
    x = synth.dna(100000, 33)
    arc = ax.encode(x)
    inf = ax.read_info(arc)
    o = oracle.info(arc)
    assert (inf.n_bytes, inf.n_blocks, inf.n_matches, inf.xxh3) == (o.n_bytes, o.n_blocks, o.n_matches, o.xxh3)
    assert inf.header_bytes == 64 + 16 * (inf.n_blocks + 1)
    with pytest.raises(ax.AceapexError):
        ax.read_info(np.zeros(64, np.uint8))


def test_encoder_rejects_bad_params():
    with pytest.raises(ax.AceapexError):
        ax.encode(b"abcd", block_size=3000)
    with pytest.raises(ax.AceapexError):
        ax.encode(b"abcd", min_match=0)

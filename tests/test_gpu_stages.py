"""Per-stage GPU parity, block by block, against the oracle.

Entropy stage: the four streams (LIT, LEN, OFF, CMD) the device decodes
from each block's rANS records (Setup) equal the oracle's block streams.
Parse stage: the matches the device parse emits (source, destination,
length; REP commands resolved through the distance history) equal the
oracle's block parse, block for block (the check the paper applies to its
prefix-sum parse in "The Last Sequential Element").  Literal placement and
the match layer are covered by the whole-decode cases.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2608_10188_amd as ax  # noqa: E402

pytestmark = pytest.mark.gpu
B = 16384


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _case(kind):
    if kind == "dna":
        arc, _ = oracle.encode(synth.dna(3 << 20, 31))
    elif kind == "text":
        arc, _ = oracle.encode(synth.text(2 << 20, 32))
    elif kind == "dna-no-rep":
        arc, _ = oracle.encode(synth.dna(1 << 20, 33), no_rep=1)
    elif kind == "text-min-match-6":
        arc, _ = oracle.encode(synth.text((1 << 20) + 333, 34), min_match=6)
    elif kind == "skewed-bytes":  # ~6.8 bits per literal: a full step takes ~28 words, the window moves every ~2 steps
        rng = np.random.default_rng(36)
        arc, _ = oracle.encode(np.minimum(rng.geometric(0.03, (1 << 20) + 4567) - 1, 255).astype(np.uint8))
    else:  # the full-size DNA workload from the library's encoder, sampled below
        arc = ax.encode(synth.dna(15500 * B, 2), threads=16)
    return arc


def _mpre(arc):
    nb = int(oracle.info(arc).n_blocks)
    return np.frombuffer(arc[64 + 8 * (nb + 1): 64 + 16 * (nb + 1)].tobytes(), "<u8")


def _blocks(arc, kind):
    nb = int(oracle.info(arc).n_blocks)
    if kind != "dna-full":
        return list(range(nb))
    rng = np.random.default_rng(35)
    return sorted(set([0, nb - 1] + rng.choice(nb, 48, replace=False).tolist()))


KINDS = ["dna", "text", "dna-no-rep", "text-min-match-6", "skewed-bytes", "dna-full"]


@pytest.mark.parametrize("kind", KINDS)
def test_entropy_stage_streams(kind):
    arc = _case(kind)
    d = ax.Decoder(arc, torch.from_numpy(arc).cuda())
    blocks = _blocks(arc, kind)
    _say("streams", kind, len(blocks), "blocks")
    if kind == "dna-full":
        got = {b: d.streams(b, 1)[0] for b in blocks}
    else:
        got = dict(enumerate(d.streams(0, len(blocks))))
        mid = len(blocks) // 2  # a run starting inside the archive
        for i, s in enumerate(d.streams(mid, 3)):
            for k in s:
                assert np.array_equal(s[k], got[mid + i][k]), (mid + i, k)
    for b in blocks:
        want = oracle.block_streams(arc, b)
        for k in ("lit", "len", "off", "cmd"):
            assert np.array_equal(got[b][k], want[k]), (kind, b, k)


@pytest.mark.parametrize("kind", KINDS)
def test_parse_stage_matches(kind):
    arc = _case(kind)
    d = ax.Decoder(arc, torch.from_numpy(arc).cuda())
    _say("parse", kind)
    d.build_index()
    mpre = _mpre(arc)
    n_rep = 0
    for b in _blocks(arc, kind):
        cmds = oracle.block_parse(arc, b)
        m = cmds[cmds["kind"] > 0]
        assert m.size == int(mpre[b + 1] - mpre[b]), b
        src, dst, ln = d.tokens(int(mpre[b]), m.size)
        assert np.array_equal(dst, m["dst"]), (kind, b)
        assert np.array_equal(src, m["src"]), (kind, b)
        assert np.array_equal(ln, m["len"]), (kind, b)
        n_rep += int((m["kind"] == 2).sum())
    if kind != "skewed-bytes":  # the skewed bytes hold (almost) no matches
        assert (n_rep == 0) == (kind == "dna-no-rep")

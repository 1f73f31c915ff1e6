"""Inputs of the served-read workload's shape, built from explicit commands.

Encoding several GiB with a match finder takes minutes, so the large parity
cases build their input and its command list together and let the oracle's
assembler write the container (the oracle's decode must then return the
input: the container is an input pinned by the oracle, not by this file).

Most blocks are constant: one literal byte, then a period-1 copy of it, as
a MATCH one byte back on even blocks and as REP slot 0 on odd ones (the
distance history starts at 1, 2, 3, 4 in every block).  Every `every`-th
block, plus the blocks beside each 2 GiB and 4 GiB boundary, carries DNA
literals and copies of four kinds: near (overlapping, periodic), from one of
the last sixteen content blocks (so blocks beyond 4 GiB copy from sources
beyond 4 GiB), from an earlier content block anywhere, from any earlier byte,
and REP of a history slot, with a REP of a distance above 2^31 following far
copies.  So the archive has 5-byte LEB128 offsets, sources and destinations
at or beyond 2^32, distances in the history above 2^32, sources in earlier
2 GiB windows, length escapes, and a ragged last block.
"""
import numpy as np

import oracle

ACGT = np.frombuffer(b"ACGT", np.uint8)


def content_blocks(nb, every, B):
    blocks = set(range(3, nb - 1, every))
    for edge in (1 << 31, 1 << 32):
        e = edge // B
        blocks.update(b for b in (e - 2, e - 1, e, e + 1) if 0 <= b < nb - 1)
    return np.array(sorted(blocks), np.int64)


def build(n, seed, B=16384, every=128, mm=4):
    """(input bytes, CMD_DTYPE commands in output order) for n bytes."""
    rng = np.random.default_rng(seed)
    nb = (n + B - 1) // B
    tail = n - (nb - 1) * B
    if tail < mm + 1:
        raise ValueError("the last block needs at least min_match + 1 bytes")
    vals = ((np.arange(nb, dtype=np.uint64) * 131 + 7) & 255).astype(np.uint8)
    x = np.empty(n, np.uint8)
    x[: (nb - 1) * B].reshape(nb - 1, B)[:] = vals[: nb - 1, None]
    x[(nb - 1) * B:] = vals[nb - 1]

    content = content_blocks(nb, every, B)
    is_content = np.zeros(nb, bool)
    is_content[content] = True

    # constant blocks: LIT 1, then a period-1 copy of the rest of the block
    cb = np.nonzero(~is_content)[0].astype(np.uint64)
    p0 = cb * B
    be = np.minimum(p0 + B, n)
    const = np.zeros(2 * cb.size, oracle.CMD_DTYPE)
    const["dst"][0::2] = p0
    const["len"][0::2] = 1
    const["kind"][0::2] = 0
    const["dst"][1::2] = p0 + 1
    const["len"][1::2] = (be - p0 - 1).astype(np.uint32)
    const["src"][1::2] = p0
    const["kind"][1::2] = np.where(cb % 2 == 0, 1, 2).astype(np.uint8)

    rows = []
    for i, b in enumerate(content):
        rows.extend(_content_block(x, rng, int(b), content[:i], B, n, mm))
    extra = np.zeros(len(rows), oracle.CMD_DTYPE)
    if rows:
        r = np.array(rows, np.uint64)
        extra["kind"], extra["dst"], extra["len"] = r[:, 0], r[:, 1], r[:, 2]
        extra["src"], extra["rep"] = r[:, 3], r[:, 4]
    cmds = np.concatenate([const, extra])
    cmds = cmds[np.argsort(cmds["dst"], kind="stable")]
    return x, cmds


def _length(rng, mm, room):
    u = rng.random()
    ln = rng.integers(mm, mm + 60) if u < 0.7 else rng.integers(64, 600) if u < 0.9 else rng.integers(600, 5000)
    return int(min(ln, room))


def _content_block(x, rng, b, earlier, B, n, mm):
    """Write block b's bytes into x and return its commands as
    (kind, dst, len, src, rep) rows."""
    p0 = b * B
    be = min(p0 + B, n)
    h = [1, 2, 3, 4]
    pos, rows, far = p0, [], False
    while pos < be:
        room = be - pos
        if pos == p0 or room < mm or rng.random() < 0.3:
            ln = int(min(room, rng.integers(1, 41) if rng.random() < 0.8 else rng.integers(41, 400)))
            x[pos: pos + ln] = ACGT[rng.integers(0, 4, ln)]
            rows.append((0, pos, ln, 0, 0))
            pos += ln
            continue
        ln = _length(rng, mm, room)
        u = rng.random()
        rep = -1
        if far and rng.random() < 0.6:
            rep = 0
        elif u < 0.3:
            src = pos - int(rng.integers(1, min(300, pos) + 1))
        elif u < 0.55 and earlier.size:
            c = int(earlier[-16:][rng.integers(0, min(16, earlier.size))])
            src = c * B + int(rng.integers(0, B))
        elif u < 0.7 and earlier.size:
            c = int(earlier[rng.integers(0, earlier.size)])
            src = c * B + int(rng.integers(0, B))
        elif u < 0.85:
            src = int(rng.integers(0, pos))
        else:
            rep = int(rng.integers(0, 4))
        if rep >= 0 and h[rep] > pos:
            rep, src = -1, pos - 1
        if rep >= 0:
            d = h[rep]
            src = pos - d
            h = [d] + h[:rep] + h[rep + 1:]
            rows.append((2, pos, ln, src, rep))
        else:
            d = pos - src
            h = [d] + h[:3]
            rows.append((1, pos, ln, src, 0))
        if d >= ln:
            x[pos: pos + ln] = x[src: src + ln]
        else:
            x[pos: pos + ln] = np.resize(x[src:pos], ln)  # periodic: the copy reads its own output
        far = d > (1 << 31)
        pos += ln
    return rows

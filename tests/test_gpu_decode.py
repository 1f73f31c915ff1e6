"""GPU parity: the HIP decoder (through the C ABI) against the oracle.

Every case decodes an oracle-encoded archive on the device into an output
buffer poisoned with 0xCC (so a byte the decoder never writes shows up), and
compares every byte with the oracle's sequential decode and with the
original input.  Case names are printed and flushed before each launch.
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


def gpu_decode(arc, copy_mode=ax.COPY_PERIODIC, repeats=1):
    arc = np.ascontiguousarray(arc, dtype=np.uint8)
    d_arc = torch.from_numpy(arc).cuda()
    dec = ax.Decoder(arc, d_arc)
    n = int(dec.info.n_bytes)
    outs = []
    out = torch.empty((max(16, n),), dtype=torch.uint8, device="cuda")
    for _ in range(repeats):
        out.fill_(0xCC)
        dec.decode_all(out=out, copy_mode=copy_mode)
        err, bad = dec.status()
        outs.append((err, bad, out[:n].cpu().numpy()))
    return outs if repeats > 1 else outs[0]


def check(name, x, arc, modes=(ax.COPY_PERIODIC, ax.COPY_SERIAL)):
    """Every mode decodes three times with one decoder (the first decode
    teaches the decoder its bulk-round and jump-pass counts; the later ones
    run what it learned); every output must equal the oracle's decode."""
    x = np.frombuffer(bytes(x), np.uint8) if isinstance(x, (bytes, bytearray)) else x
    ref = oracle.decode(arc)
    assert np.array_equal(ref, x), f"{name}: oracle round trip failed"
    for m in modes:
        _say(name, "copy_mode", m, "n", x.size)
        for k, (err, bad, got) in enumerate(gpu_decode(arc, m, repeats=3)):
            assert err == 0, f"{name}: decode {k}: device status {err} at block {bad}"
            if not np.array_equal(got, ref):
                i = int(np.nonzero(got != ref)[0][0])
                raise AssertionError(f"{name} mode {m} decode {k}: first mismatch at byte {i} (block {i // B}) "
                                     f"got {got[i]} want {ref[i]}")


@pytest.mark.parametrize("kind", ["dna", "text"])
def test_config1_shape(kind):
    x = synth.dna(4 << 20, 1) if kind == "dna" else synth.text(4 << 20, 3)
    arc, _ = oracle.encode(x)
    check(f"config1-{kind}", x, arc)


@pytest.mark.parametrize("kind", ["dna", "text"])
def test_full_size_workloads(kind):
    """The benchmark's workloads at full size (253,952,000 B DNA seed 2 and
    209,715,200 B text seed 3) in the launch configuration it times (default
    options), every byte against the oracle's decode, in both copy modes.
    The archive comes from the library's host encoder (the oracle encoder
    would take minutes at this size); the oracle's decode of it must equal
    the input first, so the archive is an input pinned by the oracle."""
    if kind == "dna":
        x = synth.dna(15500 * B, 2)
    else:
        x = synth.text(209715200, 3)
    arc = ax.encode(x, threads=16)
    check(f"full-{kind}", x, arc)


def test_no_rep_encoding():
    x = synth.dna(2 << 20, 7)
    arc, st = oracle.encode(x, no_rep=1)
    assert st.n_rep == 0
    check("no_rep", x, arc)


@pytest.mark.parametrize("kind", ["protein", "reads"])
def test_second_workload_family(kind):
    """Protein-like sequences and FASTQ-like reads, at the small shape (4 MiB,
    oracle encoder, both copy modes) and at full size (253,952,000 B, the
    library's encoder, default launch configuration)."""
    x = synth.GENERATORS[kind](4 << 20, 21)
    arc, _ = oracle.encode(x)
    check(f"{kind}-4m", x, arc)
    x = synth.workload_input(f"{kind}254")
    arc = ax.encode(x, threads=16)
    check(f"{kind}-full", x, arc, modes=(ax.COPY_PERIODIC,))


def test_full_size_no_rep_dna():
    """The history-free encoding (no REP commands: every match carries its
    offset) of the full-size DNA workload (253,952,000 B, seed 2), in the
    benchmark's launch configuration."""
    x = synth.dna(15500 * B, 2)
    arc = ax.encode(x, threads=16, no_rep=1)
    assert ax.read_info(arc).flags & 1
    check("full-dna-no-rep", x, arc, modes=(ax.COPY_PERIODIC,))


@pytest.mark.parametrize("window_log", [16, 22])
def test_window_limited_encoder(window_log):
    """Archives of the window-limited match finder (sources at most
    2^window_log bytes back), the encoder setting the served workload uses."""
    x = synth.dna(48 << 20, 9)
    arc = ax.encode(x, threads=16, window_log=window_log)
    check(f"window-log-{window_log}", x, arc, modes=(ax.COPY_PERIODIC,))


@pytest.mark.parametrize("n", [0, 1, 17, 4095, 4096, 4097, B - 1, B, B + 1, 3 * B + 5])
def test_edge_sizes(n):
    x = synth.dna(n, 40 + n)
    arc, _ = oracle.encode(x)
    check(f"edge-{n}", x, arc, modes=(ax.COPY_PERIODIC,))


@pytest.mark.parametrize("bs", [4096, 8192])
def test_small_blocks(bs):
    x = synth.text(600000, 41)
    arc, _ = oracle.encode(x, block_size=bs)
    check(f"block{bs}", x, arc)


def test_structured_inputs():
    rng = np.random.default_rng(5)
    cases = {
        "all_equal": np.full(200000, 78, np.uint8),
        "random_binary": rng.integers(0, 256, 150000, dtype=np.uint8),
        "low_entropy": rng.choice(np.frombuffer(b"ab", np.uint8), 150000, p=[0.97, 0.03]),
    }
    for period in (1, 2, 3, 7, 64, 153):
        unit = rng.integers(0, 256, period, dtype=np.uint8)
        cases[f"tandem{period}"] = np.tile(unit, 120000 // period + 1)[:120000]
    for name, x in cases.items():
        arc, _ = oracle.encode(x)
        check(name, x, arc)


def test_depth_capped_archive():
    x = synth.text(1 << 20, 42)
    arc, st = oracle.encode(x, depth_cap=2)
    assert st.max_depth <= 2
    check("depth_cap2", x, arc)


@pytest.mark.parametrize("kind,cap", [("text", 16), ("dna", 16)])
def test_full_size_depth_capped(kind, cap):
    """The full-size text and DNA workloads encoded under a depth cap (the
    library's encoder iterates forced literals until no match is deeper than
    the cap): the decode of the capped archive equals the input."""
    x = synth.text(209715200, 3) if kind == "text" else synth.dna(15500 * B, 2)
    arc, st = ax.encode(x, stats=True, threads=16, depth_cap=cap)
    assert st.max_depth <= cap
    check(f"full-{kind}-cap{cap}", x, arc, modes=(ax.COPY_PERIODIC,))


# ---------------------------------------------------------- assembled cases --

def _assemble_check(name, data, cmds, **kw):
    arc = oracle.assemble(data, cmds, **kw)
    check(name, data, arc)


def test_many_single_literal_commands():
    """16384 one-byte literal commands in one block: 64 parse chunks."""
    rng = np.random.default_rng(1)
    data = rng.integers(0, 256, 2 * B, dtype=np.uint8)
    cmds = [(0, i, 1, 0, 0) for i in range(2 * B)]
    _assemble_check("lit1x32768", data, cmds)


def test_dense_min_matches_and_reps():
    """Alternating 1-byte literals and 4-byte matches/repeats: thousands of
    tokens per block, every repeat slot, escapes absent."""
    rng = np.random.default_rng(2)
    n = 3 * B
    data = np.zeros(n, np.uint8)
    cmds = []
    pos = 0
    hist = [1, 2, 3, 4]
    while pos < n:
        bstart = pos // B * B
        if pos == bstart:
            hist = [1, 2, 3, 4]
        room = bstart + B - pos
        if room < 5 or pos < 64:
            data[pos] = rng.integers(0, 256)
            cmds.append((0, pos, 1, 0, 0))
            pos += 1
            continue
        data[pos] = rng.integers(0, 256)
        cmds.append((0, pos, 1, 0, 0))
        pos += 1
        if rng.random() < 0.5:
            r = int(rng.integers(0, 4))
            d = hist[r]
            if d <= pos:
                for k in range(4):
                    data[pos + k] = data[pos - d + k]
                cmds.append((2, pos, 4, pos - d, r))
                hist = [d] + hist[:r] + hist[r + 1:]
                pos += 4
                continue
        src = int(rng.integers(max(0, pos - 3000), pos))
        for k in range(4):
            data[pos + k] = data[src + k]
        cmds.append((1, pos, 4, src, 0))
        hist = [pos - src] + hist[:3]
        pos += 4
    _assemble_check("dense_min_matches", data, cmds)


def test_long_escapes_and_block_spanning_fill():
    """A block-long literal (2-byte LEB128 length), a block-long period-1
    repeat and a block-long period-5 match."""
    rng = np.random.default_rng(3)
    data = np.zeros(4 * B, np.uint8)
    data[:B] = rng.integers(0, 256, B)
    data[B:2 * B] = data[B - 1]
    cmds = [(0, 0, B, 0, 0), (2, B, B, 2 * B - 1 - B, 0)]  # REP slot 0 = dist 1
    data[2 * B: 2 * B + 5] = rng.integers(0, 256, 5)
    cmds.append((0, 2 * B, 5, 0, 0))
    for k in range(2 * B + 5, 3 * B):
        data[k] = data[k - 5]
    cmds.append((1, 2 * B + 5, B - 5, 2 * B, 0))
    for k in range(3 * B, 4 * B):  # copy of the first block from far back
        data[k] = data[k - 3 * B]
    cmds.append((1, 3 * B, B, 0, 0))
    _assemble_check("long_escapes", data, cmds)


def test_deep_cross_block_chain():
    """Each block copies a span written by a match of the previous block, so
    the chain depth equals the number of blocks."""
    rng = np.random.default_rng(4)
    nb = 40
    data = np.zeros(nb * B, np.uint8)
    data[:B] = rng.integers(0, 256, B)
    cmds = [(0, 0, B, 0, 0)]
    for b in range(1, nb):
        s = b * B
        # literal head, then a 500-byte match reading the previous block's match
        data[s:s + 100] = rng.integers(0, 256, 100)
        cmds.append((0, s, 100, 0, 0))
        src = s - B + 100 if b > 1 else 0
        data[s + 100:s + 600] = data[src:src + 500]
        cmds.append((1, s + 100, 500, src, 0))
        data[s + 600:s + B] = rng.integers(0, 256, B - 600)
        cmds.append((0, s + 600, B - 600, 0, 0))
    arc = oracle.assemble(data, cmds)
    d, mx = oracle.depths(arc)
    assert mx == nb - 2
    check("deep_chain", data, arc)


@pytest.mark.parametrize("rounds", [0, 2, 4])
def test_deep_chain_of_long_periodic_fills(rounds):
    """Long self-overlapping matches deep in a cross-block chain.  Block b
    holds a 300-byte match of block b-1's (chain depth b) and then a periodic
    fill of 2000+ bytes over its own last p bytes, so with two or four bulk
    rounds the deep ones reach the remainder as long pending tokens (marked
    with their bytes 256 apart over a workgroup's lanes).  Periods below,
    equal to and above 256 and unaligned destinations exercise the wrap of
    the source index and the leftover-map words a wave's 64 bytes meet.
    rounds 0: the learned count."""
    rng = np.random.default_rng(5)
    nb = 24
    periods = [1, 3, 7, 64, 100, 255, 256, 257, 300, 511, 1000]
    data = np.zeros(nb * B, np.uint8)
    data[:B] = rng.integers(0, 256, B)
    cmds = [(0, 0, B, 0, 0)]
    prev = 0  # the previous block's chained match (block 0: literal bytes)
    for b in range(1, nb):
        s = b * B
        h = 5 + 3 * b
        data[s:s + h] = rng.integers(0, 256, h)
        cmds.append((0, s, h, 0, 0))
        a = s + h
        data[a:a + 300] = data[prev:prev + 300]
        cmds.append((1, a, 300, prev, 0))
        p, f, ln = periods[b % len(periods)], a + 300, 2000 + 37 * b
        data[f:f + ln] = np.resize(data[f - p:f], ln)
        cmds.append((1, f, ln, f - p, 0))
        t = f + ln
        data[t:s + B] = rng.integers(0, 256, s + B - t)
        cmds.append((0, t, s + B - t, 0, 0))
        prev = a
    arc = oracle.assemble(data, cmds)
    ref = oracle.decode(arc)
    assert np.array_equal(ref, data)
    dec = ax.Decoder(arc, torch.from_numpy(arc).cuda())
    if rounds:
        dec.set_option(ax.OPT_BULK_ROUNDS, rounds)
    out = torch.empty((data.size,), dtype=torch.uint8, device="cuda")
    for k in range(3):
        out.fill_(0xCC)
        _say("long periodic chain: bulk rounds", rounds, "decode", k)
        dec.decode_all(out=out)
        err, bad = dec.status()
        assert err == 0, (err, bad)
        got = out.cpu().numpy()
        if not np.array_equal(got, ref):
            i = int(np.nonzero(got != ref)[0][0])
            raise AssertionError(f"decode {k}: first mismatch at byte {i} (block {i // B})")


# -------------------------------------------------------------- behaviour --

@pytest.mark.parametrize("opts", [
    {ax.OPT_BULK_ROUNDS: 1}, {ax.OPT_BULK_ROUNDS: 2, ax.OPT_TAIL_CHUNKS: 4, ax.OPT_TAIL_MODE: 1},
    {ax.OPT_BULK_ROUNDS: 8, ax.OPT_FILL_ROUNDS: 0, ax.OPT_FILL_TAIL: 1, ax.OPT_TAIL_MODE: 1},
    {ax.OPT_BULK_ROUNDS: 3, ax.OPT_FILL_TAIL: 1, ax.OPT_TAIL_CHUNKS: 16, ax.OPT_TAIL_MODE: 1},
    {ax.OPT_ROUND0_TILE: 0}, {ax.OPT_ROUND0_TILE: 0, ax.OPT_FILL_ROUNDS: 1, ax.OPT_BULK_ROUNDS: 1},
    {ax.OPT_TAIL_MODE: 1}, {ax.OPT_BULK_ROUNDS: 1, ax.OPT_JUMP_PASSES: 1},
    {ax.OPT_BULK_ROUNDS: 2, ax.OPT_JUMP_PASSES: 3}, {ax.OPT_BULK_ROUNDS: 6}])
def test_schedule_options_change_no_byte(opts):
    """Every schedule knob (rounds, fill modes, tickets per chunk run, round-0
    schedule, deep-remainder mode, jump pass limit: with one or three passes
    the gather follows the remaining chains itself) decodes a deep text
    archive and a DNA archive to the oracle's bytes."""
    for name, x in (("text", synth.text(3 << 20, 46)), ("dna", synth.dna(3 << 20, 47))):
        arc, _ = oracle.encode(x)
        dec = ax.Decoder(arc, torch.from_numpy(arc).cuda())
        for k, v in opts.items():
            dec.set_option(k, v)
        out = torch.full((x.size,), 0xCC, dtype=torch.uint8, device="cuda")
        _say("options", name, opts)
        dec.decode_all(out=out)
        err, bad = dec.status()
        assert err == 0, (err, bad)
        assert np.array_equal(out.cpu().numpy(), x), (name, opts)

def test_repeat_decode_is_deterministic():
    x = synth.text(2 << 20, 43)
    arc, _ = oracle.encode(x)
    _say("determinism")
    runs = gpu_decode(arc, repeats=4)
    for err, bad, got in runs:
        assert err == 0 and np.array_equal(got, x)


def test_corrupt_archives_report_errors_without_hanging():
    x = synth.dna(300000, 44)
    arc, _ = oracle.encode(x)
    inf = oracle.info(arc)
    hdr = 64 + 16 * (inf.n_blocks + 1)
    rng = np.random.default_rng(8)
    detected = 0
    for trial in range(24):
        bad = arc.copy()
        for _ in range(3):
            i = int(rng.integers(hdr, arc.size))
            bad[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
        _say("corrupt", trial)
        err, blk, got = gpu_decode(bad)
        assert err in (0, ax.AX_E_CORRUPT), err
        if err == 0:
            orc = oracle.decode_rc(bad, verify=False)
            # a flip the format cannot see (a raw byte, a symbol) decodes like the oracle
            if orc == 0:
                assert np.array_equal(got, oracle.decode(bad, verify=False))
        detected += err != 0
    assert detected >= 12


def test_forward_offset_is_rejected_on_device():
    """A match whose offset is not behind its position must fail in the
    parse, before anything waits on it."""
    data = np.frombuffer(b"abcdefgh" * 512, np.uint8).copy()
    arc = oracle.assemble(data, [(0, 0, 8, 0, 0), (1, 8, 4088, 0, 0)])
    # rewrite the single OFF value (LEB128 0) to point at the match itself:
    # find the OFF record (third stream) of block 0 and patch its byte
    inf = oracle.info(arc)
    base = 64 + 16 * (inf.n_blocks + 1)
    sizes = [int.from_bytes(bytes(arc[base + 4 * k: base + 4 * k + 4]), "little") for k in range(4)]
    off_rec = base + 16 + sizes[0] + sizes[1]
    assert arc[off_rec + 4] == 1 and arc[off_rec] == 1  # CONST record of one byte: LEB128(0)
    bad = arc.copy()
    bad[off_rec + 5] = 8  # src = 8 == dst
    assert oracle.decode_rc(bad, verify=False) == oracle.E_CORRUPT
    _say("forward_offset")
    err, blk, _ = gpu_decode(bad)
    assert err == ax.AX_E_CORRUPT and blk == 0


def test_stage_timing_runs():
    x = synth.dna(4 << 20, 1)
    arc, _ = oracle.encode(x)
    d_arc = torch.from_numpy(arc).cuda()
    dec = ax.Decoder(arc, d_arc)
    dec.set_timing(True)
    _say("stage_timing")
    out = dec.decode_all()
    a, p, c = dec.stage_ms()
    assert a > 0 and p > 0 and c >= 0
    assert np.array_equal(out.cpu().numpy(), x)

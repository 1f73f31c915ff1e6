"""GPU parity of the batched decoder: many archives of uneven sizes and both
generators in one plan, every output byte compared with the oracle; the
captured-graph replay must give the same bytes on every replay."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2608_10188_amd as ax  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _archives(count, seed, max_size=300000):
    sizes, kinds = synth.batch_plan(count, seed)
    rng = np.random.default_rng(seed)
    xs, arcs = [], []
    for i in range(count):
        n = int(min(int(sizes[i]) // 64, max_size)) + int(rng.integers(0, 5000))
        x = synth.dna(n, 1000 + i) if kinds[i] == 0 else synth.text(n, 1000 + i)
        arc, _ = oracle.encode(x, block_size=16384)
        xs.append(x)
        arcs.append(arc)
    return xs, arcs


def _run_batch(arcs, graph=False, repeats=1, window_probe=False):
    decs, outs = [], []
    for arc in arcs:
        d = ax.Decoder(arc, torch.from_numpy(arc).cuda())
        decs.append(d)
        outs.append(torch.full((max(16, int(d.info.n_bytes)),), 0xCC, dtype=torch.uint8, device="cuda"))
    bt = ax.Batch(decs, outs)
    if graph:
        bt.set_option(ax.OPT_GRAPH, 1)
    results = []
    for r in range(repeats):
        for o in outs:
            o.fill_(0xCC)
        torch.cuda.synchronize()
        bt.decode()
        err, bad = bt.status()
        results.append((err, [o[: int(d.info.n_bytes)].cpu().numpy() for d, o in zip(decs, outs)]))
    return results


def test_batch_matches_oracle():
    xs, arcs = _archives(48, 4)
    _say("batch48")
    (err, got), = _run_batch(arcs)
    assert err == 0
    for i, (x, arc, g) in enumerate(zip(xs, arcs, got)):
        ref = oracle.decode(arc)
        assert np.array_equal(ref, x)
        assert np.array_equal(g, ref), f"archive {i}"


def test_batch_graph_replays_identically():
    xs, arcs = _archives(24, 5)
    _say("batch24 graph")
    runs = _run_batch(arcs, graph=True, repeats=3)
    for err, got in runs:
        assert err == 0
        for x, g in zip(xs, got):
            assert np.array_equal(g, x)


def test_batch_with_empty_and_tiny_archives():
    xs = [np.zeros(0, np.uint8), np.frombuffer(b"a", np.uint8), synth.dna(5000, 9), synth.text(70000, 10),
          np.zeros(0, np.uint8)]
    arcs = [oracle.encode(x)[0] for x in xs]
    _say("batch empty/tiny")
    (err, got), = _run_batch(arcs)
    assert err == 0
    for x, g in zip(xs, got):
        assert np.array_equal(g, x)


def test_full_size_batch_sampled():
    """The benchmark's batch at full size (4096 archives, 64 KiB-64 MiB,
    60 % DNA / 40 % text, plan seed 4, archive i seeded 1000 + i), one plan
    as timed: every archive against the XXH3 of its input, 64 archives drawn
    at random byte by byte against the oracle's decode.  Archives come from
    the library's host encoder; each sampled one is pinned by the oracle's
    decode equalling its input."""
    import concurrent.futures as cf

    xxhash = pytest.importorskip("xxhash")
    sizes, kinds = synth.batch_plan(4096, 4)

    def make(i):
        x = synth.dna(int(sizes[i]), 1000 + i) if kinds[i] == 0 else synth.text(int(sizes[i]), 1000 + i)
        return ax.encode(x, threads=1), xxhash.xxh3_64_intdigest(x.tobytes()), x.size

    with cf.ThreadPoolExecutor(max_workers=16) as pool:
        made = list(pool.map(make, range(4096)))
    decs, outs = [], []
    for arc, _, n in made:
        decs.append(ax.Decoder(arc, torch.from_numpy(arc).cuda()))
        outs.append(torch.full((max(16, n),), 0xCC, dtype=torch.uint8, device="cuda"))
    bt = ax.Batch(decs, outs)
    _say("batch4096 full size")
    bt.decode()
    err, bad = bt.status()
    assert err == 0, f"device status {err} at block {bad}"
    sample = set(np.random.default_rng(4).choice(4096, 64, replace=False).tolist())
    for i, ((arc, h, n), o) in enumerate(zip(made, outs)):
        got = o[:n].cpu().numpy()
        assert xxhash.xxh3_64_intdigest(got.tobytes()) == h, f"archive {i}"
        if i in sample:
            ref = oracle.decode(arc)
            assert xxhash.xxh3_64_intdigest(ref.tobytes()) == h, f"archive {i}: oracle"
            assert np.array_equal(got, ref), f"archive {i}"

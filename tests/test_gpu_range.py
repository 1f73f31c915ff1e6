"""GPU parity of random access: the library's byte-precise source closure
against the oracle's, range decodes (into a compact scratch sized by the
closure) against the original bytes, capacity errors returned before any
launch, and the serving loop's results alone and in the mix."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2608_10188_amd as ax  # noqa: E402
from paper_2608_10188_amd.serve import Server  # noqa: E402

pytestmark = pytest.mark.gpu
B = 16384


def _say(*a):
    print("[gpu case]", *a, flush=True)


@pytest.fixture(scope="module")
def dna_archive():
    x = synth.dna(6 << 20, 61)
    arc, _ = oracle.encode(x)
    return x, arc


def _decoder_with_index(arc):
    d = ax.Decoder(arc, torch.from_numpy(arc).cuda())
    d.build_index()
    return d


def _ranges(n_bytes, count, seed):
    rng = np.random.default_rng(seed)
    out = [(0, 1), (n_bytes - 1, 1), (0, n_bytes), (B - 3, 6), (5 * B, B), (7 * B - 1, 2 * B + 2)]
    while len(out) < count:
        ln = int(min(n_bytes, np.exp(rng.uniform(0, np.log(600000)))))
        off = int(rng.integers(0, n_bytes - ln + 1))
        out.append((off, ln))
    return out


@pytest.mark.parametrize("kind", ["dna", "text"])
def test_closure_matches_oracle(kind, dna_archive):
    if kind == "dna":
        x, arc = dna_archive
    else:
        x = synth.text(3 << 20, 62)
        arc, _ = oracle.encode(x)
    _say("closure", kind)
    d = _decoder_with_index(arc)
    rs = _ranges(x.size, 40, 7)
    sizes, _ = d.closure_sizes([r[0] for r in rs], [r[1] for r in rs])
    for (off, ln), size in zip(rs, sizes):
        mask, k = oracle.closure(arc, off, ln)
        blocks, ntok, nb = d.closure_blocks([off], [ln])
        assert nb == k and np.array_equal(np.nonzero(mask)[0].astype(np.uint64), blocks), (off, ln)
        assert size == k, (off, ln)


def test_union_closure_is_union(dna_archive):
    x, arc = dna_archive
    d = _decoder_with_index(arc)
    rs = _ranges(x.size, 12, 8)
    union = set()
    for off, ln in rs:
        union |= set(np.nonzero(oracle.closure(arc, off, ln)[0])[0].tolist())
    blocks, _, _ = d.closure_blocks([r[0] for r in rs], [r[1] for r in rs], threads=4)
    assert sorted(union) == blocks.tolist()


def test_decode_ranges_match_original(dna_archive):
    x, arc = dna_archive
    d = _decoder_with_index(arc)
    rp = ax.RangePlan(d, max_blocks=512, max_tokens=1 << 18)
    work = torch.empty(rp.workspace_bytes, dtype=torch.uint8, device="cuda")
    # the scratch is sized by the closure limits, not by the archive
    assert rp.workspace_bytes < 600 * B * 160
    rs = _ranges(x.size, 30, 9)
    rs = [r for r in rs if r[1] <= 64 * B]
    for batch in (rs[:1], rs[:7], rs):
        _say("decode_ranges", len(batch))
        outs = [torch.full((max(1, ln),), 0xCC, dtype=torch.uint8, device="cuda") for _, ln in batch]
        work.fill_(0xCC)  # stale scratch and slot-table contents must not matter
        rp.decode([r[0] for r in batch], [r[1] for r in batch], outs, work)
        err, bad = ax.workspace_status(work)
        assert err == 0, (err, bad)
        for (off, ln), o in zip(batch, outs):
            assert np.array_equal(o[:ln].cpu().numpy(), x[off:off + ln]), (off, ln)


def test_decode_ranges_into_unaligned_views(dna_archive):
    """Outputs that are views of one buffer at odd offsets (as a server packs
    them), ranges of 1 B to several 4 KiB gather chunks."""
    x, arc = dna_archive
    d = _decoder_with_index(arc)
    rp = ax.RangePlan(d, max_blocks=512, max_tokens=1 << 18)
    work = torch.empty(rp.workspace_bytes, dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(12)
    lens = [1, 3, 4095, 4096, 4097, 12289, 70001, 16384, 5, 200000]
    offs = [int(rng.integers(0, x.size - ln)) for ln in lens]
    _say("unaligned views", len(lens))
    buf = torch.full((sum(lens) + 7,), 0xCC, dtype=torch.uint8, device="cuda")
    outs = list(torch.split(buf[7:], lens))
    rp.decode(offs, lens, outs, work)
    got = buf.cpu().numpy()
    assert (got[:7] == 0xCC).all()
    at = 7
    for off, ln in zip(offs, lens):
        assert np.array_equal(got[at: at + ln], x[off: off + ln]), (off, ln)
        at += ln


def test_block_straddling_sweep(dna_archive):
    x, arc = dna_archive
    d = _decoder_with_index(arc)
    rp = ax.RangePlan(d, max_blocks=512, max_tokens=1 << 18)
    work = torch.empty(rp.workspace_bytes, dtype=torch.uint8, device="cuda")
    rs = [(b * B - k, 2 * k) for b in range(1, x.size // B) for k in (1, 7, 300)]
    _say("straddle", len(rs))
    outs = [torch.empty(ln, dtype=torch.uint8, device="cuda") for _, ln in rs]
    for i in range(0, len(rs), 64):
        rp.decode([r[0] for r in rs[i:i + 64]], [r[1] for r in rs[i:i + 64]], outs[i:i + 64], work)
    torch.cuda.synchronize()
    for (off, ln), o in zip(rs, outs):
        assert np.array_equal(o.cpu().numpy(), x[off:off + ln])


def test_capacity_errors_before_any_launch(dna_archive):
    """A closure above the plan's limits, an output shorter than its range
    and a short workspace are all refused with AX_E_CAPACITY before anything
    is enqueued (the output keeps its poison)."""
    x, arc = dna_archive
    d = _decoder_with_index(arc)
    rp = ax.RangePlan(d, max_blocks=2, max_tokens=1 << 16)
    work = torch.empty(rp.workspace_bytes, dtype=torch.uint8, device="cuda")
    out = torch.full((10 * B,), 0xCC, dtype=torch.uint8, device="cuda")
    _say("capacity: closure")
    with pytest.raises(ax.AceapexError) as ei:
        rp.decode([0], [10 * B], [out], work)
    assert ei.value.code == ax.AX_E_CAPACITY
    rp2 = ax.RangePlan(d, max_blocks=512, max_tokens=1 << 18)
    work2 = torch.empty(rp2.workspace_bytes, dtype=torch.uint8, device="cuda")
    _say("capacity: short output")
    with pytest.raises(ax.AceapexError) as ei:
        rp2.decode([5 * B], [B], [out[: B - 1]], work2)
    assert ei.value.code == ax.AX_E_CAPACITY
    _say("capacity: short workspace")
    with pytest.raises(ax.AceapexError) as ei:
        rp2.decode([5 * B], [B], [out], work2[: rp2.workspace_bytes - 256])
    assert ei.value.code == ax.AX_E_CAPACITY
    need = d.range_workspace(5 * B, B)
    with pytest.raises(ax.AceapexError) as ei:
        d.decode_range(5 * B, B, out, torch.empty(need - 256, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == ax.AX_E_CAPACITY
    with pytest.raises(ax.AceapexError) as ei:
        d.decode_range(5 * B, B, out[: B - 1], torch.empty(need, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == ax.AX_E_CAPACITY
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0xCC).all()


def test_decode_range_with_its_own_workspace(dna_archive):
    """aceapex_decode_range with exactly aceapex_range_workspace bytes, for
    ranges from one byte to several blocks: every byte equals the input, and
    the workspace is sized by the closure (far below the archive)."""
    x, arc = dna_archive
    d = _decoder_with_index(arc)
    for off, ln in _ranges(x.size, 16, 13):
        if ln > 40 * B:
            continue
        need = d.range_workspace(off, ln)
        blocks, _, nb = d.closure_blocks([off], [ln])
        assert need < (nb + 1) * B + 4 * d.info.n_blocks + nb * 140 * 1024 + (1 << 20)
        work = torch.full((need,), 0xCC, dtype=torch.uint8, device="cuda")
        out = torch.full((max(1, ln),), 0xCC, dtype=torch.uint8, device="cuda")
        _say("decode_range", off, ln, need)
        d.decode_range(off, ln, out, work)
        assert np.array_equal(out[:ln].cpu().numpy(), x[off:off + ln]), (off, ln)


def test_serving_results_same_alone_and_in_mix(dna_archive):
    """Continuous batching changes no byte: every request's result is the
    same decoded alone (one batch each) and in a Poisson mix."""
    x, arc = dna_archive
    srv = Server(arc, torch.from_numpy(arc).cuda(), slots=3, max_blocks=1024, max_tokens=1 << 18, max_batch=64)
    n = 300
    arr, off, ln = synth.trace(n, 55, x.size, B, 50000.0, 16384, 262144)
    alone = [torch.full((int(v),), 0xCC, dtype=torch.uint8, device="cuda") for v in ln]
    mix = [torch.full((int(v),), 0xCC, dtype=torch.uint8, device="cuda") for v in ln]
    _say("serve alone")
    srv.run_alone(off, ln, alone)
    _say("serve mix")
    res = srv.run(arr, off, ln, mix)
    assert res["batches"] < n  # requests were batched
    for i in range(n):
        a, m = alone[i].cpu().numpy(), mix[i].cpu().numpy()
        assert np.array_equal(a, m), i
        assert np.array_equal(m, x[int(off[i]):int(off[i]) + int(ln[i])]), i
    assert np.all(res["latency_ns"] > 0)

"""The allocation-free whole-archive decode (aceapex_decode_all_static,
whose workspace is the library's static device scratch) against
aceapex_decode_all with a caller workspace: two static calls in a row, the
second on a smaller archive (so it runs over what the first left in the
scratch), every byte equal to the other entry point's and to the oracle's
decode; an archive whose workspace exceeds the scratch is refused before
anything is enqueued."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2608_10188_amd as ax  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _decoder(x):
    arc, _ = oracle.encode(x)
    ref = oracle.decode(arc)
    assert np.array_equal(ref, x)
    return ax.Decoder(arc, torch.from_numpy(arc).cuda()), ref


def test_static_decode_matches_decode_all():
    big, ref_big = _decoder(synth.dna(3 << 20, 81))
    small, ref_small = _decoder(synth.text((1 << 20) + 4099, 82))
    small.set_option(ax.OPT_GRAPH, 1)  # the static decode never captures a graph
    assert small.info.n_bytes < big.info.n_bytes
    for d in (big, small):
        assert d.workspace_bytes <= ax.STATIC_SCRATCH_BYTES
    outs = []
    for name, d in (("big", big), ("small", small)):
        n = int(d.info.n_bytes)
        out = torch.full((n,), 0xCC, dtype=torch.uint8, device="cuda")
        _say("decode_all_static", name, n)
        d.decode_all_static(out)
        assert d.static_status() == (0, (1 << 64) - 1)
        outs.append(out)
    for name, d, ref, got in (("big", big, ref_big, outs[0]), ("small", small, ref_small, outs[1])):
        n = int(d.info.n_bytes)
        work = torch.full((d.workspace_bytes,), 0xCC, dtype=torch.uint8, device="cuda")
        want = torch.full((n,), 0x33, dtype=torch.uint8, device="cuda")
        _say("decode_all", name, n)
        d.decode_all(out=want, work=work)
        assert d.status(work=work)[0] == 0
        w, g = want.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(g, w), name
        assert np.array_equal(g, ref), name


def test_static_decode_refuses_an_archive_beyond_the_scratch():
    x = synth.dna(40 << 20, 83)
    arc = ax.encode(x, threads=16)
    d = ax.Decoder(arc, torch.from_numpy(arc).cuda())
    assert d.workspace_bytes > ax.STATIC_SCRATCH_BYTES
    out = torch.full((x.size,), 0xCC, dtype=torch.uint8, device="cuda")
    _say("decode_all_static over capacity", d.workspace_bytes)
    with pytest.raises(ax.AceapexError) as ei:
        d.decode_all_static(out)
    assert ei.value.code == ax.AX_E_CAPACITY
    with pytest.raises(ax.AceapexError) as ei:
        d.decode_all_static(out[: x.size - 1])
    assert ei.value.code == ax.AX_E_CAPACITY
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0xCC).all()

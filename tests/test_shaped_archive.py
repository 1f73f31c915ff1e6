"""CPU checks of the large-shape input builder at a small size: the
oracle's decode of the assembled container returns the input (so the
builder's commands and bytes agree), and the commands cover what the large
GPU cases rely on."""
import numpy as np

import oracle
import shaped_archive

B = 16384


def test_builder_round_trips_through_the_oracle():
    n = 200 * B + 777
    x, cmds = shaped_archive.build(n, 3, every=8)
    assert np.all(np.diff(cmds["dst"].astype(np.int64)) > 0)
    arc = oracle.assemble(x, cmds)
    assert np.array_equal(oracle.decode(arc), x)
    assert oracle.info(arc).n_blocks == 201
    kinds = cmds["kind"]
    m = kinds > 0
    dist = cmds["dst"][m].astype(np.int64) - cmds["src"][m].astype(np.int64)
    assert (kinds == 0).any() and (kinds == 1).any() and (kinds == 2).any()
    assert set(np.unique(cmds["rep"][kinds == 2]).tolist()) == {0, 1, 2, 3}
    assert (cmds["len"][m] > 63 + 4).any()       # length escapes
    assert (dist < cmds["len"][m]).any()         # overlapping (periodic) copies
    assert (dist > 64 * B).any()                 # far sources


def test_content_blocks_include_the_window_edges():
    nb = ((1 << 32) + (1 << 28)) // B + 1
    c = set(shaped_archive.content_blocks(nb, 128, B).tolist())
    for edge in (1 << 31, 1 << 32):
        assert {edge // B - 1, edge // B} <= c

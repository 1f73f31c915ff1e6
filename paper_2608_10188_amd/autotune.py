"""Autotuner for decode plans.

Tries schedule knobs of a plan (a Batch or a Decoder) on its real input,
keeps only configurations whose output is byte-identical to the reference
configuration's (knobs may change schedules, never bytes), and picks the
fastest.  Runs on the device; the caller supplies outputs to compare.
"""
import itertools

from . import (OPT_BULK_ROUNDS, OPT_FILL_ROUNDS, OPT_FILL_TAIL, OPT_GRAPH, OPT_ROUND0_TILE, OPT_TAIL_CHUNKS,
               OPT_TAIL_MODE)

DEFAULT = {OPT_BULK_ROUNDS: 4, OPT_FILL_ROUNDS: 0, OPT_FILL_TAIL: 0, OPT_TAIL_CHUNKS: 1, OPT_ROUND0_TILE: 1,
           OPT_TAIL_MODE: 0, OPT_GRAPH: 1}

GRID = {
    OPT_BULK_ROUNDS: [1, 2, 4, 8],
    OPT_FILL_ROUNDS: [0, 1],
    OPT_ROUND0_TILE: [1, 0],
    OPT_TAIL_MODE: [0, 1],
}


def candidates():
    keys = list(GRID)
    for vals in itertools.product(*(GRID[k] for k in keys)):
        c = dict(DEFAULT)
        c.update(zip(keys, vals))
        yield c


def tune(plan, run, outputs, reps=3):
    """plan: object with set_option; run(): enqueue one decode; outputs: list
    of device tensors written by run().  Returns (best_config, table)."""
    import torch

    def apply(cfg):
        for k, v in cfg.items():
            plan.set_option(k, v)

    def timed():
        run()  # warm (and graph capture)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    apply(DEFAULT)
    run()
    torch.cuda.synchronize()
    reference = [o.clone() for o in outputs]
    table = []
    best, best_ms = dict(DEFAULT), None
    for cfg in candidates():
        apply(cfg)
        for o in outputs:
            o.fill_(0xCC)
        ms = timed()
        same = all(torch.equal(a, b) for a, b in zip(outputs, reference))
        table.append((cfg, ms, same))
        if same and (best_ms is None or ms < best_ms):
            best, best_ms = cfg, ms
    apply(best)
    return best, table

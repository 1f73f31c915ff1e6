"""Serving loop: random-access byte ranges against an archive held compressed
in device memory, with continuous batching.

Requests (offset, length) arrive on an open-loop schedule.  Each slot owns a
stream and one range-plan workspace sized by closure limits (blocks and
matches of a batch's union source closure, plus a compact scratch of those
blocks), so the device memory of serving is slots x workspace, independent of
the archive's size.  A request's own closure size is computed once, when it
arrives; whenever a slot is free, the requests that have arrived are
admitted in arrival order while the sum of their closure sizes fits the
slot's limits (the sum bounds the union, so an admitted batch always fits)
and decoded as one batch by the library on that slot's stream
(aceapex_decode_ranges: union closure on the host, plan upload, entropy,
parse and match layer of the closure blocks, copy of each range to its
output).  Requests that arrive while batches run join the next batch as a
slot frees up, and batches on different slots overlap on the device.
Latency is arrival to completion, read from HIP events on the device
timeline.
"""
import collections
import gc
import time

import numpy as np

from . import COPY_PERIODIC, Decoder, RangePlan


class Server:
    def __init__(self, h_archive, d_archive, slots=3, max_blocks=4096, max_tokens=1 << 20, max_batch=256):
        import torch

        self.dec = Decoder(h_archive, d_archive)
        dev = d_archive.device
        self.dec.build_index()
        self.dec._work = None  # the whole-archive workspace is only needed for the index
        self.slots = []
        for _ in range(slots):
            plan = RangePlan(self.dec, max_blocks, max_tokens)
            work = torch.empty(max(256, plan.workspace_bytes), dtype=torch.uint8, device=dev)
            self.slots.append({"plan": plan, "work": work, "stream": torch.cuda.Stream(device=dev)})
        torch.cuda.synchronize()
        self.max_blocks, self.max_tokens = int(max_blocks), int(max_tokens)
        self.workspace_bytes = sum(int(s["work"].numel()) for s in self.slots)
        self.max_batch = max_batch
        self.device = dev

    def closure_size(self, off, length):
        """(blocks, matches) of one range's source closure (host)."""
        _, tokens, blocks = self.dec.closure_blocks([off], [length], threads=1, want_blocks=False)
        return blocks, tokens

    def _launch(self, slot, ids, offs, lens, outs):
        s = self.slots[slot]
        s["plan"].decode([int(offs[i]) for i in ids], [int(lens[i]) for i in ids], [outs[i] for i in ids], s["work"],
                         COPY_PERIODIC, stream=s["stream"])

    def run(self, arrivals_ns, offs, lens, outs, realtime=True, max_batch=None, slots=None):
        """Serve every request; outs[i] receives range i (a CUDA uint8 tensor
        of lens[i] bytes).  Returns a dict with per-request latency (ns,
        device timeline), host-observed latency (ns) and batch statistics.
        max_batch=1 with slots=1 serves one request at a time, in order."""
        max_batch = max_batch or self.max_batch
        # the collector would stop the loop for tens of milliseconds now and
        # then (every batch allocates events and lists): off while serving
        gc_was_on = gc.isenabled()
        gc.disable()
        try:
            return self._run(arrivals_ns, offs, lens, outs, realtime, max_batch, slots)
        finally:
            if gc_was_on:
                gc.enable()

    def _run(self, arrivals_ns, offs, lens, outs, realtime, max_batch, slots):
        import torch

        n = len(offs)
        arrivals = np.asarray(arrivals_ns, dtype=np.int64)
        free = collections.deque(range(min(len(self.slots), slots or len(self.slots))))
        inflight = {}
        queue = collections.deque()
        size = [None] * n  # closure (blocks, matches), computed on arrival
        done_ev = [None] * n
        host_done = np.zeros(n, np.int64)
        batch_sizes, batch_blocks = [], []
        nxt = completed = 0
        torch.cuda.synchronize()
        origin = torch.cuda.Event(enable_timing=True)
        origin.record(torch.cuda.current_stream())
        t0 = time.perf_counter_ns()
        while completed < n:
            now = time.perf_counter_ns() - t0
            arrived = nxt
            while arrived < n and (not realtime or arrivals[arrived] <= now):
                arrived += 1
            if arrived > nxt:  # the closure sizes of all new arrivals, in one parallel call
                nb, nt = self.dec.closure_sizes(offs[nxt:arrived], lens[nxt:arrived])
                for k in range(arrived - nxt):
                    size[nxt + k] = (int(nb[k]), int(nt[k]))
                    if size[nxt + k][0] > self.max_blocks or size[nxt + k][1] > self.max_tokens:
                        raise ValueError(f"request {nxt + k}: closure {size[nxt + k]} exceeds a slot's limits")
                    queue.append(nxt + k)
                nxt = arrived
            for slot in list(inflight):
                ev, ids = inflight[slot]
                if ev.query():
                    t = time.perf_counter_ns() - t0
                    for i in ids:
                        host_done[i] = t
                    completed += len(ids)
                    del inflight[slot]
                    free.append(slot)
            progressed = False
            while free and queue:
                slot = free.popleft()
                # admission by scratch: arrival order, while the summed
                # closure sizes fit the slot's workspace limits
                take, nb, nt = [], 0, 0
                while queue and len(take) < max_batch:
                    b, t = size[queue[0]]
                    if take and (nb + b > self.max_blocks or nt + t > self.max_tokens):
                        break
                    take.append(queue.popleft())
                    nb, nt = nb + b, nt + t
                self._launch(slot, take, offs, lens, outs)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.slots[slot]["stream"])
                for i in take:
                    done_ev[i] = ev
                inflight[slot] = (ev, take)
                batch_sizes.append(len(take))
                batch_blocks.append(self.slots[slot]["plan"].last()[0])
                progressed = True
            if not progressed and completed < n:
                time.sleep(20e-6)
        torch.cuda.synchronize()
        ev_ms = {}
        for ev in done_ev:
            if id(ev) not in ev_ms:
                ev_ms[id(ev)] = origin.elapsed_time(ev)
        dev_done = np.array([ev_ms[id(done_ev[i])] * 1e6 for i in range(n)], dtype=np.float64)
        if not realtime:
            arrivals = np.zeros(n, np.int64)
        return {
            "latency_ns": dev_done - arrivals,
            "host_latency_ns": host_done - arrivals,
            "batches": len(batch_sizes),
            "batch_size_mean": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
            "closure_blocks_mean": float(np.mean(batch_blocks)) if batch_blocks else 0.0,
            "wall_ns": int(time.perf_counter_ns() - t0),
        }

    def run_alone(self, offs, lens, outs):
        """Each request alone: one batch per request, one slot, in order."""
        import torch

        for i in range(len(offs)):
            self._launch(0, [i], offs, lens, outs)
        torch.cuda.synchronize()

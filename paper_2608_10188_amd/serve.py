"""Serving loop: random-access byte ranges against an archive held compressed
in device memory, with continuous batching.

Requests (offset, length) arrive on an open-loop schedule.  Whenever a slot
is free, every request that has arrived and fits the slot's scratch limits
(blocks and matches of the union source closure) is admitted into one batch,
and the batch is decoded by the library on that slot's stream
(aceapex_decode_ranges: union closure on the host, plan upload, entropy,
parse and match layer of the closure blocks, copy of each range to its
output).  Requests that arrive while batches run join the next batch as a
slot frees up, and batches on different slots overlap on the device.  Each
slot owns its stream, workspace and a scratch output of the archive's size,
so concurrent batches never write the same bytes.  Latency is arrival to
completion, read from HIP events on the device timeline.
"""
import collections
import gc
import time

import numpy as np

from . import AX_E_CAPACITY, COPY_PERIODIC, AceapexError, Decoder, RangePlan


class Server:
    def __init__(self, h_archive, d_archive, slots=3, max_blocks=4096, max_tokens=1 << 20, max_batch=256):
        import torch

        self.dec = Decoder(h_archive, d_archive)
        n = int(self.dec.info.n_bytes)
        dev = d_archive.device
        self.slots = []
        for _ in range(slots):
            full = torch.empty(max(16, n), dtype=torch.uint8, device=dev)
            plan = RangePlan(self.dec, max_blocks, max_tokens)
            work = torch.empty(max(256, plan.workspace_bytes), dtype=torch.uint8, device=dev)
            self.slots.append({"full": full, "plan": plan, "work": work, "stream": torch.cuda.Stream(device=dev)})
        self.dec.build_index(self.slots[0]["full"])
        self.dec._work = None  # the whole-archive workspace is only needed for the index
        torch.cuda.synchronize()
        self.max_batch = max_batch
        self.device = dev

    def _launch(self, slot, ids, offs, lens, outs):
        s = self.slots[slot]
        s["plan"].decode([int(offs[i]) for i in ids], [int(lens[i]) for i in ids], [outs[i] for i in ids], s["full"],
                         s["work"], COPY_PERIODIC, stream=s["stream"])

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
            while nxt < n and (not realtime or arrivals[nxt] <= now):
                queue.append(nxt)
                nxt += 1
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
                take = [queue[k] for k in range(min(len(queue), max_batch))]
                while True:
                    try:
                        self._launch(slot, take, offs, lens, outs)
                        break
                    except AceapexError as e:  # admission by scratch: shrink the batch
                        if e.code != AX_E_CAPACITY or len(take) == 1:
                            raise
                        take = take[: len(take) // 2]
                for _ in take:
                    queue.popleft()
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

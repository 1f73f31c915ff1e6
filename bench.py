"""Benchmark: device-resident full decode of the 254 MB synthetic DNA archive.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dna254|text200|dna4|batch|serve]
                [--copy periodic|serial] [--no-rep] [--no-cpu-baseline]

One step = one aceapex_decode_all of the whole archive (rANS of the four
streams of every block, command parse with literal placement, match copy with
periodic fills scheduled by source readiness), inputs resident in HBM.
Prints one JSON line.  The archive is generated and encoded on the host first
(outside the timed region); the decode is checked byte for byte against the
original before timing.  After the timed steps, 16 KiB reads of the same
archive are served one at a time (closed loop) for their p50/p99 latency.

--workload batch: thousands of archives in one plan against the plain
per-archive loop.  --workload serve: a synthetic DNA archive held compressed
on the device (32 GiB by default) served to open-loop Poisson request traces
with continuous batching, against one-request-at-a-time service.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded GB/s device-resident (254 MB DNA) vs HBM peak; p50/p99 us per 16 KB read"
HBM_PEAK_GBS = 8000.0

# HBM bytes moved by one whole decode of the 254 MB DNA workload (all its
# kernels), from two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE,
# each scaled by the same counter on a plain 256 MiB device copy in the same
# run).  They hold only for the decoder source they were taken on (first 16
# hex digits of its SHA-256); otherwise the line reports traffic null.
TRAFFIC_SOURCE = "fb8af562ee6cd7c8"
TRAFFIC_MB = 1952.4  # read + write MB per decode

WORKLOADS = {
    # name: (generator, bytes, seed, description)
    "dna254": ("dna", 15500 * 16384, 2, "synthetic DNA 253,952,000 B, 15,500 x 16 KiB blocks"),
    "text200": ("text", 209715200, 3, "synthetic English-like text 209,715,200 B, 12,800 x 16 KiB blocks"),
    "dna4": ("dna", 4 * 1024 * 1024, 1, "synthetic DNA 4 MiB, 256 x 16 KiB blocks"),
}


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dna254", choices=sorted(WORKLOADS) + ["batch", "serve"])
    ap.add_argument("--batch-count", type=int, default=4096, help="archives in the batched workload")
    ap.add_argument("--autotune", action="store_true", help="batched workload: tune knobs per size class")
    ap.add_argument("--streams", type=int, default=1,
                    help="batched workload: archives dealt over this many plans, each on its own stream")
    ap.add_argument("--copy", default="periodic", choices=["periodic", "serial"])
    ap.add_argument("--no-rep", action="store_true")
    ap.add_argument("--depth-cap", type=int, default=0, help="encoder depth cap L (0 = none)")
    ap.add_argument("--syms-per-lane", type=int, default=0,
                    help="encoder rANS lane rule S (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--threads", type=int, default=16, help="encoder threads (0 = all)")
    ap.add_argument("--reads", type=int, default=1000, help="closed-loop 16 KiB reads after the timed steps")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration under a profiler)")
    ap.add_argument("--serve-bytes", type=int, default=32 << 30, help="serving archive size")
    ap.add_argument("--rates", default="2000,5000,20000,50000,200000", help="serving arrival rates, req/s")
    ap.add_argument("--requests", type=int, default=10000, help="requests per serving trace point")
    ap.add_argument("--sizes", default="16k,mixed", help="serving request sizes: 16k and/or mixed (16 KiB-1 MiB)")
    ap.add_argument("--slots", type=int, default=3, help="serving slots (concurrent batches)")
    ap.add_argument("--max-blocks", type=int, default=8192, help="serving admission limit: closure blocks per batch")
    ap.add_argument("--max-tokens", type=int, default=1 << 21, help="serving admission limit: matches per batch")
    ap.add_argument("--bulk-rounds", type=int, default=0, help="level-synchronous copy rounds (0 = library default)")
    ap.add_argument("--tail-chunks", type=int, default=0, help="chunks per persistent-launch ticket (0 = default)")
    ap.add_argument("--fill", default="", help="fill modes 'R,T' for rounds and tail (0 lane/wave, 1 segmented)")
    ap.add_argument("--graph", type=int, default=0, help="1: each decode replays the plan captured as one hipGraph")
    ap.add_argument("--tail-mode", type=int, default=0, help="deep remainder: 0 pointer jumping, 1 persistent chase")
    ap.add_argument("--jump-passes", type=int, default=0, help="at most this many jump passes (0 = automatic)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def host_cpu():
    """Host CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


def cpu_baseline(arc, n_bytes, x):
    """The oracle's sequential decode on one host core over the whole archive
    (median of 5, about 3 s of CPU work at this size), and its encoder on a
    bounded 32 MiB prefix of the input (about 10 s)."""
    import oracle

    times = []
    for _ in range(5):
        t = time.perf_counter()
        oracle.decode(arc, verify=False)
        times.append(time.perf_counter() - t)
    t = float(np.median(times))
    prefix = x[: 32 << 20]
    t0 = time.perf_counter()
    oracle.encode(prefix)
    enc_s = time.perf_counter() - t0
    return {"value": n_bytes / t / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"whole archive ({n_bytes} B), median of 5 single-threaded oracle decodes "
                      f"(min {min(times):.3f} s, max {max(times):.3f} s)",
            "encode_gbs": round(prefix.size / enc_s / 1e9, 5),
            "encode_sample": f"oracle encoder on the first {prefix.size} B of the input, {enc_s:.2f} s",
            "host": host_cpu()}


def store_probe(torch, dev, n_bytes, reps=20):
    """Coalesced-write ceiling on this GPU: torch's fill of an n-byte buffer
    (a plain store kernel, 16-byte vector stores) and a device copy of the
    same size, timed with events; GB/s of bytes written."""
    a = torch.empty(n_bytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    out = {}
    for name, fn in (("fill", lambda: a.fill_(7)), ("copy", lambda: b.copy_(a))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 4), "written_gbs": round(n_bytes / ms / 1e6, 1)}
    out["copy"]["moved_gbs"] = round(2 * n_bytes / out["copy"]["ms"] / 1e6, 1)
    del a, b
    return out


def _pcts(ns):
    ns = np.asarray(ns, dtype=np.float64)
    return round(float(np.percentile(ns, 50)) / 1e3, 1), round(float(np.percentile(ns, 99)) / 1e3, 1)


def read_latency(ax, dec, x, count, size, seed):
    """Closed loop: `count` reads of `size` bytes at trace-generated offsets
    (80% Zipf-local, 20% uniform), each issued alone through
    aceapex_decode_range and waited for, with a workspace of the largest
    aceapex_range_workspace among them.  Latency runs from the host call
    (closure, plan upload, kernels) to the device event after the copy-out;
    every read is checked against the input."""
    import torch

    import synth

    dev = dec.device
    _, offs, lens = synth.trace(count, seed, x.size, 16384, 1000.0, size, size)
    need = max(dec.range_workspace(int(o), size) for o in offs)
    work = torch.empty(max(256, need), dtype=torch.uint8, device=dev)
    outs = torch.empty((count, size), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    lat = []
    for i in range(count):
        torch.cuda.synchronize()
        t = time.perf_counter_ns()
        dec.decode_range(int(offs[i]), size, outs[i], work, stream=stream)
        end = torch.cuda.Event()
        end.record(stream)
        end.synchronize()
        lat.append(time.perf_counter_ns() - t)
    got = outs.cpu().numpy()
    bad = sum(not np.array_equal(got[i], x[int(offs[i]): int(offs[i]) + size]) for i in range(count))
    p50, p99 = _pcts(lat)
    return {"p50_us": p50, "p99_us": p99, "reads": count, "bytes": size, "mismatches": int(bad),
            "workspace_bytes": int(need), "mode": "closed loop, one read at a time"}


# ------------------------------------------------- served workload (config 5)
#
# A DNA archive held compressed in HBM; Poisson request traces at several
# arrival rates, served by the continuous-batching loop, against the same
# trace served one request at a time through the same range decoder.

def run_serve(args, log):
    import torch

    import synth
    import paper_2608_10188_amd as ax
    from paper_2608_10188_amd.serve import Server

    n = int(args.serve_bytes)
    marks = set()

    def gen_progress(done, total):
        g = done * 8 // total
        if g not in marks:
            marks.add(g)
            log(f"generated {done >> 20} of {total >> 20} MiB")

    t0 = time.time()
    x = synth.dna_segmented(n, 5, threads=16, progress=gen_progress)
    log(f"generated {n} B in {time.time() - t0:.1f}s")
    t0 = time.time()
    arc, st = ax.encode(x, stats=True, window_log=30 if n >= (1 << 32) else 0, threads=args.threads,
                        progress=lambda d, t: log(f"encoded {d >> 20} of {t >> 20} MiB in {time.time() - t0:.0f}s"))
    log(f"encoded to {arc.size} B (ratio {n / arc.size:.3f}) in {time.time() - t0:.1f}s; "
        f"{st.n_matches} matches over {st.n_blocks} blocks")
    dev = torch.device("cuda:0")
    d_arc = torch.from_numpy(arc).to(dev)
    t0 = time.time()
    srv = Server(arc, d_arc, slots=args.slots, max_blocks=args.max_blocks, max_tokens=args.max_tokens)
    log(f"server ready in {time.time() - t0:.1f}s (token index built on the device)")
    unloaded = read_latency(ax, srv.dec, x, args.reads, 16384, 54)
    log(f"unloaded 16 KiB reads: p50 {unloaded['p50_us']} us, p99 {unloaded['p99_us']} us")

    rates = [float(r) for r in args.rates.split(",") if r]
    points, count = [], int(args.requests)
    skip = count // 20  # the first 5% of each trace warm the loop up
    for mode in [m for m in args.sizes.split(",") if m]:
        lmin, lmax = (16384, 16384) if mode == "16k" else (16384, 1 << 20)
        for k, rate in enumerate(rates):
            arr, offs, lens = synth.trace(count, 55 + k, n, 16384, rate, lmin, lmax)
            buf = torch.empty(int(lens.sum()), dtype=torch.uint8, device=dev)
            outs = list(torch.split(buf, [int(v) for v in lens]))
            r = srv.run(arr, offs, lens, outs)
            got = buf.cpu().numpy()
            at, bad = 0, 0
            for i in range(count):
                o, ln = int(offs[i]), int(lens[i])
                bad += not np.array_equal(got[at: at + ln], x[o: o + ln])
                at += ln
            req_bytes = float(lens.sum())
            p50, p99 = _pcts(r["latency_ns"][skip:])
            h50, h99 = _pcts(r["host_latency_ns"][skip:])
            pt = {"sizes": mode, "rate": rate, "p50_us": p50, "p99_us": p99, "host_p50_us": h50, "host_p99_us": h99,
                  "served_req_s": round(count / (r["wall_ns"] / 1e9), 1),
                  "requested_gbs": round(req_bytes / r["wall_ns"], 3), "batches": r["batches"],
                  "batch_size_mean": round(r["batch_size_mean"], 2),
                  "closure_blocks_mean": round(r["closure_blocks_mean"], 1),
                  "decoded_gbs": round(r["closure_blocks_mean"] * r["batches"] * int(srv.dec.info.block_size)
                                       / r["wall_ns"], 3),
                  "mismatches": int(bad)}
            if mode == "16k":
                b = srv.run(arr, offs, lens, outs, max_batch=1, slots=1)
                b50, b99 = _pcts(b["latency_ns"][skip:])
                pt["one_at_a_time"] = {"p50_us": b50, "p99_us": b99,
                                       "served_req_s": round(count / (b["wall_ns"] / 1e9), 1),
                                       "requested_gbs": round(req_bytes / b["wall_ns"], 3)}
            del buf, outs, got
            log(json.dumps(pt))
            points.append(pt)
    best = max(points, key=lambda p: p["requested_gbs"]) if points else None
    res = {
        "metric": "served range reads: p50/p99 us per 16 KB read and aggregate requested GB/s",
        "value": best["requested_gbs"] if best else None, "unit": "GB/s", "n_gpus": 1,
        "steps": count, "warmup": skip, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"synthetic DNA {n} B held compressed ({arc.size} B), Poisson range reads",
                   "n_bytes": n, "archive_bytes": int(arc.size), "blocks": int(st.n_blocks),
                   "matches": int(st.n_matches), "slots": args.slots, "max_blocks": args.max_blocks,
                   "serving_workspace_bytes": int(srv.workspace_bytes),
                   "max_tokens": args.max_tokens, "requests_per_point": count},
        "unloaded_16k": unloaded, "points": points,
    }
    print(json.dumps(res), flush=True)


# ------------------------------------------------- batched workload (config 4)
#
# One plan decoding every archive (launch sequence captured as a hipGraph,
# optionally autotuned per size class) against the plain per-archive decode
# looped over the same archives on the same stream.

CLASSES = [(0, 1 << 20), (1 << 20, 8 << 20), (8 << 20, 1 << 62)]  # size classes for the autotuner


def _make(i, size, kind):
    import xxhash

    import synth
    import paper_2608_10188_amd as ax

    x = synth.dna(size, 1000 + i) if kind == 0 else synth.text(size, 1000 + i)
    h = xxhash.xxh3_64_intdigest(x.tobytes())
    arc = ax.encode(x, threads=1)
    return arc, h, size


def run_batch(args, log):
    import torch
    import xxhash

    import synth
    import paper_2608_10188_amd as ax
    from paper_2608_10188_amd import autotune

    count = args.batch_count
    sizes, kinds = synth.batch_plan(count, 4)
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
        made = list(pool.map(_make, range(count), [int(v) for v in sizes], [int(k) for k in kinds]))
    total = sum(m[2] for m in made)
    comp = sum(m[0].size for m in made)
    log(f"{count} archives, {total} B decoded, {comp} B compressed, built in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    decs, outs = [], []
    for arc, h, n in made:
        d = ax.Decoder(arc, torch.from_numpy(arc).to(dev))
        decs.append(d)
        outs.append(torch.empty(max(16, n), dtype=torch.uint8, device=dev))
    batch = ax.Batch(decs, outs)
    work = batch.workspace()
    log(f"batch plan: workspace {batch.workspace_bytes / 2**30:.2f} GiB")

    # correctness (poisoned outputs), outside the timed region
    for o in outs:
        o.fill_(0xCC)
    batch.decode()
    err, bad = batch.status()
    bad_archives = 0
    for (arc, h, n), o in zip(made, outs):
        if xxhash.xxh3_64_intdigest(o[:n].cpu().numpy().tobytes()) != h:
            bad_archives += 1
    if err or bad_archives:
        print(json.dumps({"metric": "batched decoded GB/s", "value": None, "error": f"status {err}, {bad_archives} bad"}))
        raise SystemExit(1)

    def time_it(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    tuned = {}
    if args.autotune:
        # one plan per size class, each tuned on its own archives
        class_plans = []
        for lo, hi in CLASSES:
            idx = [i for i, m in enumerate(made) if lo <= m[2] < hi]
            if not idx:
                continue
            cb = ax.Batch([decs[i] for i in idx], [outs[i] for i in idx])
            cw = cb.workspace()
            best, table = autotune.tune(cb, lambda cb=cb, cw=cw: cb.decode(work=cw), [outs[i] for i in idx])
            tuned[f"{lo}-{hi}"] = {"archives": len(idx), "best": {str(k): v for k, v in best.items()},
                                   "ms": [round(t[1], 3) for t in table if t[2]], "all_identical": all(t[2] for t in table)}
            class_plans.append((cb, cw))
        batched_ms = time_it(lambda: [cb.decode(work=cw) for cb, cw in class_plans], args.steps, args.warmup)
    elif args.streams > 1:
        # independent archives: sorted by matches per block and dealt round
        # robin over S plans (similar mixes), each with its own workspace and
        # stream, so one plan's dependency-bound persistent launch overlaps
        # the others' work
        order = sorted(range(count), key=lambda i: -decs[i].info.n_matches / max(1, decs[i].info.n_blocks))
        groups = [order[g::args.streams] for g in range(args.streams)]
        plans = []
        for g in groups:
            gb = ax.Batch([decs[i] for i in g], [outs[i] for i in g])
            gb.set_option(ax.OPT_GRAPH, 1)
            if args.bulk_rounds:
                gb.set_option(ax.OPT_BULK_ROUNDS, args.bulk_rounds)
            plans.append((gb, gb.workspace(), torch.cuda.Stream(device=dev)))

        def run_streams():
            cur = torch.cuda.current_stream()
            for _, _, st in plans:
                st.wait_stream(cur)
            for gb, gw, st in plans:
                gb.decode(work=gw, stream=st)
            for _, _, st in plans:
                cur.wait_stream(st)

        for o in outs:
            o.fill_(0xCC)
        run_streams()
        torch.cuda.synchronize()
        bad_archives = sum(xxhash.xxh3_64_intdigest(o[:n].cpu().numpy().tobytes()) != h
                           for (arc, h, n), o in zip(made, outs))
        errs = [gb.status(stream=st, work=gw)[0] for gb, gw, st in plans]
        if any(errs) or bad_archives:
            print(json.dumps({"metric": "batched decoded GB/s", "value": None,
                              "error": f"status {errs}, {bad_archives} bad (streams)"}))
            raise SystemExit(1)
        batched_ms = time_it(run_streams, args.steps, args.warmup)
    else:
        batch.set_option(ax.OPT_GRAPH, 1)
        if args.bulk_rounds:
            batch.set_option(ax.OPT_BULK_ROUNDS, args.bulk_rounds)
        batched_ms = time_it(lambda: batch.decode(work=work), args.steps, args.warmup)
    err, _ = batch.status()

    # plain decode looped over the archives on the same stream
    ws = max(d.workspace_bytes for d in decs)
    shared = torch.empty(max(256, ws), dtype=torch.uint8, device=dev)
    loop_steps = max(1, min(args.steps, 3))
    loop_ms = time_it(lambda: [d.decode_all(out=o, work=shared) for d, o in zip(decs, outs)], loop_steps, 1)
    err2, _ = ax.workspace_status(shared)

    res = {
        "metric": "batched decoded GB/s (4096 archives, 64 KiB-64 MiB, 60% DNA / 40% text)",
        "value": round(total / (batched_ms / 1e3) / 1e9, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(batched_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"batch of {count} archives", "n_bytes": total, "archive_bytes": comp,
                   "autotuned": bool(args.autotune), "bulk_rounds": None if args.autotune else (args.bulk_rounds or 4),
                   "streams": 1 if args.autotune else args.streams},
        "plain_loop_gbs": round(total / (loop_ms / 1e3) / 1e9, 3), "plain_loop_ms": round(loop_ms, 3),
        "speedup_vs_plain_loop": round(loop_ms / batched_ms, 3), "status": [err, err2],
        "autotune": tuned or None,
    }
    print(json.dumps(res), flush=True)


def main():
    args = parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args, log)
        return
    if args.workload == "serve":
        run_serve(args, log)
        return
    import torch
    import xxhash

    import synth
    import paper_2608_10188_amd as ax

    gen, n, seed, desc = WORKLOADS[args.workload]
    t0 = time.time()
    x = synth.dna(n, seed) if gen == "dna" else synth.text(n, seed)
    log(f"generated {n} B in {time.time() - t0:.1f}s")
    t0 = time.time()
    enc_kw = {"rans_min_syms_per_lane": args.syms_per_lane} if args.syms_per_lane else {}
    if args.depth_cap:
        enc_kw["depth_cap"] = args.depth_cap
    arc, st = ax.encode(x, stats=True, no_rep=int(args.no_rep), threads=args.threads, **enc_kw)
    log(f"encoded to {arc.size} B (ratio {n / arc.size:.3f}) in {time.time() - t0:.1f}s; "
        f"{st.n_commands} commands, {st.n_matches} matches, {st.n_rep} repeats")
    want = xxhash.xxh3_64_intdigest(x.tobytes())

    dev = torch.device("cuda:0")
    d_arc = torch.from_numpy(arc).to(dev)
    dec = ax.Decoder(arc, d_arc)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    work = dec.workspace()
    mode = ax.COPY_SERIAL if args.copy == "serial" else ax.COPY_PERIODIC
    if args.bulk_rounds:
        dec.set_bulk_rounds(args.bulk_rounds)
    if args.tail_chunks:
        dec.set_option(ax.OPT_TAIL_CHUNKS, args.tail_chunks)
    if args.fill:
        fr, ft = (int(v) for v in args.fill.split(","))
        dec.set_option(ax.OPT_FILL_ROUNDS, fr)
        dec.set_option(ax.OPT_FILL_TAIL, ft)
    if args.graph:
        dec.set_option(ax.OPT_GRAPH, 1)
    if args.tail_mode:
        dec.set_option(ax.OPT_TAIL_MODE, args.tail_mode)
    if args.jump_passes:
        dec.set_option(ax.OPT_JUMP_PASSES, args.jump_passes)
    stream = torch.cuda.current_stream()
    if args.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE under a
        # counter profiler give the scale factor for the decode's counters
        a = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # correctness first (poisoned output), outside the timed region
    out.fill_(0xCC)
    dec.decode_all(out=out, copy_mode=mode)
    err, bad = dec.status()
    got = out.cpu().numpy()
    ok = err == 0 and xxhash.xxh3_64_intdigest(got.tobytes()) == want and np.array_equal(got, x)
    if not ok:
        log(f"DECODE MISMATCH err={err} block={bad}")
        print(json.dumps({"metric": METRIC, "value": None, "error": "decode mismatch"}))
        sys.exit(1)
    del got

    for _ in range(args.warmup):
        dec.decode_all(out=out, copy_mode=mode)
    torch.cuda.synchronize()
    # throughput: K back-to-back decodes on the stream, bracketed by events
    # (one event before each step as well, for the per-step spread)
    t_start = time.perf_counter()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for k in range(args.steps):
        dec.decode_all(out=out, copy_mode=mode)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    gpu_ms = evs[0].elapsed_time(evs[-1])
    step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    # stage split: K more decodes with the library's stage events (HIP events
    # recorded on the decode stream around the rANS, parse, bulk-round and
    # remainder kernels of every window)
    dec.set_timing(True)
    stage = np.zeros(4)
    for _ in range(args.steps):
        dec.decode_all(out=out, copy_mode=mode)
        stage += np.array(dec.stage_ms(remainder=True))  # waits for this decode's last event
    dec.set_timing(False)
    err, bad = dec.status()
    if err:
        log(f"device status {err} during timing")
        sys.exit(1)
    # the timed decodes ran what the decoder learned from the first ones
    # (bulk-round and jump-pass counts): the last one's output is checked too
    if xxhash.xxh3_64_intdigest(out.cpu().numpy().tobytes()) != want:
        log("DECODE MISMATCH after timing")
        print(json.dumps({"metric": METRIC, "value": None, "error": "decode mismatch after timing"}))
        sys.exit(1)
    ms_per_step = gpu_ms / args.steps
    value = n / (ms_per_step / 1e3) / 1e9
    ans_ms, parse_ms, copy_ms, rem_ms = (stage / args.steps).tolist()

    # algorithmic bytes per decode (the HBM floor of the whole path): output
    # N written, compressed archive C read, match sources S = sum over matches
    # of min(len, dist) read
    s_bytes = int(st.n_src_bytes)
    match_bytes = int(st.n_match_bytes)
    c_bytes = int(arc.size)
    b_alg = n + c_bytes + s_bytes
    d_bytes = int(st.n_lit_bytes + st.n_commands + st.n_off_bytes + st.n_len_bytes)  # decoded stream symbols

    stages = {"ans": ans_ms, "parse": parse_ms, "copy": copy_ms}
    # per-stage algorithmic bytes (extras; byte definitions in the design notes):
    #   ans:   read compressed payload C, write decoded stream symbols D
    #   parse: read decoded symbols D, write the output N (tile) and tokens (16 B per match)
    #   copy:  read match sources S, write match bytes M
    alg = {"ans": c_bytes + d_bytes, "parse": d_bytes + n + 16 * st.n_matches, "copy": s_bytes + match_bytes}
    import hashlib

    src_hash = hashlib.sha256(open(os.path.join(ROOT, "paper_2608_10188_amd", "csrc", "decoder.hip"), "rb").read())
    traffic = None
    defaults = not (args.no_rep or args.syms_per_lane or args.depth_cap or args.bulk_rounds or args.fill
                    or args.tail_chunks or args.copy != "periodic" or args.tail_mode or args.jump_passes)
    if (args.workload == "dna254" and defaults and TRAFFIC_MB is not None
            and src_hash.hexdigest()[:16] == TRAFFIC_SOURCE):
        traffic = int(TRAFFIC_MB * 1e6)
    achieved = b_alg / (ms_per_step / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "whole decode (every kernel of one aceapex_decode_all)",
                "alg_bytes": b_alg, "alg_def": "N + C + S: output, compressed archive, match sources",
                "stages": {k: {"alg_bytes": int(alg[k]), "ms": round(stages[k], 4),
                               "achieved_gbs": round(alg[k] / (stages[k] / 1e3) / 1e9, 2)} for k in stages}}
    probe = store_probe(torch, dev, n)
    probe["decoded_frac_of_fill"] = round(value / probe["fill"]["written_gbs"], 5)
    probe["alg_frac_of_copy"] = round(achieved / probe["copy"]["moved_gbs"], 5)

    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": desc, "n_bytes": n, "archive_bytes": c_bytes,
                   "ratio": round(n / c_bytes, 4), "blocks": int(dec.info.n_blocks),
                   "commands": int(st.n_commands), "matches": int(st.n_matches), "repeats": int(st.n_rep),
                   "copy_mode": args.copy, "no_rep": bool(args.no_rep), "depth_cap": args.depth_cap,
                   "max_depth": int(st.max_depth) if args.depth_cap else None, "bulk_rounds": args.bulk_rounds or 4, "fill": args.fill or "0,0", "tail_chunks": args.tail_chunks or 1,
                   "graph": bool(args.graph), "tail_mode": "chase" if args.tail_mode else "jump",
                   "jump_passes": args.jump_passes or "auto"},
        "decoded_frac_of_hbm_peak": round(value / HBM_PEAK_GBS, 5),
        "step_ms": {"min": round(float(step_ms.min()), 4), "median": round(float(np.median(step_ms)), 4),
                    "max": round(float(step_ms.max()), 4)},
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        "remainder_ms": round(rem_ms, 4),
        "store_probe": probe,
        "stage_share": {k: round(v / max(1e-9, sum(stages.values())), 4) for k, v in stages.items()},
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }
    if args.reads:
        t0 = time.time()
        dec.build_index(work=work)
        res["read_16k"] = read_latency(ax, dec, x, args.reads, 16384, 54)
        log(f"16 KiB reads: {res['read_16k']} ({time.time() - t0:.1f}s)")
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(arc, n, x)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

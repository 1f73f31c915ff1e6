"""Measurement studies on one MI355X, beside the benchmark.

Each study prints one JSON line per measured point (stderr carries progress)
and a final summary line.  Every decode is checked against its input (XXH3
and every byte) before it is timed; inputs are the seeded synthetic corpora.

  depth     The encoder's depth cap L (matches deeper than L forced to
            literals, iterated until no token is deeper; the paper's "Depth
            Does Not Govern Latency" section and Table 3): ratio(L), maximum
            depth, forced bytes, decode time and stage split per L, and the
            least-squares fit latency = c + a * levels + b * copied MB of
            the reconciling model, on the DNA and text workloads.
  minmatch  Bit-perfect minimum-match sweep (the encoder never emits a match
            shorter than m; literals take the rest): ratio, commands,
            matches, copied share and the entropy / parse / copy split per m.
  corpora   The four synthetic corpora (DNA, English-like text, proteins,
            FASTQ-like reads; Table 2's four-corpus spread): ratio, commands
            and matches per block, copied share, token depth median / p99 /
            max (the genome vs reads depth tails), decode GB/s and split.
  seek      Single-request seeks into a resident DNA archive ("Random Access
            at Scale", the reconciling model's F + c * tokens): 16 KiB reads
            by position decile, widths of 1 to 1000 blocks, the least-squares
            fit over all reads, and an equal-token-mass control on a 254 MB
            archive (the read's closure matches above a depth forced to
            literals, the same number of leaf matches, or none).

  streamdiff  (host only) the depth cap's stream-diff invariant at full size
            with the oracle encoder: the blocks whose payloads differ between
            the uncapped and capped archives are exactly those holding a
            forced position.

Usage: python studies.py {depth,minmatch,corpora,seek,streamdiff} [options]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

B = 16384


def log(*a):
    print("[study]", *a, file=sys.stderr, flush=True)


def emit(obj):
    print(json.dumps(obj), flush=True)


def timed_decode(torch, ax, arc, x, steps=10, warmup=2, options=None):
    """Whole-archive decode of `arc` (checked against x first): ms per decode
    from events around `steps` back-to-back decodes, then the library's stage
    split averaged over `steps` more."""
    import xxhash

    dev = torch.device("cuda:0")
    d_arc = torch.from_numpy(arc).to(dev)
    dec = ax.Decoder(arc, d_arc)
    for k, v in (options or {}).items():
        dec.set_option(k, v)
    out = torch.empty(max(16, x.size), dtype=torch.uint8, device=dev)
    out.fill_(0xCC)
    dec.decode_all(out=out)
    err, bad = dec.status()
    got = out[: x.size].cpu().numpy()
    if err or xxhash.xxh3_64_intdigest(got.tobytes()) != xxhash.xxh3_64_intdigest(x.tobytes()) \
            or not np.array_equal(got, x):
        raise RuntimeError(f"decode mismatch (device status {err}, block {bad})")
    del got
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        dec.decode_all(out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        dec.decode_all(out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    dec.set_timing(True)
    stage = np.zeros(4)
    for _ in range(steps):
        dec.decode_all(out=out)
        stage += np.array(dec.stage_ms(remainder=True))
    dec.set_timing(False)
    stage /= steps
    del out, d_arc
    return {"ms": round(ms, 4), "gbs": round(x.size / ms / 1e6, 2),
            "ans_ms": round(stage[0], 4), "parse_ms": round(stage[1], 4), "copy_ms": round(stage[2], 4),
            "remainder_ms": round(stage[3], 4)}


def lstsq(cols, y, names):
    """Least-squares fit y = sum coef_i * col_i; coefficients and residual RMS."""
    A = np.column_stack(cols).astype(np.float64)
    coef, *_ = np.linalg.lstsq(A, np.asarray(y, np.float64), rcond=None)
    rms = float(np.sqrt(np.mean((A @ coef - y) ** 2)))
    return {**{n: float(c) for n, c in zip(names, coef)}, "rms": rms}


def enc_stats(st, n):
    return {"ratio": round(n / st.comp_bytes, 4), "commands": int(st.n_commands), "matches": int(st.n_matches),
            "match_bytes": int(st.n_match_bytes), "literal_bytes": int(st.n_lit_bytes),
            "copied_share": round(st.n_match_bytes / n, 4)}


# ----------------------------------------------------------------- depth ---

def study_depth(args):
    import torch

    import synth
    import paper_2608_10188_amd as ax

    caps = [int(c) for c in args.caps.split(",")]
    summary = {}
    for wl in args.workloads.split(","):
        x = synth.workload_input(wl)
        pts = []
        base_lit = None
        for L in caps:
            t0 = time.time()
            # an uncapped encode reports no depth: a cap above any depth runs
            # the depth pass without forcing anything (same streams)
            arc, st = ax.encode(x, stats=True, threads=args.threads, depth_cap=L if L else 65535)
            es = enc_stats(st, x.size)
            if base_lit is None and L == 0:
                base_lit = st.n_lit_bytes
            log(f"{wl} L={L or 'inf'}: encoded in {time.time() - t0:.1f}s, max depth {st.max_depth}")
            r = timed_decode(torch, ax, arc, x, args.steps, args.warmup)
            pt = {"study": "depth", "workload": wl, "cap": L or None, "max_depth": int(st.max_depth),
                  "levels": int(st.max_depth) + 1, "encode_passes": int(st.passes), **es,
                  "forced_bytes": None if base_lit is None else int(st.n_lit_bytes - base_lit),
                  "bytes_identity": int(st.n_lit_bytes + st.n_match_bytes) == x.size, **r}
            emit(pt)
            pts.append(pt)
        ms = np.array([p["ms"] for p in pts])
        lv = np.array([p["levels"] for p in pts], np.float64)
        mb = np.array([p["match_bytes"] / 1e6 for p in pts])
        one = np.ones_like(ms)
        summary[wl] = {
            "linear_levels": lstsq([one, lv, mb], ms, ["c_ms", "a_ms_per_level", "b_ms_per_copied_mb"]),
            "log_levels": lstsq([one, np.log2(lv), mb], ms, ["c_ms", "a_ms_per_log2_level", "b_ms_per_copied_mb"]),
            "ms_range": [float(ms.min()), float(ms.max())],
        }
    emit({"study": "depth", "summary": summary})


# -------------------------------------------------------------- minmatch ---

def study_minmatch(args):
    import torch

    import synth
    import paper_2608_10188_amd as ax

    for wl in args.workloads.split(","):
        x = synth.workload_input(wl)
        for m in [int(v) for v in args.min_matches.split(",")]:
            arc, st = ax.encode(x, stats=True, threads=args.threads, min_match=m)
            r = timed_decode(torch, ax, arc, x, args.steps, args.warmup)
            emit({"study": "minmatch", "workload": wl, "min_match": m, **enc_stats(st, x.size), **r})


# --------------------------------------------------------------- corpora ---

def study_corpora(args):
    import torch

    import oracle
    import synth
    import paper_2608_10188_amd as ax

    for wl in args.workloads.split(","):
        x = synth.workload_input(wl)
        arc, st = ax.encode(x, stats=True, threads=args.threads)
        t0 = time.time()
        d, dmax = oracle.depths(arc)
        log(f"{wl}: token depths in {time.time() - t0:.1f}s")
        nb = (x.size + B - 1) // B
        r = timed_decode(torch, ax, arc, x, args.steps, args.warmup)
        emit({"study": "corpora", "workload": wl, "n_bytes": int(x.size), **enc_stats(st, x.size),
              "commands_per_block": round(st.n_commands / nb, 1), "matches_per_block": round(st.n_matches / nb, 1),
              "depth_median": float(np.median(d)) if d.size else 0.0,
              "depth_p99": float(np.percentile(d, 99)) if d.size else 0.0, "depth_max": int(dmax),
              "pending_after_4_levels": int((d >= 4).sum()), **r})


# ------------------------------------------------------------------ seek ---

def one_read(torch, dec, off, ln, out, work, stream):
    torch.cuda.synchronize()
    t = time.perf_counter_ns()
    dec.decode_range(off, ln, out, work, stream=stream)
    end = torch.cuda.Event()
    end.record(stream)
    end.synchronize()
    return (time.perf_counter_ns() - t) / 1e3


def measure_reads(torch, dec, x, ranges, reps, check=True):
    """Each range read `reps` times alone (closed loop); per range the median
    latency in us, its closure (blocks, matches) and a byte check."""
    dev = dec.device
    need = max(dec.range_workspace(o, ln) for o, ln in ranges)
    work = torch.empty(max(256, need), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    res = []
    for o, ln in ranges:
        out = torch.empty(ln, dtype=torch.uint8, device=dev)
        lat = [one_read(torch, dec, o, ln, out, work, stream) for _ in range(reps)]
        _, tok, nb = dec.closure_blocks([o], [ln], want_blocks=False)
        ok = (not check) or np.array_equal(out.cpu().numpy(), x[o: o + ln])
        res.append({"off": int(o), "len": int(ln), "us_p50": float(np.median(lat)), "us_min": float(min(lat)),
                    "closure_blocks": int(nb), "closure_matches": int(tok), "ok": bool(ok)})
    return res


def force_literals(cmds, pick):
    """The commands with the matches at indices `pick` turned into literal
    commands, and every repeat match written as an explicit match with the
    source it resolved to (a forced match no longer enters the distance
    history, so history-relative commands after it would change meaning)."""
    out = cmds.copy()
    out["kind"][pick] = 0
    out["kind"][out["kind"] == 2] = 1
    out["rep"] = 0
    return out


def closure_tokens(dec, target, mpre):
    """Archive indices of the matches in the blocks of a range's closure."""
    blocks, _, _ = dec.closure_blocks([target[0]], [target[1]])
    b = blocks.astype(np.int64)
    return np.concatenate([np.arange(mpre[k], mpre[k + 1], dtype=np.int64) for k in b]) if b.size else \
        np.zeros(0, np.int64)


def study_seek(args):
    import torch

    import oracle
    import synth
    import paper_2608_10188_amd as ax

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(91)
    # (1)-(3) on a large archive
    n = int(args.bytes)
    t0 = time.time()
    marks = set()

    def progress(done, total, what):
        g = done * 8 // max(1, total)
        if (what, g) not in marks:
            marks.add((what, g))
            log(f"{what} {done >> 20} of {total >> 20} MiB in {time.time() - t0:.0f}s")

    x = synth.dna_segmented(n, 5, threads=16, progress=lambda d, t: progress(d, t, "generated"))
    log(f"generated {n} B in {time.time() - t0:.1f}s")
    t0 = time.time()
    arc = ax.encode(x, window_log=30 if n >= (1 << 32) else 0, threads=args.threads,
                    progress=lambda d, t: progress(d, t, "encoded"))
    log(f"encoded to {arc.size} B in {time.time() - t0:.1f}s")
    dec = ax.Decoder(arc, torch.from_numpy(arc).to(dev))
    dec.build_index()
    dec._work = None
    torch.cuda.empty_cache()
    nb = n // B
    deciles = []
    for q in range(10):
        lo, hi = q * nb // 10, (q + 1) * nb // 10 - 2
        rs = [(int(b) * B + int(rng.integers(0, B)), B) for b in rng.integers(lo, hi, args.per_decile)]
        res = measure_reads(torch, dec, x, rs, 1)
        lat = np.array([r["us_p50"] for r in res])
        pt = {"study": "seek", "part": "position", "decile": q, "reads": len(res),
              "us_p50": float(np.percentile(lat, 50)), "us_p99": float(np.percentile(lat, 99)),
              "closure_blocks_mean": float(np.mean([r["closure_blocks"] for r in res])),
              "closure_matches_mean": float(np.mean([r["closure_matches"] for r in res])),
              "mismatches": int(sum(not r["ok"] for r in res))}
        emit(pt)
        deciles.append((pt, res))
    widths = []
    for w in (1, 10, 100, 1000):
        rs = [(int(b) * B, w * B) for b in rng.integers(0, nb - w, args.per_width)]
        res = measure_reads(torch, dec, x, rs, 3)
        pt = {"study": "seek", "part": "width", "blocks": w, "reads": len(res),
              "us_p50": float(np.median([r["us_p50"] for r in res])),
              "closure_blocks_mean": float(np.mean([r["closure_blocks"] for r in res])),
              "closure_matches_mean": float(np.mean([r["closure_matches"] for r in res])),
              "mismatches": int(sum(not r["ok"] for r in res))}
        emit(pt)
        widths.append((pt, res))
    allr = [r for _, res in deciles + widths for r in res]
    tok = np.array([r["closure_matches"] for r in allr], np.float64)
    us = np.array([r["us_p50"] for r in allr])
    fit = lstsq([np.ones_like(tok), tok], us, ["F_us", "c_us_per_token"])
    pos = [p["us_p50"] for p, _ in deciles]
    del dec, x, arc
    torch.cuda.empty_cache()

    # (4) equal-token-mass control on the 254 MB DNA workload: the block whose
    # own matches reach deepest is read whole from three archives of the same
    # bytes: its closure's matches deeper than --cut-depth forced to literals
    # (A), as many leaf matches (depth 0) forced (B), or none (C)
    x = synth.workload_input("dna254")
    arc0 = ax.encode(x, threads=args.threads)
    depth, _ = oracle.depths(arc0)
    nbk = int(oracle.info(arc0).n_blocks)
    mpre = np.frombuffer(arc0[64 + 8 * (nbk + 1): 64 + 16 * (nbk + 1)].tobytes(), "<u8").astype(np.int64)
    tblk = np.searchsorted(mpre, np.arange(depth.size), side="right") - 1
    deepest = np.zeros(nbk, np.int64)
    np.maximum.at(deepest, tblk, depth.astype(np.int64))
    tb = int(np.argmax(deepest))
    target = (tb * B, min(B, x.size - tb * B))
    cmds = oracle.parse_all(arc0)
    mi = np.nonzero(cmds["kind"] > 0)[0]  # command index of match t (archive order)
    dec0 = ax.Decoder(arc0, torch.from_numpy(arc0).to(dev))
    dec0.build_index()
    clo = closure_tokens(dec0, target, mpre)
    del dec0
    # A cuts every chain of the closure above depth `cut_depth`; B forces as
    # many leaf matches (depth 0), so both remove the same token mass
    deep = clo[depth[clo] > args.cut_depth]
    leaves = clo[depth[clo] == 0]
    leaf = leaves[rng.choice(leaves.size, min(deep.size, leaves.size), replace=False)] if leaves.size else leaves
    control = {}
    for name, pick in (("A_deep", mi[deep]), ("B_leaf", mi[leaf]), ("C_placebo", mi[:0])):
        arc = oracle.assemble(x, force_literals(cmds, pick))
        d2, dm2 = oracle.depths(arc)
        mp2 = np.frombuffer(arc[64 + 8 * (nbk + 1): 64 + 16 * (nbk + 1)].tobytes(), "<u8").astype(np.int64)
        dec = ax.Decoder(arc, torch.from_numpy(arc).to(dev))
        dec.build_index()
        c2 = closure_tokens(dec, target, mp2)
        res = measure_reads(torch, dec, x, [target], args.control_reps)[0]
        control[name] = {"forced_tokens": int(pick.size), "closure_blocks": res["closure_blocks"],
                         "closure_matches": res["closure_matches"],
                         "closure_max_depth": int(d2[c2].max()) if c2.size else 0, "archive_max_depth": int(dm2),
                         "us_p50": res["us_p50"], "us_min": res["us_min"], "ok": res["ok"]}
        emit({"study": "seek", "part": "control", "variant": name, "target_block": tb, **control[name]})
        del dec
    emit({"study": "seek", "summary": {"archive_bytes_n": n, "fit": fit,
                                        "position_p50_us": {"min": min(pos), "max": max(pos),
                                                            "spread": (max(pos) - min(pos)) / float(np.median(pos))},
                                        "width_p50_us": {p["blocks"]: p["us_p50"] for p, _ in widths},
                                        "control": control}})


# ------------------------------------------------------------ streamdiff ---

def study_streamdiff(args):
    """The depth cap's stream-diff invariant at full size, on the host (no
    GPU): with the oracle encoder, the blocks whose payload bytes differ
    between the uncapped and the capped archive are exactly the blocks that
    hold a forced position, and both archives decode to the input."""
    import oracle
    import synth

    for wl in args.workloads.split(","):
        x = synth.workload_input(wl)
        for L in [int(c) for c in args.caps.split(",") if int(c)]:
            t0 = time.time()
            a0, _ = oracle.encode(x)
            a1, st, forced = oracle.encode_forced(x, depth_cap=L)
            nb = int(oracle.info(a0).n_blocks)
            o0 = np.frombuffer(a0[64: 64 + 8 * (nb + 1)].tobytes(), "<u8").astype(np.int64)
            o1 = np.frombuffer(a1[64: 64 + 8 * (nb + 1)].tobytes(), "<u8").astype(np.int64)
            h0, h1 = 64 + 16 * (nb + 1), 64 + 16 * (nb + 1)
            differ = np.array([not np.array_equal(a0[h0 + o0[b]: h0 + o0[b + 1]], a1[h1 + o1[b]: h1 + o1[b + 1]])
                               for b in range(nb)])
            pad = np.zeros(nb * B, np.uint8)
            pad[: x.size] = forced
            holds = pad.reshape(nb, B).any(axis=1)
            ok = bool(np.array_equal(oracle.decode(a1), x))
            emit({"study": "streamdiff", "workload": wl, "cap": L, "blocks": nb, "forced_bytes": int(forced.sum()),
                  "blocks_with_forced": int(holds.sum()), "blocks_differing": int(differ.sum()),
                  "invariant": bool(np.array_equal(differ, holds)), "capped_max_depth": int(st.max_depth),
                  "decodes_to_input": ok, "seconds": round(time.time() - t0, 1)})


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("study", choices=["depth", "minmatch", "corpora", "seek", "streamdiff"])
    ap.add_argument("--workloads", default=None)
    ap.add_argument("--caps", default="0,64,32,24,16")
    ap.add_argument("--min-matches", default="4,6,8,12,16,24,32")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--bytes", type=float, default=32 * 2 ** 30, help="seek: archive size")
    ap.add_argument("--per-decile", type=int, default=100)
    ap.add_argument("--per-width", type=int, default=10)
    ap.add_argument("--cut-depth", type=int, default=4, help="seek control: closure matches deeper than this are forced")
    ap.add_argument("--control-reps", type=int, default=200)
    args = ap.parse_args()
    defaults = {"depth": "dna254,text200", "minmatch": "dna254,text200",
                "corpora": "dna254,text200,protein254,reads254", "seek": "", "streamdiff": "dna254"}
    if args.workloads is None:
        args.workloads = defaults[args.study]
    {"depth": study_depth, "minmatch": study_minmatch, "corpora": study_corpora, "seek": study_seek,
     "streamdiff": study_streamdiff}[args.study](args)


if __name__ == "__main__":
    main()

"""Benchmark: encode + decode throughput of the integer octree codec on one MI355X.

One step = encode one synthetic 64-beam frame (14-level octree, C = 32 int8
model) and decode it again, inputs and outputs resident in HBM.  The frames
cycle through the 8 seeded scans of that workload.  Reported:

* value: whole-job encode+decode Mpts/s (points / (t_enc + t_dec)) over the
  timed steps, with frames/s, per-frame p50/p99 ms, encode and decode rates;
* batched vs plain: the uneven 32-frame batch (16/32/64 beams, 14-level
  octrees, C = 32) through the batched calls against the same frames one by
  one, and 8 frames of the 128-beam, 18-level, C = 64 workload per batch;
* served: a Poisson stream of encode/decode requests from 24 simulated
  sensors (16-128 beams, 14-18 levels, C = 32/64) through the continuous-
  batching server, with p50/p99 request latency and sustained Mpts/s;
* roofline of the dominant kernel, timed with HIP events on the library's
  stream, against MI355X peaks;
* cpu_baseline: the CPU oracle on one frame of the same workload.
Every GPU stream of the timed frames is checked byte for byte against the
oracle's stream of the same frame ("bit_exact").
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# plain 32-bit VALU lane operations: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--chunk-log2", type=int, default=8)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain comparisons")
    ap.add_argument("--no-serve", action="store_true", help="skip the served (continuous batching) run")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-mode lines")
    ap.add_argument("--only-128beam", action="store_true",
                    help="run only the 128-beam batched comparison after the plain loop (profiling)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-base", action="store_true", help="skip the base-geometry lines")
    ap.add_argument("--no-schedules", action="store_true",
                    help="skip the schedule variants of the ablations")
    ap.add_argument("--no-chunks", action="store_true",
                    help="skip the range-coder chunk-size lines")
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (counter calibration under a profiler)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(frames shard across GPUs with no exchange; see the design notes)"}))
        sys.exit(2)
    import torch

    from paper_2603_25260_amd import lpcc, synth

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cfg = synth.CONFIGS["cfg2"]
    D, C = cfg.scan.D, cfg.C
    blob = synth.make_weights(cfg.weight_seed, C, D, cfg.n_deep)
    model = lpcc.Model(blob, 0)
    ctx = lpcc.Context(0, stream.cuda_stream)
    cl = args.chunk_log2

    frames = [synth.make_scan(cfg.scan, s) for s in cfg.seeds[:args.frames]]
    dxyz = [torch.from_numpy(f).to(dev) for f in frames]
    npts = [len(f) for f in frames]
    cap = max(npts) * 8 + 65536
    dbs = torch.zeros(cap, dtype=torch.uint8, device=dev)
    dout = torch.zeros((max(npts), 3), dtype=torch.int32, device=dev)

    def step(i):
        k = i % len(frames)
        t0 = time.perf_counter()
        n = lpcc.encode_frame(ctx, model, dxyz[k], cl, out=dbs)
        t1 = time.perf_counter()
        m = lpcc.decode_frame(ctx, model, dbs, length=n, out=dout)
        t2 = time.perf_counter()
        return n, m, t1 - t0, t2 - t1

    # streams of every frame (kept for the bit-exactness check), and warm-up
    lens = {}
    for k in range(len(frames)):
        n, m, _, _ = step(k)
        lens[k] = bytes(dbs[:n].cpu().numpy())
        assert m == len(np.unique(frames[k], axis=0)), "decoded point count differs"
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    enc_t, dec_t = [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        n, m, te, td = step(i)
        enc_t.append(te)
        dec_t.append(td)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    pts = sum(npts[i % len(frames)] for i in range(args.steps))
    frame_ms = np.array([(a + b) * 1e3 for a, b in zip(enc_t, dec_t)])
    res = {
        "metric": "encode+decode Mpts/s & frames/s (bit-exact); batched vs plain; p99 frame ms",
        "value": round(pts / wall / 1e6, 3),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8/i32",
        "data": "synthetic",
        "config": {"workload": "64-beam x 2048-az synthetic scan, 14-level octree (1 cm), C=32 int8, "
                               "4 re-densified depths, plain per-frame encode+decode",
                   "points_per_frame_mean": int(np.mean(npts)), "frames": len(frames),
                   "chunk_log2": cl},
        "frames_per_s": round(args.steps / wall, 2),
        "encode_mpts_s": round(pts / sum(enc_t) / 1e6, 3),
        "decode_mpts_s": round(pts / sum(dec_t) / 1e6, 3),
        "p50_frame_ms": round(float(np.percentile(frame_ms, 50)), 3),
        "p99_frame_ms": round(float(np.percentile(frame_ms, 99)), 3),
    }

    if args.calib_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # ---- kernel roofline: HIP events around every launch of one family
    fam_stats = {}
    for fam in ("predict", "conv", "rc_decode", "up", "rc_encode"):
        ctx.timing_enable(fam)
        for i in range(len(frames)):
            step(i)
        launches, ms, units = ctx.timing_read()
        fam_stats[fam] = (launches, ms, units)
    ctx.timing_enable("")
    res["kernel_ms_per_frame"] = {f: round(v[1] / len(frames), 4) for f, v in fam_stats.items()}
    launches, ms, units = fam_stats["predict"]
    # k_predict: per node, fc2 requantisation of 255 logits and the integer
    # softmax / frequency table (15 integer operations per logit) plus the
    # fc1 requantisation (6 per channel); the C^2 + 255 C MACs run on MFMA.
    ops = units * (255 * 15 + 6 * C)
    achieved = ops / (ms / 1e3) / 1e12 if ms > 0 else 0.0
    avg_ms = ms / max(launches, 1)
    traffic = None
    if _source_hash() == PROFILED_MODEL_HIP:
        traffic = int(PREDICT_BYTES_PER_LAUNCH)
    res["roofline"] = {"kernel": "k_predict", "bound": "alu", "achieved": round(achieved, 3),
                       "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s (32-bit integer lane ops)",
                       "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": traffic,
                       "launches": launches, "avg_launch_ms": round(avg_ms, 4), "nodes": units,
                       "ops_per_node": 255 * 15 + 6 * C}
    # the longest kernel by time is the serial range decoder (latency bound:
    # one chunk of 2^c symbols per wave, one symbol after the other)
    dl, dms, dunits = fam_stats["rc_decode"]
    res["range_decoder"] = {"kernel": "k_rc_decode", "ms_per_frame": round(dms / len(frames), 4),
                            "symbols_per_chunk": 1 << cl, "launches": dl,
                            "avg_launch_ms": round(dms / max(dl, 1), 4),
                            "ns_per_serial_symbol": round(dms * 1e6 / max(dl, 1) / (1 << cl), 1),
                            "cdf_row_gbs": round(dunits * 512 / (dms / 1e3) / 1e9, 1) if dms > 0 else None}

    if args.only_128beam:
        res["batched_128beam"] = _bench_128beam(lpcc, synth, torch, dev, ctx)
        print(json.dumps(res))
        return

    # ---- graph mode: the same plain loop with every launch batch captured
    # into HIP graphs and replayed (executable graphs updated in place)
    gctx = lpcc.Context(0, stream.cuda_stream)
    gctx.set_graphs(True)

    def gstep(i):
        k = i % len(frames)
        n = lpcc.encode_frame(gctx, model, dxyz[k], cl, out=dbs)
        lpcc.decode_frame(gctx, model, dbs, length=n, out=dout)
        return n

    if not args.no_graph:
        for i in range(2 * len(frames)):
            n = gstep(i)
            if i < len(frames):
                assert bytes(dbs[:n].cpu().numpy()) == lens[i], "graph-mode stream differs"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            gstep(i)
        torch.cuda.synchronize()
        gw = time.perf_counter() - t0
        res["graph_mode"] = {"value": round(pts / gw / 1e6, 3), "unit": "Mpts/s",
                             "ms_per_step": round(gw / args.steps * 1e3, 3), **gctx.graph_stats()}

    # ---- PCIe-inclusive rate: host coordinates in, host bytes out, and back
    t0 = time.perf_counter()
    for k in range(len(frames)):
        hb = lpcc.encode_frame(ctx, model, frames[k], cl)
        lpcc.decode_frame(ctx, model, hb)
    res["host_io_mpts_s"] = round(sum(npts) / (time.perf_counter() - t0) / 1e6, 3)

    # ---- bit-exactness of the timed streams against the oracle, and the
    # oracle's own rate on the host cores: P frames, one per thread (the
    # oracle is C called through ctypes, which releases the interpreter lock)
    if not args.no_cpu:
        from concurrent.futures import ThreadPoolExecutor

        from oracle import oracle as O
        P = min(3, len(frames), os.cpu_count() or 1)

        def one(k):
            a = time.perf_counter()
            ref = O.encode(blob, frames[k], cl)
            b = time.perf_counter()
            dec = O.decode(blob, ref)
            return ref, dec, b - a, time.perf_counter() - b

        O.lut()  # the oracle builds its exponent table on first use: once, before the threads
        t0 = time.perf_counter()
        with ThreadPoolExecutor(P) as ex:
            outs = list(ex.map(one, range(P)))
        wall = time.perf_counter() - t0
        res["bit_exact"] = all(outs[k][0] == lens[k] and len(outs[k][1]) == len(np.unique(frames[k], axis=0))
                               for k in range(P))
        res["stream_bytes_per_point"] = round(len(outs[0][0]) / npts[0], 3)
        te = np.mean([o[2] for o in outs])
        td = np.mean([o[3] for o in outs])
        res["cpu_baseline"] = {"value": round(sum(npts[:P]) / wall / 1e6, 4), "unit": "Mpts/s", "cores": P,
                               "kind": "oracle",
                               "sample": f"{P} frames ({sum(npts[:P])} points) of the same workload, one per "
                                         f"thread, encode + decode in {wall:.1f} s wall; per frame encode "
                                         f"{te:.1f} s + decode {td:.1f} s, single-threaded C each"}

    # ---- batched vs plain on the uneven 32-frame batch
    if not args.no_batch:
        bframes = [synth.make_scan(synth.batch_scan_spec(s), s) for s in range(3001, 3033)]
        bd = [torch.from_numpy(f).to(dev) for f in bframes]
        bcap = [len(f) * 8 + 65536 for f in bframes]
        bouts = [torch.zeros(c_, dtype=torch.uint8, device=dev) for c_ in bcap]
        bdec = [torch.zeros((len(f), 3), dtype=torch.int32, device=dev) for f in bframes]
        bpts = sum(len(f) for f in bframes)
        # warm
        ln, st = lpcc.encode_batch(ctx, model, bd, cl, outs=bouts)
        lpcc.decode_batch(ctx, model, bouts, lengths=ln, outs=bdec)
        reps = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ln, st = lpcc.encode_batch(ctx, model, bd, cl, outs=bouts)
            nout, st2 = lpcc.decode_batch(ctx, model, bouts, lengths=ln, outs=bdec)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        assert st == [0] * 32 and st2 == [0] * 32
        t0 = time.perf_counter()
        plain_lens = []
        for _ in range(reps):
            plain_lens = []
            for i in range(32):
                n = lpcc.encode_frame(ctx, model, bd[i], cl, out=dbs)
                plain_lens.append(n)
                lpcc.decode_frame(ctx, model, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / reps
        # the batch again with its launch batches captured into graphs
        gctx.set_graphs(not args.no_graph)
        lpcc.encode_batch(gctx, model, bd, cl, outs=bouts)
        lg, _ = lpcc.encode_batch(gctx, model, bd, cl, outs=bouts)
        lpcc.decode_batch(gctx, model, bouts, lengths=lg, outs=bdec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            lg, _ = lpcc.encode_batch(gctx, model, bd, cl, outs=bouts)
            lpcc.decode_batch(gctx, model, bouts, lengths=lg, outs=bdec)
        torch.cuda.synchronize()
        tg = (time.perf_counter() - t0) / reps
        res["batched"] = {"workload": "32 uneven frames (16/32/64 beams, 1024-2048 az), 14-level, C=32",
                          "points": bpts, "batched_mpts_s": round(bpts / tb / 1e6, 3),
                          "batched_graph_mpts_s": round(bpts / tg / 1e6, 3),
                          "plain_mpts_s": round(bpts / tp / 1e6, 3), "speedup": round(tp / tb, 3),
                          "same_lengths": plain_lens == ln and lg == ln}
        res["batched_128beam"] = _bench_128beam(lpcc, synth, torch, dev, ctx)
    if not args.no_schedules:
        res["schedules"] = _bench_schedules(lpcc, synth, torch, dev, ctx, frames, dxyz, cl, dbs, dout)
    if not args.no_base:
        res["base_geometry"] = _bench_base(lpcc, torch, model, frames, dxyz, cl, dbs, dout, D - cfg.n_deep - 1)
    if not args.no_chunks:
        res["chunk_sizes"] = _bench_chunks(lpcc, torch, ctx, model, frames, dxyz, dbs, dout)
    if not args.no_serve:
        from paper_2603_25260_amd import serve
        rep_ = serve.run(duration_s=args.serve_seconds, n_sensors=24, rate_hz=10.0, seed=5000, slots=4,
                         max_batch=4, chunk_log2=cl, frames_per_sensor=1, verify=False, realtime=True)
        res["served"] = {"workload": "Poisson arrivals, 24 sensors x 10 Hz, 16-128 beams, 14-18 levels, "
                                     "C=32 (D<=16) / 64, 50% encode / 50% decode",
                         "seconds": args.serve_seconds, **{k: rep_[k] for k in (
                             "requests", "ok", "p50_ms", "p99_ms", "sustained_mpts_s", "offered_req_s",
                             "mean_batch", "slots", "max_batch")}}
    print(json.dumps(res))


def _bench_128beam(lpcc, synth, torch, dev, ctx):
    """8 frames of the 128-beam, 18-level (1 mm), C = 64 workload: batched
    (one launch per level family for all 8) against the plain per-frame path;
    the stream of the first frame is checked against the oracle's digest."""
    import hashlib
    cfg = synth.CONFIGS["cfg4"]
    D, C = cfg.scan.D, cfg.C
    model = lpcc.Model(synth.make_weights(cfg.weight_seed, C, D, cfg.n_deep), 0)
    frames = [synth.make_scan(cfg.scan, s) for s in cfg.seeds[:8]]
    bd = [torch.from_numpy(f).to(dev) for f in frames]
    pts = sum(len(f) for f in frames)
    outs = [torch.zeros(len(f) * 8 + 65536, dtype=torch.uint8, device=dev) for f in frames]
    decs = [torch.zeros((len(f), 3), dtype=torch.int32, device=dev) for f in frames]
    ln, st = lpcc.encode_batch(ctx, model, bd, 8, outs=outs)
    lpcc.decode_batch(ctx, model, outs, lengths=ln, outs=decs)
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ln, st = lpcc.encode_batch(ctx, model, bd, 8, outs=outs)
        nout, st2 = lpcc.decode_batch(ctx, model, outs, lengths=ln, outs=decs)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    assert st == [0] * 8 and st2 == [0] * 8
    t0 = time.perf_counter()
    for _ in range(reps):
        for i in range(8):
            n = lpcc.encode_frame(ctx, model, bd[i], 8, out=outs[i])
            lpcc.decode_frame(ctx, model, outs[i], length=n, out=decs[i])
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / reps
    exact = None
    dig = os.path.join(ROOT, "tests", "golden", "digests.json")
    if os.path.exists(dig):
        want = json.load(open(dig)).get("cfg4", {}).get(str(cfg.seeds[0]))
        if want:
            got = hashlib.sha256(bytes(outs[0][:ln[0]].cpu().numpy())).hexdigest()
            exact = got == want["stream_c8"]["sha256"]
    return {"workload": "8 frames, 128-beam x 2048-az, 18-level octree (1 mm), C=64, 5 re-densified depths",
            "points": pts, "batched_mpts_s": round(pts / tb / 1e6, 3), "plain_mpts_s": round(pts / tp / 1e6, 3),
            "speedup": round(tp / tb, 3), "batched_ms_per_frame": round(tb / 8 * 1e3, 3),
            "bit_exact_first_frame": exact}


def _bench_schedules(lpcc, synth, torch, dev, ctx, frames, dxyz, cl, dbs, dout):
    """Plain encode+decode of the same 64-beam frames under the schedule
    variants of the paper's ablations, each its own seeded model: the
    threshold t = L - n_deep with n_deep = 3, 4 (the default) and 5, and the
    module ablation without cross-scale propagation, with re-densification
    (+GRED, n_deep = 4) and without (the baseline, n_deep = 0)."""
    cfg = synth.CONFIGS["cfg2"]
    out = []
    for nd, xfp in ((3, True), (4, True), (5, True), (4, False), (0, False)):
        m = lpcc.Model(synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, nd, xfp=xfp), 0)
        lens = []
        for k in range(len(frames)):  # warm-up (and the first call's tile tuning)
            n = lpcc.encode_frame(ctx, m, dxyz[k], cl, out=dbs)
            lpcc.decode_frame(ctx, m, dbs, length=n, out=dout)
            lens.append(n)
        reps = 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for k in range(len(frames)):
                n = lpcc.encode_frame(ctx, m, dxyz[k], cl, out=dbs)
                lpcc.decode_frame(ctx, m, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        pts = sum(len(f) for f in frames)
        name = ("GRED+XFP" if xfp else "GRED") + f", t = L-{nd}" if nd > 0 or xfp else "baseline (no GRED, no XFP)"
        out.append({"schedule": name, "n_deep": nd, "xfp": xfp, "k0": cfg.scan.D - nd - 1,
                    "mpts_s": round(pts / wall / 1e6, 3), "ms_per_frame": round(wall / len(frames) * 1e3, 3),
                    "bytes_per_point": round(sum(lens) / pts, 3)})
    return out


def _bench_chunks(lpcc, torch, ctx, model, frames, dxyz, dbs, dout):
    """Plain encode+decode of the same 64-beam frames with range-coder chunks
    of 2^c nodes: the decoder's serial path per depth is one chunk, so a
    smaller c shortens it at the cost of a length field and a coder flush per
    chunk (c = 8 is the headline setting)."""
    out = []
    for c in (6, 7, 8, 10):
        lens = []
        for k in range(len(frames)):  # warm-up
            n = lpcc.encode_frame(ctx, model, dxyz[k], c, out=dbs)
            lpcc.decode_frame(ctx, model, dbs, length=n, out=dout)
            lens.append(n)
        reps = 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for k in range(len(frames)):
                n = lpcc.encode_frame(ctx, model, dxyz[k], c, out=dbs)
                lpcc.decode_frame(ctx, model, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        pts = sum(len(f) for f in frames)
        out.append({"chunk_log2": c, "mpts_s": round(pts / wall / 1e6, 3),
                    "ms_per_frame": round(wall / len(frames) * 1e3, 3),
                    "bytes_per_point": round(sum(lens) / pts, 4)})
    return out


def _bench_base(lpcc, torch, model, frames, dxyz, cl, dbs, dout, k0):
    """Plain encode+decode of the same 64-beam frames with the depths below B
    coded from their own code counts (the model from depth B on), for a few
    B up to the dense fusion depth k0; B = 0 is the headline path."""
    out = []
    for B in (0, 3, 6, k0):
        bctx = lpcc.Context(0, torch.cuda.current_stream().cuda_stream)
        bctx.set_base_depth(B)
        lens = []
        for k in range(len(frames)):  # warm-up and tile tuning
            n = lpcc.encode_frame(bctx, model, dxyz[k], cl, out=dbs)
            lpcc.decode_frame(bctx, model, dbs, length=n, out=dout)
            lens.append(n)
        reps = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for k in range(len(frames)):
                n = lpcc.encode_frame(bctx, model, dxyz[k], cl, out=dbs)
                lpcc.decode_frame(bctx, model, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        pts = sum(len(f) for f in frames)
        out.append({"B": B, "mpts_s": round(pts / wall / 1e6, 3), "ms_per_frame": round(wall / len(frames) * 1e3, 3),
                    "bytes_per_point": round(sum(lens) / pts, 4)})
        bctx.close()
    return out


# HBM bytes per k_predict launch (read + write, scaled FETCH_SIZE / WRITE_SIZE
# counters of profiles/64beam_D14_C32_plain_counters.md averaged over the 340
# decode-mode launches of 16 nodes per wave, 612 of 4 nodes per wave and 96
# encode-mode launches of that run) and the kernel source they were taken on;
# a changed kernel source reports traffic = null
PROFILED_MODEL_HIP = "97428f804563bbc7"
PREDICT_BYTES_PER_LAUNCH = (340 * (2354.3 + 30761.3) + 612 * (210.1 + 376.0) + 96 * (9157.3 + 966.6)) / 1048 * 1024


def _source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_2603_25260_amd", "csrc", "model.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]

if __name__ == "__main__":
    main()

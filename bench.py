"""Benchmark: encode + decode throughput of the integer octree codec on one MI355X.

Headline (``value``): the 128-beam workload (18-level octree at 1 mm, C = 64
int8 model, 5 re-densified depths), 8 frames per batched call.  One step =
one batched encode of the 8 frames and one batched decode of the 8 streams,
inputs and outputs resident in HBM; ``value`` = points / (t_enc + t_dec) in
Mpts/s over the timed steps.  Every timed step writes its own output
buffers, and afterwards every stream of every timed step is checked byte for
byte against the CPU oracle's stream of that frame (sha256 digests in
tests/golden/digests.json, written by a script that calls only the oracle)
and every decode against the sorted unique input ("bit_exact").

The same JSON line carries, each checked the same way:

* ``plain``: the 128-beam frames one by one through the per-frame calls;
* ``cfg1`` / ``cfg2``: the 16-beam (12 levels, C = 16) and 64-beam
  (14 levels, C = 32) frames through the per-frame calls;
* ``batched``: 32 frames of uneven size (16/32/64 beams, 14 levels, C = 32)
  through one batched encode + decode against the same frames one by one;
* ``served``: Poisson request streams from 24 simulated sensors (16-128
  beams, 14-18 levels, C = 32/64) through the continuous-batching server at
  the nominal load (10 Hz per sensor, 60 s), 4x that load, all requests of a
  trace at once (capacity), and the nominal load under a 512 MiB budget;
* ``roofline``: the kernel family with the most GPU time in a headline step,
  timed with HIP events on the library's stream, its algorithmic work (the
  method's own MACs, bytes and integer operations: present neighbour pairs
  and occupied children only, counted from the input by ``octree_stats``)
  against MI355X peaks; ``roofline_families`` gives every family;
* ``cpu_baseline``: the CPU oracle on slices of the same frames, one worker
  process per host core of this process's CPU set (at most 16);
* schedule variants, base depths, range-coder chunk sizes, graph mode and
  level-aware parameter sharing on the 64-beam frames.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_I8_PEAK_TOPS = 5000.0
# plain 32-bit VALU lane operations: 256 CUs x 64 lanes per clock x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
CHUNK = 8  # range-coder chunks of 2^8 nodes (the oracle digests use the same)
DIGESTS = os.path.join(ROOT, "tests", "golden", "digests.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tiling", type=int, default=0,
                    help="fix the GEMM row blocks per wave (1, 2, 4; 0 = autotuned)")
    ap.add_argument("--only-headline", action="store_true",
                    help="the headline steps and the family timings only (profiling)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the schedule, base-depth, chunk-size and graph-mode lines")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (counter calibration under a profiler)")
    ap.add_argument("--tuning-out", default="",
                    help="write the headline context's autotuner table (JSON) after the warm-up steps")
    ap.add_argument("--tuning-in", default="",
                    help="start the headline context from an autotuner table written by --tuning-out "
                         "(separate profiler passes then launch the same kernels)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# reference outputs: oracle digests and the expected decode (sorted unique
# voxels in Morton order, x the most significant bit of each triple)
# ---------------------------------------------------------------------------
def morton_np(xyz, D):
    x = xyz.astype(np.uint64)
    m = np.zeros(len(xyz), np.uint64)
    for b in range(D):
        for a, sh in ((0, 2), (1, 1), (2, 0)):
            m |= ((x[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + sh)
    return m


def expected_decode(xyz, D):
    u = np.unique(xyz, axis=0)
    return u[np.argsort(morton_np(u, D), kind="stable")]


def sha(b):
    return hashlib.sha256(b).hexdigest()


def load_digests():
    return json.load(open(DIGESTS)).get("streams", {}) if os.path.exists(DIGESTS) else {}


# ---------------------------------------------------------------------------
# algorithmic work of one frame (the method's own: present neighbour pairs,
# occupied children), counted from the input coordinates
# ---------------------------------------------------------------------------
def octree_stats(xyz, D, kmax):
    """N[d] nodes at depth d (d = 0..D) and P[j] present 3x3x3 neighbour
    pairs, the node itself included, at depth j (j = 0..kmax)."""
    v = np.unique(xyz.astype(np.int64), axis=0)
    N = np.zeros(D + 1, np.int64)
    P = np.zeros(kmax + 1, np.int64)
    for d in range(D + 1):
        c = np.unique(v >> (D - d), axis=0) if d < D else v
        N[d] = len(c)
        if d > kmax:
            continue
        key = (c[:, 0] << (2 * d)) | (c[:, 1] << d) | c[:, 2]
        key.sort()
        side = 1 << d
        tot = 0
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    q = c + np.array([dx, dy, dz])
                    ok = np.all((q >= 0) & (q < side), axis=1)
                    qk = (q[ok, 0] << (2 * d)) | (q[ok, 1] << d) | q[ok, 2]
                    pos = np.searchsorted(key, qk)
                    pos[pos >= len(key)] = 0
                    tot += int(np.count_nonzero(key[pos] == qk))
        P[d] = tot
    return N, P


def frame_work(N, P, C, D, n_deep):
    """Per-family algorithmic work of coding one frame once (the encoder and
    the decoder each do all of it): int8 MACs, compulsory HBM bytes and
    integer VALU operations.  Gathers count once per present pair, outputs
    once per row, neighbour tables 27 x 4 B per row read."""
    k0 = D - n_deep - 1
    w = {f: {"macs": 0, "bytes": 0, "ops": 0, "nodes": 0}
         for f in ("conv", "down", "skip", "emb", "up", "predict", "rc")}

    def add(f, macs=0, by=0, ops=0, nodes=0):
        w[f]["macs"] += int(macs)
        w[f]["bytes"] += int(by)
        w[f]["ops"] += int(ops)
        w[f]["nodes"] += int(nodes)

    for d in range(D):
        if 1 <= d <= k0:  # ResBlock at d-1, upsampling to d
            j = d - 1
            add("conv", 2 * P[j] * C * C, 2 * (P[j] * C + N[j] * C + 108 * N[j]) + N[j] * C)
            add("up", N[d] * (C + 8) * C, N[j] * (C + 1) + N[d] * C)
        elif d > k0:
            add("emb", N[d - 1] * 8 * C, N[d - 1] * (1 + C))
            for j in range(d - 1, k0, -1):
                add("down", N[j] * C * C, N[j] * C + N[j - 1] * (C + 5))
            add("conv", P[k0] * 3 * C * C,
                P[k0] * 2 * C + P[k0] * C + 2 * N[k0] * C + 2 * 108 * N[k0] + N[k0] * C)
            add("skip", N[k0] * 2 * C * C, N[k0] * 3 * C)
            for j in range(k0, d):
                add("up", N[j + 1] * (C + 8) * C, N[j] * (C + 5) + N[j + 1] * C)
        add("predict", N[d] * (C * C + 255 * C), N[d] * C, N[d] * 255 * 12, N[d])
        add("rc", 0, 0, 0, N[d])
    return w


def step_work(ws, stream_bytes):
    """Algorithmic work per family of one encode + one decode of the frames
    whose frame_work dicts are ``ws``.  The predictor writes 4 B per node in
    encode mode and a 510 B frequency-table row in decode mode; the range
    decoder reads that row and the stream."""
    fam = {}
    for f in ("conv", "down", "skip", "emb", "up"):
        fam[f] = {k: 2 * sum(w[f][k] for w in ws) for k in ("macs", "bytes", "ops", "nodes")}
    n = sum(w["predict"]["nodes"] for w in ws)
    p = {k: sum(w["predict"][k] for w in ws) for k in ("macs", "bytes", "ops")}
    fam["predict"] = {"macs": 2 * p["macs"], "bytes": 2 * p["bytes"] + n * (4 + 510), "ops": 2 * p["ops"],
                      "nodes": 2 * n}
    fam["rc_encode"] = {"macs": 0, "bytes": n * 4 + stream_bytes, "ops": 0, "nodes": n}
    fam["rc_decode"] = {"macs": 0, "bytes": n * 510 + stream_bytes, "ops": 0, "nodes": n}
    return fam


# bound of each family's roofline: the model stages gather rows from HBM, the
# softmax is plain integer arithmetic, the coders move frequency rows
FAMILY_BOUND = {"conv": "hbm", "down": "hbm", "skip": "hbm", "emb": "hbm", "up": "hbm", "predict": "alu",
                "rc_encode": "hbm", "rc_decode": "hbm"}


# HBM bytes per headline step and family, (read, write), from rocprofv3
# FETCH_SIZE and WRITE_SIZE over the steps after the warm-up step, scaled by
# what the same counters read for a 256 MiB device copy (fetch x2, write x1).
# They hold for the library sources whose digest is TRAFFIC_SOURCES; any other
# source tree reports traffic null.
TRAFFIC_SOURCES = "4f84387de7fb0e09"
FAMILY_TRAFFIC = {
    "conv": (5806464438, 2248017152),
    "down": (1584201319, 2081497216),
    "skip": (1708494149, 853240960),
    "emb": (3487946, 170779264),
    "up": (4595275146, 4374389462),
    "predict": (1692923554, 6725538311),
    "rc_encode": (58749844, 19132036),
    "rc_decode": (8108543862, 25131215),
    "hash": (505213627, 806670806),
    "expand": (136333824, 170685344),
    "pack": (32347899, 15933342),
}


def code_lines(text):
    """The lines of a C++ source without // comments, trailing blanks and
    empty lines (a comment edit leaves the digest unchanged)."""
    out = []
    for line in text.splitlines():
        i = line.find("//")
        if i >= 0:
            line = line[:i]
        line = line.rstrip()
        if line:
            out.append(line)
    return out


def library_sources_digest():
    """sha256[:16] of the library's sources in name order, by code_lines."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2603_25260_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), encoding="utf-8") as f:
            h.update("\n".join(code_lines(f.read())).encode())
            h.update(b"\n")
    return h.hexdigest()[:16]


def roofline_of(fam, work, launches, ms, traffic_ok=False):
    bound = FAMILY_BOUND[fam]
    s = ms / 1e3
    if bound == "alu":
        achieved, peak, unit = work["ops"] / s / 1e12, VALU_PEAK_TOPS, "Tops/s (32-bit integer lane ops)"
    else:
        achieved, peak, unit = work["bytes"] / s / 1e9, HBM_PEAK_GBS, "GB/s"
    out = {"kernel_family": fam, "bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 1),
           "unit": unit, "frac": round(achieved / peak, 4), "traffic": None, "launches": launches,
           "avg_launch_ms": round(ms / max(launches, 1), 5), "total_ms": round(ms, 3),
           "algorithmic_bytes": work["bytes"], "algorithmic_int8_macs": work["macs"],
           "algorithmic_int_ops": work["ops"]}
    if traffic_ok and fam in FAMILY_TRAFFIC and launches:
        rd, wr = FAMILY_TRAFFIC[fam]
        out["traffic"] = int((rd + wr) / launches)
        out["traffic_read"] = int(rd / launches)
        out["traffic_write"] = int(wr / launches)
        out["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        out["algorithmic_bytes_per_launch"] = int(work["bytes"] / launches)
    if work["macs"]:
        out["int8_mfma_frac"] = round(2 * work["macs"] / s / 1e12 / MFMA_I8_PEAK_TOPS, 5)
    return out


# launch families of the library (its timing names); the octree build's
# sort and level kernels are launched outside them
FAMILIES = ("conv", "down", "skip", "emb", "up", "predict", "rc_encode", "rc_decode", "hash", "expand", "pack",
            "base")


# ---------------------------------------------------------------------------
def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (frames are independent: "
                                   "several GPUs would each code their own frames, with no exchange)"}))
        sys.exit(2)
    import torch

    from paper_2603_25260_amd import lpcc, synth

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    digests = load_digests()
    cfg = synth.CONFIGS["cfg4"]
    D, C = cfg.scan.D, cfg.C
    blob = synth.make_weights(cfg.weight_seed, C, D, cfg.n_deep)
    model = lpcc.Model(blob, 0)
    ctx = lpcc.Context(0, stream.cuda_stream)
    if args.tiling:
        ctx.set_tiling(args.tiling)
    if args.tuning_in:
        with open(args.tuning_in) as fh:
            ctx.set_tuning(json.load(fh))
    frames = [synth.make_scan(cfg.scan, s) for s in cfg.seeds]
    nf = len(frames)
    dx = [torch.from_numpy(f).to(dev) for f in frames]
    npts = [len(f) for f in frames]
    pts = sum(npts)
    want = [digests.get("cfg4", {}).get(str(s)) for s in cfg.seeds]
    expect = [expected_decode(f, D) for f in frames]

    def new_outs():
        return ([torch.empty(n * 8 + 65536, dtype=torch.uint8, device=dev) for n in npts],
                [torch.empty((n, 3), dtype=torch.int32, device=dev) for n in npts])

    def batch_step(outs, decs):
        t0 = time.perf_counter()
        ln, st = lpcc.encode_batch(ctx, model, dx, CHUNK, outs=outs)
        t1 = time.perf_counter()
        nout, st2 = lpcc.decode_batch(ctx, model, outs, lengths=ln, outs=decs)
        t2 = time.perf_counter()
        if st != [0] * nf or st2 != [0] * nf:
            raise RuntimeError(f"batched call failed: {st} {st2}")
        return ln, nout, t1 - t0, t2 - t1

    def check(outs, decs, ln, nout):
        ok = True
        for k in range(nf):
            b = bytes(outs[k][:ln[k]].cpu().numpy())
            ok &= want[k] is not None and (len(b), sha(b)) == (want[k]["bytes"], want[k]["sha256"])
            ok &= nout[k] == len(expect[k]) and np.array_equal(decs[k][:nout[k]].cpu().numpy(), expect[k])
        return bool(ok)

    wo, wd = new_outs()
    for _ in range(max(args.warmup, 1)):
        ln, nout, _, _ = batch_step(wo, wd)
    warm_exact = check(wo, wd, ln, nout)
    if args.tuning_out:
        with open(args.tuning_out, "w") as fh:
            json.dump(ctx.tuning(), fh)
    stream_bytes = sum(ln)
    bufs = [new_outs() for _ in range(args.steps)]
    torch.cuda.synchronize()
    enc_t, dec_t, lens = [], [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ln, nout, te, td = batch_step(*bufs[i])
        enc_t.append(te)
        dec_t.append(td)
        lens.append((ln, nout))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    exact = warm_exact and all(check(bufs[i][0], bufs[i][1], *lens[i]) for i in range(args.steps))
    del bufs
    step_ms = np.array([(a + b) * 1e3 for a, b in zip(enc_t, dec_t)])
    tot = pts * args.steps
    res = {
        "metric": "encode+decode Mpts/s & frames/s (bit-exact); batched vs plain; p99 frame ms",
        "value": round(tot / wall / 1e6, 3),
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
        "config": {"workload": "8 frames per batched call of a 128-beam x 2048-az synthetic scan, 18-level "
                               "octree (1 mm), C=64 int8, 5 re-densified depths; encode + decode",
                   "frames_per_step": nf, "points_per_frame_mean": int(np.mean(npts)), "chunk_log2": CHUNK},
        "bit_exact": exact,
        "bit_exact_frames": nf * (args.steps + 1),
        "frames_per_s": round(nf * args.steps / wall, 2),
        "encode_mpts_s": round(tot / sum(enc_t) / 1e6, 3),
        "decode_mpts_s": round(tot / sum(dec_t) / 1e6, 3),
        "p50_step_ms": round(float(np.percentile(step_ms, 50)), 3),
        "p99_step_ms": round(float(np.percentile(step_ms, 99)), 3),
        "p99_frame_ms": round(float(np.percentile(step_ms, 99)), 3),
        "frame_ms_amortised": round(float(np.median(step_ms)) / nf, 3),
        "stream_bytes_per_point": round(stream_bytes / pts, 4),
    }
    if args.calib_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ---- roofline: HIP events around every launch of one family, over
    # two headline steps per family, against the algorithmic work
    k0 = D - cfg.n_deep - 1
    ws = [frame_work(*octree_stats(f, D, k0), C, D, cfg.n_deep) for f in frames]
    work = step_work(ws, stream_bytes)
    wo, wd = new_outs()
    fam_t = {}
    for fam in FAMILIES:
        ctx.timing_enable(fam)
        for _ in range(2):
            batch_step(wo, wd)
        launches, ms, _units = ctx.timing_read()
        fam_t[fam] = (launches // 2, ms / 2)
    ctx.timing_enable("")
    res["kernel_ms_per_step"] = {f: round(v[1], 3) for f, v in fam_t.items()}
    res["launches_per_step"] = {f: v[0] for f, v in fam_t.items()}
    src = library_sources_digest()
    res["library_sources"] = src
    fams = {f: roofline_of(f, work[f], *fam_t[f], traffic_ok=(src == TRAFFIC_SOURCES))
            for f in work if fam_t[f][0] > 0}
    dom = max(fams, key=lambda f: fams[f]["total_ms"])
    res["roofline"] = fams[dom]
    res["roofline_families"] = fams
    res["algorithmic_per_step"] = {f: {k: int(v) for k, v in work[f].items()} for f in work}
    if args.only_headline:
        print(json.dumps(res))
        return

    # ---- the same frames one by one through the per-frame calls
    res["plain"] = _plain(lpcc, torch, dev, ctx, model, frames, D, want, expect, reps=2)
    res["plain"]["batched_speedup"] = round(res["value"] / res["plain"]["mpts_s"], 3)
    for name in ("cfg1", "cfg2"):
        c_ = synth.CONFIGS[name]
        m_ = lpcc.Model(synth.make_weights(c_.weight_seed, c_.C, c_.scan.D, c_.n_deep), 0)
        fr = [synth.make_scan(c_.scan, s) for s in c_.seeds]
        res[name] = _plain(lpcc, torch, dev, ctx, m_, fr, c_.scan.D,
                           [digests.get(name, {}).get(str(s)) for s in c_.seeds],
                           [expected_decode(f, c_.scan.D) for f in fr], reps=3)
        res[name]["workload"] = {"cfg1": "16-beam x 1024-az, 12-level octree, C=16, plain per-frame",
                                 "cfg2": "64-beam x 2048-az, 14-level octree (1 cm), C=32, plain per-frame"}[name]
    res["batched"] = _batched32(lpcc, synth, torch, dev, ctx, digests)
    if not args.no_extras:
        c2 = synth.CONFIGS["cfg2"]
        m2 = lpcc.Model(synth.make_weights(c2.weight_seed, c2.C, c2.scan.D, c2.n_deep), 0)
        f2 = [synth.make_scan(c2.scan, s) for s in c2.seeds]
        d2 = [torch.from_numpy(f).to(dev) for f in f2]
        cap = max(len(f) for f in f2) * 8 + 65536
        dbs = torch.empty(cap, dtype=torch.uint8, device=dev)
        dout = torch.empty((max(len(f) for f in f2), 3), dtype=torch.int32, device=dev)
        res["graph_mode"] = _graph_mode(lpcc, torch, stream, m2, f2, d2, dbs, dout)
        res["schedules"] = _bench_schedules(lpcc, synth, torch, ctx, f2, d2, dbs, dout)
        res["base_geometry"] = _bench_base(lpcc, torch, m2, f2, d2, dbs, dout, c2.scan.D - c2.n_deep - 1)
        res["chunk_sizes"] = _bench_chunks(lpcc, torch, ctx, m2, f2, d2, dbs, dout)
        res["parameter_sharing"] = _bench_shared(lpcc, synth, torch, ctx, f2, d2, dbs, dout)
    if not args.no_serve:
        res["served"] = _served(args.serve_seconds, digests)
    if not args.no_cpu:
        res["cpu_baseline"] = _cpu_baseline(cfg, res["value"])
    print(json.dumps(res))


def _plain(lpcc, torch, dev, ctx, model, frames, D, want, expect, reps):
    """Encode + decode of every frame through the per-frame calls, all
    streams and decodes of the timed repetitions checked."""
    dx = [torch.from_numpy(f).to(dev) for f in frames]
    outs = [[torch.empty(len(f) * 8 + 65536, dtype=torch.uint8, device=dev) for f in frames] for _ in range(reps)]
    decs = [[torch.empty((len(f), 3), dtype=torch.int32, device=dev) for f in frames] for _ in range(reps)]
    for k in range(len(frames)):  # warm-up (and the first calls' tile tuning)
        n = lpcc.encode_frame(ctx, model, dx[k], CHUNK, out=outs[0][k])
        lpcc.decode_frame(ctx, model, outs[0][k], length=n, out=decs[0][k])
    torch.cuda.synchronize()
    ft, lens = [], []
    t0 = time.perf_counter()
    for r in range(reps):
        for k in range(len(frames)):
            a = time.perf_counter()
            n = lpcc.encode_frame(ctx, model, dx[k], CHUNK, out=outs[r][k])
            m = lpcc.decode_frame(ctx, model, outs[r][k], length=n, out=decs[r][k])
            ft.append(time.perf_counter() - a)
            lens.append((n, m))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ok = True
    for r in range(reps):
        for k in range(len(frames)):
            n, m = lens[r * len(frames) + k]
            b = bytes(outs[r][k][:n].cpu().numpy())
            ok &= want[k] is not None and (len(b), sha(b)) == (want[k]["bytes"], want[k]["sha256"])
            ok &= m == len(expect[k]) and np.array_equal(decs[r][k][:m].cpu().numpy(), expect[k])
    pts = reps * sum(len(f) for f in frames)
    ms = np.array(ft) * 1e3
    return {"frames": len(frames), "points": sum(len(f) for f in frames), "mpts_s": round(pts / wall / 1e6, 3),
            "frames_per_s": round(reps * len(frames) / wall, 2),
            "p50_frame_ms": round(float(np.percentile(ms, 50)), 3),
            "p99_frame_ms": round(float(np.percentile(ms, 99)), 3), "bit_exact": bool(ok),
            "bit_exact_frames": reps * len(frames)}


def _batched32(lpcc, synth, torch, dev, ctx, digests):
    """The uneven 32-frame batch (16/32/64 beams, 14 levels, C = 32) through
    one batched encode + decode, against the same frames one by one; every
    stream of both forms checked against the oracle's digests."""
    cfg = synth.CONFIGS["cfg2"]
    D = cfg.scan.D
    model = lpcc.Model(synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep), 0)
    seeds = list(range(3001, 3033))
    frames = [synth.make_scan(synth.batch_scan_spec(s), s) for s in seeds]
    want = [digests.get("cfg3", {}).get(str(s)) for s in seeds]
    expect = [expected_decode(f, D) for f in frames]
    bd = [torch.from_numpy(f).to(dev) for f in frames]
    outs = [torch.empty(len(f) * 8 + 65536, dtype=torch.uint8, device=dev) for f in frames]
    decs = [torch.empty((len(f), 3), dtype=torch.int32, device=dev) for f in frames]
    pts = sum(len(f) for f in frames)
    ln, _ = lpcc.encode_batch(ctx, model, bd, CHUNK, outs=outs)
    lpcc.decode_batch(ctx, model, outs, lengths=ln, outs=decs)
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ln, st = lpcc.encode_batch(ctx, model, bd, CHUNK, outs=outs)
        nout, st2 = lpcc.decode_batch(ctx, model, outs, lengths=ln, outs=decs)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    ok_b = st == [0] * 32 and st2 == [0] * 32
    for k in range(32):
        b = bytes(outs[k][:ln[k]].cpu().numpy())
        ok_b &= want[k] is not None and (len(b), sha(b)) == (want[k]["bytes"], want[k]["sha256"])
        ok_b &= np.array_equal(decs[k][:nout[k]].cpu().numpy(), expect[k])
    plain = _plain(lpcc, torch, dev, ctx, model, frames, D, want, expect, reps=1)
    return {"workload": "32 uneven frames (16/32/64 beams, 1024-2048 az), 14-level, C=32",
            "points": pts, "batched_mpts_s": round(pts / tb / 1e6, 3), "plain_mpts_s": plain["mpts_s"],
            "speedup": round(plain["mpts_s"] and (pts / tb / 1e6) / plain["mpts_s"], 3),
            "bit_exact": bool(ok_b and plain["bit_exact"]), "bit_exact_frames": 64,
            "batched_ms": round(tb * 1e3, 3)}


def _served(seconds, digests):
    from paper_2603_25260_amd import serve
    ref = digests.get("fleet", {})
    keys = ("requests", "ok", "encode_jobs", "decode_jobs", "p50_ms", "p99_ms", "sustained_mpts_s",
            "offered_req_s", "mean_batch", "max_in_flight", "bytes_peak", "budget_bytes", "checked", "mismatches",
            "failed")
    out = {"workload": "Poisson arrivals, 24 sensors, 16-128 beams, 14-18 levels, C=32 (D<=16) / 64, "
                       "50% encode / 50% decode; encode results checked against the oracle's digests, "
                       "decode results against the sorted unique input; 'failed' counts jobs by status "
                       "(-6: the job's workspace alone exceeds the budget)",
           "runs": []}
    for label, rate, secs, realtime, budget in (
            ("nominal: 10 Hz per sensor", 10.0, seconds, True, 0),
            ("4x nominal: 40 Hz per sensor", 40.0, min(seconds, 10.0), True, 0),
            ("capacity: every request of a 10 s nominal trace at once", 10.0, min(seconds, 10.0), False, 0),
            ("nominal under a 512 MiB budget", 10.0, min(seconds, 10.0), True, 512 << 20)):
        rep = serve.run(duration_s=secs, n_sensors=24, rate_hz=rate, seed=5000, slots=4, max_batch=4,
                        hbm_budget=budget, chunk_log2=CHUNK, frames_per_sensor=1, realtime=realtime,
                        reference=(ref, expected_decode))
        out["runs"].append({"load": label, "seconds": secs, **{k: rep.get(k) for k in keys}})
    return out


def _cpu_baseline(cfg, gpu_value):
    """The CPU oracle (single-threaded C) on slices of the headline frames:
    one worker process per core of this process's CPU set (at most 16), each
    encoding and decoding a different 16384-point slice of a 128-beam frame
    with the same model."""
    import multiprocessing as mp
    cores = min(16, len(os.sched_getaffinity(0)))
    model_name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model_name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    n_slice = 16384
    tasks = [(k % len(cfg.seeds), (k // len(cfg.seeds)) * n_slice, n_slice) for k in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        outs = pool.map(_oracle_job, tasks)
    wall = time.perf_counter() - t0
    pts = sum(o[0] for o in outs)
    te = float(np.mean([o[1] for o in outs]))
    td = float(np.mean([o[2] for o in outs]))
    v = pts / wall / 1e6
    return {"value": round(v, 5), "unit": "Mpts/s", "cores": cores, "kind": "oracle",
            "cpu_model": model_name,
            "sample": f"{cores} slices of {n_slice} points of the 128-beam frames (same C=64, 18-level model), "
                      f"one per worker process, encode + decode, {wall:.1f} s wall; one slice on one core: "
                      f"encode {te:.1f} s + decode {td:.1f} s",
            "single_core_mpts_s": round(n_slice / (te + td) / 1e6, 6),
            "gpu_over_cpu": round(gpu_value / v, 1) if v > 0 else None}


def _oracle_job(task):
    fi, start, n = task
    from oracle import oracle as O
    from paper_2603_25260_amd import synth
    cfg = synth.CONFIGS["cfg4"]
    blob = synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[fi])[start:start + n]
    O.lut()
    a = time.perf_counter()
    bs = O.encode(blob, xyz, CHUNK)
    b = time.perf_counter()
    O.decode(blob, bs)
    return len(xyz), b - a, time.perf_counter() - b


def _graph_mode(lpcc, torch, stream, model, frames, dx, dbs, dout):
    """The 64-beam frames one by one with every launch batch captured into
    HIP graphs and replayed (executable graphs updated in place), against
    the same loop with direct launches."""
    gctx = lpcc.Context(0, stream.cuda_stream)
    dctx = lpcc.Context(0, stream.cuda_stream)
    out = {}
    for name, c in (("direct", dctx), ("graph", gctx)):
        c.set_graphs(name == "graph")
        for k in range(2 * len(frames)):
            n = lpcc.encode_frame(c, model, dx[k % len(frames)], CHUNK, out=dbs)
            lpcc.decode_frame(c, model, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(2 * len(frames)):
            n = lpcc.encode_frame(c, model, dx[k % len(frames)], CHUNK, out=dbs)
            lpcc.decode_frame(c, model, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        out[name + "_mpts_s"] = round(2 * sum(len(f) for f in frames) / (time.perf_counter() - t0) / 1e6, 3)
    out.update(gctx.graph_stats())
    gctx.close()
    dctx.close()
    return out


def _bench_schedules(lpcc, synth, torch, ctx, frames, dxyz, dbs, dout):
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
            n = lpcc.encode_frame(ctx, m, dxyz[k], CHUNK, out=dbs)
            lpcc.decode_frame(ctx, m, dbs, length=n, out=dout)
            lens.append(n)
        reps = 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for k in range(len(frames)):
                n = lpcc.encode_frame(ctx, m, dxyz[k], CHUNK, out=dbs)
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


def _bench_shared(lpcc, synth, torch, ctx, frames, dxyz, dbs, dout):
    """Level-aware parameter sharing: blob sizes of the per-depth and the
    shared models (64-beam C = 32 and 128-beam C = 64 workloads), and the
    64-beam frames encoded and decoded with each."""
    out = {}
    for name in ("cfg2", "cfg4"):
        c = synth.CONFIGS[name]
        out[f"blob_bytes_{name}"] = {
            "per_depth": len(synth.make_weights(c.weight_seed, c.C, c.scan.D, c.n_deep)),
            "shared": len(synth.make_weights(c.weight_seed, c.C, c.scan.D, c.n_deep, shared=True))}
    c = synth.CONFIGS["cfg2"]
    for label, sh in (("per_depth", False), ("shared", True)):
        m = lpcc.Model(synth.make_weights(c.weight_seed, c.C, c.scan.D, c.n_deep, shared=sh), 0)
        for k in range(len(frames)):
            n = lpcc.encode_frame(ctx, m, dxyz[k], CHUNK, out=dbs)
            lpcc.decode_frame(ctx, m, dbs, length=n, out=dout)
        reps = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for k in range(len(frames)):
                n = lpcc.encode_frame(ctx, m, dxyz[k], CHUNK, out=dbs)
                lpcc.decode_frame(ctx, m, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        out[f"{label}_mpts_s_64beam"] = round(sum(len(f) for f in frames) / wall / 1e6, 3)
    return out


def _bench_base(lpcc, torch, model, frames, dxyz, dbs, dout, k0):
    """Plain encode+decode of the same 64-beam frames with the depths below B
    coded from their own code counts (the model from depth B on), for a few
    B up to the dense fusion depth k0; B = 0 is the model at every depth."""
    out = []
    for B in (0, 3, 6, k0):
        bctx = lpcc.Context(0, torch.cuda.current_stream().cuda_stream)
        bctx.set_base_depth(B)
        lens = []
        for k in range(len(frames)):  # warm-up and tile tuning
            n = lpcc.encode_frame(bctx, model, dxyz[k], CHUNK, out=dbs)
            lpcc.decode_frame(bctx, model, dbs, length=n, out=dout)
            lens.append(n)
        reps = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for k in range(len(frames)):
                n = lpcc.encode_frame(bctx, model, dxyz[k], CHUNK, out=dbs)
                lpcc.decode_frame(bctx, model, dbs, length=n, out=dout)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        pts = sum(len(f) for f in frames)
        out.append({"B": B, "mpts_s": round(pts / wall / 1e6, 3), "ms_per_frame": round(wall / len(frames) * 1e3, 3),
                    "bytes_per_point": round(sum(lens) / pts, 4)})
        bctx.close()
    return out


if __name__ == "__main__":
    main()

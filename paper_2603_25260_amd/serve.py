"""Serving driver: a Poisson request stream from many simulated sensors into
the continuous-batching server of the library (lpcc_server_*).

Each sensor has its own beam count and octree depth; sensors with D <= 16 use
the C = 32 model of their depth, deeper ones the C = 64 model.  Requests are
half encode jobs (a fresh scan of the sensor) and half decode jobs (a stream
the server encoded earlier for that sensor).  Inputs and outputs live in
device memory.  The driver submits each job at its arrival time, collects
completions, and reports p50 / p99 latency (arrival -> completion) and the
sustained point rate; with ``verify`` every result is compared with the same
job run alone through the per-frame calls, and with ``reference`` = (digests,
expect) every encode result with the sha256 digest of the oracle's stream of
that frame (keyed "sensor_frame") and every decode result with expect(xyz, D).
"""
from __future__ import annotations

import dataclasses
import hashlib
import time

import numpy as np

from . import lpcc, synth


@dataclasses.dataclass
class Sensor:
    idx: int
    beams: int
    D: int
    model: int                  # index into the server's model list
    frames: list                # host int32 [n, 3] scans
    dframes: list = None        # device tensors
    streams: list = None        # device uint8 streams of encoded frames
    stream_len: list = None


def build_fleet(n_sensors=24, seed=5000, frames_per_sensor=2, depths=(14, 15, 16, 17, 18),
                beams=(16, 32, 64, 128), azimuths=2048):
    spec = synth.fleet_spec(n_sensors, seed, depths, beams)
    keys = sorted({synth.fleet_model(D) for _, D in spec})
    sensors = []
    for i, (b, D) in enumerate(spec):
        scan = synth.fleet_scan_spec(b, D, azimuths)
        frames = [synth.make_scan(scan, synth.fleet_frame_seed(seed, i, k)) for k in range(frames_per_sensor)]
        sensors.append(Sensor(i, b, D, keys.index(synth.fleet_model(D)), frames))
    return keys, sensors


def poisson_trace(n_sensors, rate_hz, duration_s, seed, enc_frac=0.5):
    """Arrival times (s), sensor index and kind (0 encode / 1 decode)."""
    rng = np.random.default_rng(seed)
    total_rate = n_sensors * rate_hz
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / total_rate)
        if t >= duration_s:
            break
        out.append((t, int(rng.integers(n_sensors)), 0 if rng.random() < enc_frac else 1))
    return out


def run(duration_s=5.0, n_sensors=24, rate_hz=10.0, seed=5000, slots=4, max_batch=4, hbm_budget=0,
        chunk_log2=8, frames_per_sensor=2, verify=False, depths=(14, 15, 16, 17, 18), beams=(16, 32, 64, 128),
        azimuths=2048, realtime=True, reference=None):
    import torch

    dev = torch.device("cuda:0")
    keys, sensors = build_fleet(n_sensors, seed, frames_per_sensor, depths, beams, azimuths)
    models = [lpcc.Model(synth.make_weights(1, C, D, nd), 0) for (C, D, nd) in keys]
    ctx = lpcc.Context(0)
    # device inputs; streams for decode jobs made by earlier encodes
    for s in sensors:
        s.dframes = [torch.from_numpy(f).to(dev) for f in s.frames]
        s.streams, s.stream_len = [], []
        for f in s.dframes:
            buf = torch.zeros(int(f.shape[0]) * 8 + 65536, dtype=torch.uint8, device=dev)
            n = lpcc.encode_frame(ctx, models[s.model], f, chunk_log2, out=buf)
            s.streams.append(buf)
            s.stream_len.append(n)
    torch.cuda.synchronize()
    trace = poisson_trace(n_sensors, rate_hz, duration_s, seed)
    # per-job output buffers (kept until completion)
    jobs = []
    for k, (t, si, kind) in enumerate(trace):
        s = sensors[si]
        fi = k % len(s.frames)
        if kind == 0:
            out = torch.zeros(int(s.dframes[fi].shape[0]) * 8 + 65536, dtype=torch.uint8, device=dev)
        else:
            out = torch.zeros((int(s.dframes[fi].shape[0]), 3), dtype=torch.int32, device=dev)
        jobs.append((t, si, kind, fi, out))
    server = lpcc.Server(models, 0, slots=slots, max_batch=max_batch, hbm_budget=hbm_budget)
    tickets = {}
    done = []
    t0 = time.monotonic_ns()
    for (t, si, kind, fi, out) in jobs:
        s = sensors[si]
        arrive = t0 + int(t * 1e9)
        if realtime:
            while True:
                now = time.monotonic_ns()
                if now >= arrive:
                    break
                done += server.poll(256, 0)
                if arrive - now > 200_000:
                    time.sleep((arrive - now) / 2e9)
        else:
            arrive = time.monotonic_ns()
        if kind == 0:
            tk = server.submit(0, s.model, s.dframes[fi], out, chunk_log2=chunk_log2, t_arrival_ns=arrive)
        else:
            tk = server.submit(1, s.model, s.streams[fi], out, in_len=s.stream_len[fi], t_arrival_ns=arrive)
        tickets[tk] = (si, kind, fi, out)
    server.drain()
    done += server.poll(100000, 0)
    wall = (time.monotonic_ns() - t0) / 1e9
    stats = server.stats()
    lat = np.array([(d["t_done_ns"] - d["t_arrival_ns"]) / 1e6 for d in done])
    # most jobs on the GPU at one time (start -> done intervals overlapping)
    ev = sorted([(d["t_start_ns"], 1) for d in done] + [(d["t_done_ns"], -1) for d in done])
    run_, max_run = 0, 0
    for _, e in ev:
        run_ += e
        max_run = max(max_run, run_)
    pts = sum(d["n_points"] for d in done if d["status"] == 0)
    rep = {
        "requests": len(done),
        "ok": sum(d["status"] == 0 for d in done),
        "encode_jobs": sum(d["kind"] == 0 for d in done),
        "decode_jobs": sum(d["kind"] == 1 for d in done),
        "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
        "failed": {str(c): sum(d["status"] == c for d in done) for c in sorted({d["status"] for d in done}) if c != 0},
        "mean_batch": round(float(np.mean([d["batch"] for d in done])), 2) if done else None,
        "max_in_flight": max_run,
        "sustained_mpts_s": round(pts / wall / 1e6, 3),
        "server_mpts_s": round(stats["mpts_per_s"], 3),
        "offered_req_s": round(len(trace) / duration_s, 1),
        "wall_s": round(wall, 3),
        "models": [f"C{C}_D{D}" for (C, D, _) in keys],
        "slots": slots, "max_batch": max_batch,
        "budget_bytes": int(stats["bytes_budget"]),
        "bytes_peak": int(stats["bytes_peak"]),
    }
    if verify:
        mism = 0
        for d in done:
            si, kind, fi, out = tickets[d["ticket"]]
            s = sensors[si]
            if d["status"] != 0:
                mism += 1
                continue
            if kind == 0:
                ref = lpcc.encode_frame(ctx, models[s.model], s.dframes[fi], chunk_log2)
                got = out[:d["out_len"]].cpu().numpy().tobytes()
                mism += got != ref
            else:
                ref = lpcc.decode_frame(ctx, models[s.model], s.streams[fi], length=s.stream_len[fi])
                got = out[:d["out_len"]].cpu().numpy()
                mism += not np.array_equal(got, ref)
        rep["mismatches_vs_alone"] = int(mism)
    if reference is not None:
        digests, expect = reference
        mism, checked, exp_cache = 0, 0, {}
        for d in done:
            si, kind, fi, out = tickets[d["ticket"]]
            s = sensors[si]
            if d["status"] != 0:  # refused or failed: reported under "failed"
                continue
            checked += 1
            if kind == 0:
                want = digests.get(f"{si}_{fi}")
                got = out[:d["out_len"]].cpu().numpy().tobytes()
                mism += want is None or (len(got), hashlib.sha256(got).hexdigest()) != (want["bytes"], want["sha256"])
            else:
                if (si, fi) not in exp_cache:
                    exp_cache[(si, fi)] = expect(s.frames[fi], s.D)
                mism += not np.array_equal(out[:d["out_len"]].cpu().numpy(), exp_cache[(si, fi)])
        rep["checked"] = checked
        rep["mismatches"] = int(mism)
    server.close()
    return rep

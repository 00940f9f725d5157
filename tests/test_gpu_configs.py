"""Byte-for-byte parity of every frame of every workload at full size, in the
form each workload is run in: the GPU's streams against sha256 digests of the
CPU oracle's streams (tests/golden/make_digests.py calls only the oracle and
the seeded input generator), and every decode against the sorted unique input.

* 16-beam (12 levels, C = 16) and 64-beam (14 levels, C = 32) frames through
  the per-frame calls;
* the 32 uneven frames of the batching workload (16/32/64 beams, 14 levels,
  C = 32) through one batched encode and one batched decode;
* the 8 frames of the 128-beam workload (18 levels, 1 mm, C = 64) as one batch;
* one frame of each of the 24 sensors of the serving fleet (14-18 levels,
  C = 32 / 64) submitted together to the continuous-batching server, encode
  and decode jobs mixed in flight.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
STREAMS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json"))).get("streams", {})


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_25260_amd import lpcc
    lpcc.lib()
    return lpcc


def _sha(b):
    return hashlib.sha256(b).hexdigest()


def _sorted_unique(xyz, D):
    u = np.unique(xyz, axis=0)
    return u[np.argsort(O.morton(u, D))]


def _need(group, n):
    got = STREAMS.get(group, {})
    if len(got) < n:
        pytest.skip(f"digests of {group} not generated ({len(got)} of {n})")
    return got


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_plain_frames_match_oracle(L, name):
    cfg = synth.CONFIGS[name]
    want = _need(name, len(cfg.seeds))
    m = L.Model(synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), 0)
    ctx = L.Context(0)
    for seed in cfg.seeds:
        print(name, seed, flush=True)
        xyz = synth.make_scan(cfg.scan, seed)
        bs = L.encode_frame(ctx, m, torch.from_numpy(xyz).cuda(), 8)
        assert (len(bs), _sha(bs)) == (want[str(seed)]["bytes"], want[str(seed)]["sha256"]), seed
        assert np.array_equal(L.decode_frame(ctx, m, bs), _sorted_unique(xyz, cfg.scan.D)), seed


def _batch_round_trip(L, m, frames, D, want_keys, want):
    ctx = L.Context(0)
    dev = [torch.from_numpy(f).cuda() for f in frames]
    outs = [torch.zeros(len(f) * 8 + 65536, dtype=torch.uint8, device="cuda") for f in frames]
    lens, st = L.encode_batch(ctx, m, dev, 8, outs=outs)
    assert st == [0] * len(frames)
    streams = [bytes(o[:n].cpu().numpy()) for o, n in zip(outs, lens)]
    for k, b in zip(want_keys, streams):
        assert (len(b), _sha(b)) == (want[k]["bytes"], want[k]["sha256"]), k
    decs = [torch.zeros((len(f), 3), dtype=torch.int32, device="cuda") for f in frames]
    nout, st = L.decode_batch(ctx, m, outs, lengths=lens, outs=decs)
    assert st == [0] * len(frames)
    for f, x, n in zip(frames, decs, nout):
        assert np.array_equal(x[:n].cpu().numpy(), _sorted_unique(f, D))
    return streams


def test_uneven_batch_of_32_matches_oracle(L):
    want = _need("cfg3", 32)
    cfg = synth.CONFIGS["cfg2"]
    m = L.Model(synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), 0)
    seeds = list(range(3001, 3033))
    frames = [synth.make_scan(synth.batch_scan_spec(s), s) for s in seeds]
    print("32-frame uneven batch", sum(len(f) for f in frames), "points", flush=True)
    _batch_round_trip(L, m, frames, cfg.scan.D, [str(s) for s in seeds], want)


def test_128beam_batch_of_8_matches_oracle(L):
    cfg = synth.CONFIGS["cfg4"]
    want = _need("cfg4", len(cfg.seeds))
    m = L.Model(synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), 0)
    frames = [synth.make_scan(cfg.scan, s) for s in cfg.seeds]
    print("8-frame 128-beam batch", sum(len(f) for f in frames), "points", flush=True)
    _batch_round_trip(L, m, frames, cfg.scan.D, [str(s) for s in cfg.seeds], want)


def test_128beam_batch_of_24_matches_oracle(L):
    """The eight 128-beam frames three times over in one batched call (5.7 M
    points): the finest depths' CDF rows then take about 2.9 GB, so the
    device offsets of rows, tables and features go past 2^31 bytes; every
    stream still equals the oracle's digest of its frame."""
    cfg = synth.CONFIGS["cfg4"]
    want = _need("cfg4", len(cfg.seeds))
    m = L.Model(synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), 0)
    frames = [synth.make_scan(cfg.scan, s) for s in cfg.seeds] * 3
    print("24-frame 128-beam batch", sum(len(f) for f in frames), "points", flush=True)
    _batch_round_trip(L, m, frames, cfg.scan.D, [str(s) for s in cfg.seeds] * 3, want)


def test_served_fleet_matches_oracle(L):
    """Every sensor's frame is encoded and its oracle-checked stream decoded
    through the server at once (48 jobs, 8 models, 14-18 levels, C = 32/64)."""
    from paper_2603_25260_amd import serve
    want = _need("fleet", 24)
    keys, sensors = serve.build_fleet(24, 5000, frames_per_sensor=1)
    models = [L.Model(synth.make_weights(1, C, D, nd), 0) for (C, D, nd) in keys]
    srv = L.Server(models, 0, slots=4, max_batch=4)
    jobs = []
    for s in sensors:
        x = torch.from_numpy(s.frames[0]).cuda()
        out = torch.zeros(len(s.frames[0]) * 8 + 65536, dtype=torch.uint8, device="cuda")
        jobs.append((s, 0, srv.submit(0, s.model, x, out, chunk_log2=8), out, x))
    srv.drain()
    done = {d["ticket"]: d for d in srv.poll(1000)}
    streams = {}
    for s, kind, t, out, _ in jobs:
        d = done[t]
        assert d["status"] == 0
        b = bytes(out[:d["out_len"]].cpu().numpy())
        k = f"{s.idx}_0"
        assert (len(b), _sha(b)) == (want[k]["bytes"], want[k]["sha256"]), k
        streams[s.idx] = b
    # decode jobs of the checked streams, all in flight together
    dj = []
    for s in sensors:
        bs = torch.from_numpy(np.frombuffer(streams[s.idx], np.uint8).copy()).cuda()
        out = torch.zeros((len(s.frames[0]), 3), dtype=torch.int32, device="cuda")
        dj.append((s, srv.submit(1, s.model, bs, out, in_len=len(streams[s.idx])), out, bs))
    srv.drain()
    done = {d["ticket"]: d for d in srv.poll(1000)}
    for s, t, out, _ in dj:
        d = done[t]
        assert d["status"] == 0
        assert np.array_equal(out[:d["out_len"]].cpu().numpy(), _sorted_unique(s.frames[0], s.D)), s.idx
    st = srv.stats()
    assert st["bytes_peak"] <= st["bytes_budget"]
    srv.close()

"""Full-size parity on the largest workloads: the GPU's CDF rows of every depth
and its encoded stream equal the CPU oracle's, checked through sha256 digests
that tests/golden/make_digests.py computed with the oracle alone (a
128-beam, 18-level, C = 64 frame takes the oracle minutes).  Also: decode
round trips and batched = per-frame at full size."""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DIGESTS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json")))


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_25260_amd import lpcc
    lpcc.lib()
    return lpcc


def _sorted_unique(xyz, D):
    u = np.unique(xyz, axis=0)
    return u[np.argsort(O.morton(u, D))]


LEVEL_CASES = [(n, int(s)) for n in ("cfg2", "cfg4") for s in sorted(DIGESTS.get(n, {}))]


@pytest.mark.parametrize("name,seed", LEVEL_CASES)
def test_fullsize_levels_and_stream(L, name, seed):
    cfg = synth.CONFIGS[name]
    D = cfg.scan.D
    blob = synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    xyz = synth.make_scan(cfg.scan, seed)
    want = DIGESTS[name][str(seed)]
    dx = torch.from_numpy(xyz).cuda()
    out = torch.zeros((len(xyz), 256), dtype=torch.int32, device="cuda")
    for d in range(D):
        print(name, seed, "depth", d, flush=True)
        n = L.level_probs(ctx, m, dx, d, out=out)
        assert n == want["levels"][str(d)]["rows"]
        got = hashlib.sha256(out[:n].cpu().numpy().astype("<i4").tobytes()).hexdigest()
        assert got == want["levels"][str(d)]["sha256"], f"{name} depth {d}"
    bs = L.encode_frame(ctx, m, dx, 8)
    assert len(bs) == want["stream_c8"]["bytes"]
    assert hashlib.sha256(bs).hexdigest() == want["stream_c8"]["sha256"]
    dec = L.decode_frame(ctx, m, bs)
    assert np.array_equal(dec, _sorted_unique(xyz, D))


def test_fullsize_batch_equals_plain_128beam(L):
    cfg = synth.CONFIGS["cfg4"]
    blob = synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    frames = [torch.from_numpy(synth.make_scan(cfg.scan, s)).cuda() for s in cfg.seeds[1:4]]
    print("128-beam batch of", len(frames), flush=True)
    got, st = L.encode_batch(ctx, m, frames, 8)
    assert st == [0] * len(frames)
    for f, b in zip(frames, got):
        assert b == L.encode_frame(ctx, m, f, 8)
    dec, st = L.decode_batch(ctx, m, got)
    assert st == [0] * len(frames)
    for f, x in zip(frames, dec):
        assert np.array_equal(x, _sorted_unique(f.cpu().numpy(), cfg.scan.D))

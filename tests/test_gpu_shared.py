"""GPU parity of level-aware parameter sharing: a shared weight blob (one
weight tensor per role across depths, per-depth biases and requantisation;
the future work of Sec. S2, last paragraph) through the library's per-frame
and batched calls gives the oracle's CDF rows and streams byte for byte."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


@pytest.mark.parametrize("name,n,zp", [("cfg1", 6000, False), ("cfg2", 12000, False), ("cfg1", 3000, True)])
def test_shared_blob_matches_oracle(L, name, n, zp):
    cfg = synth.CONFIGS[name]
    D = cfg.scan.D
    blob = synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep, shared=True, zero_points=zp)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[1])[:n]
    print(name, n, zp, len(blob), "bytes", flush=True)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    bs = L.encode_frame(ctx, m, torch.from_numpy(xyz).cuda(), 8)
    assert bs == O.encode(blob, xyz, 8)
    assert np.array_equal(L.decode_frame(ctx, m, bs), _sorted_unique(xyz, D))
    for d in (0, D // 2, D - 1):
        assert np.array_equal(L.level_probs(ctx, m, xyz, d), O.level_probs(blob, xyz, d)), d


def test_shared_blob_batch(L):
    cfg = synth.CONFIGS["cfg2"]
    D = cfg.scan.D
    blob = synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep, shared=True)
    frames = [synth.make_scan(cfg.scan, s)[:k] for s, k in zip(cfg.seeds[:3], (9000, 4000, 15000))]
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    dev = [torch.from_numpy(f).cuda() for f in frames]
    outs = [torch.zeros(len(f) * 8 + 65536, dtype=torch.uint8, device="cuda") for f in frames]
    lens, st = L.encode_batch(ctx, m, dev, 8, outs=outs)
    assert st == [0] * 3
    for f, o, n in zip(frames, outs, lens):
        assert bytes(o[:n].cpu().numpy()) == O.encode(blob, f, 8)

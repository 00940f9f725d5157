"""The ablation schedules of Table 4 on the GPU: without cross-scale feature
propagation (blob version 2), with re-densified depths (+GRED) and without
(n_deep = 0, the baseline).  CDF rows and streams equal the oracle's, decode
round trips, batches and base depths included."""
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


def _note(*a):
    print(*a, flush=True)


def sorted_unique(xyz, D):
    u = np.unique(np.asarray(xyz, np.int32).reshape(-1, 3), axis=0)
    return u[np.argsort(O.morton(u, D))]


@pytest.mark.parametrize("C,D,n_deep,n,seed,zp", [(16, 7, 0, 1500, 1, False), (32, 8, 3, 3000, 2, False),
                                                  (64, 7, 2, 1200, 3, False), (32, 8, 3, 2000, 4, True)])
def test_no_propagation_matches_oracle(L, C, D, n_deep, n, seed, zp):
    blob = synth.make_weights(seed, C, D, n_deep, zero_points=zp, xfp=False)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    xyz = synth.random_cloud(n, D, seed)
    _note("C", C, "D", D, "n_deep", n_deep, "zp", zp)
    for d in range(D):
        assert np.array_equal(L.level_probs(ctx, m, xyz, d), O.level_probs(blob, xyz, d)), d
    want = O.encode(blob, xyz, 6)
    got = L.encode_frame(ctx, m, xyz, 6)
    assert got == want
    assert np.array_equal(L.decode_frame(ctx, m, got), sorted_unique(xyz, D))
    ctx.set_base_depth(2)
    got = L.encode_frame(ctx, m, xyz, 6)
    assert got == O.encode(blob, xyz, 6, base=2)
    assert np.array_equal(L.decode_frame(ctx, m, got), sorted_unique(xyz, D))


@pytest.mark.parametrize("nd", [0, 4])
def test_ablation_schedules_64beam_scene(L, nd):
    """Baseline (n_deep = 0) and +GRED (n_deep = 4) on every fifth point of a
    64-beam scene, 14-level octree, C = 32."""
    cfg = synth.CONFIGS["cfg2"]
    blob = synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, nd, xfp=False)
    m = L.Model(blob, 0)
    xyz = np.ascontiguousarray(synth.make_scan(cfg.scan, cfg.seeds[0])[::5])
    _note("cfg2 no-xfp n_deep", nd, len(xyz))
    want = O.encode(blob, xyz, 8)
    ctx = L.Context(0)
    got = L.encode_frame(ctx, m, xyz, 8)
    assert got == want
    assert np.array_equal(L.decode_frame(ctx, m, got), sorted_unique(xyz, cfg.scan.D))


def test_no_propagation_batch(L):
    C, D, n_deep = 16, 9, 3
    blob = synth.make_weights(8, C, D, n_deep, xfp=False)
    m = L.Model(blob, 0)
    frames = [synth.random_cloud(n, D, 500 + n) for n in (1800, 600, 2400)]
    ctx = L.Context(0)
    got, st = L.encode_batch(ctx, m, frames, 7)
    assert st == [0] * 3
    for f, g in zip(frames, got):
        assert g == O.encode(blob, f, 7)
    dec, st = L.decode_batch(ctx, m, got)
    assert st == [0] * 3
    for f, x in zip(frames, dec):
        assert np.array_equal(x, sorted_unique(f, D))

"""Base-geometry coding on the GPU (depths below B coded from the counts of
their own codes, the model from depth B on): streams equal the oracle's byte
for byte for every admissible B, decode round trips from host and device
buffers, batches (one B, and frames of different B in one decode call),
and the error paths."""
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


@pytest.mark.parametrize("C,D,n_deep,n,seed", [(16, 8, 2, 2000, 11), (32, 9, 3, 4000, 12), (64, 7, 2, 1200, 13)])
def test_every_base_matches_oracle(L, C, D, n_deep, n, seed):
    blob = synth.make_weights(seed, C, D, n_deep)
    m = L.Model(blob, 0)
    xyz = synth.random_cloud(n, D, seed)
    want_xyz = sorted_unique(xyz, D)
    k0 = D - n_deep - 1
    for B in range(1, k0 + 1):
        ctx = L.Context(0)
        ctx.set_base_depth(B)
        _note("C", C, "D", D, "B", B)
        want = O.encode(blob, xyz, 6, base=B)
        got = L.encode_frame(ctx, m, xyz, 6)
        assert got == want, B
        assert np.array_equal(L.decode_frame(ctx, m, got), want_xyz), B


def test_64beam_scene_base5_device_buffers(L):
    cfg = synth.CONFIGS["cfg2"]
    blob = synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    m = L.Model(blob, 0)
    xyz = np.ascontiguousarray(synth.make_scan(cfg.scan, cfg.seeds[0])[::5])
    _note("cfg2 B=5", len(xyz))
    want = O.encode(blob, xyz, 8, base=5)
    ctx = L.Context(0)
    ctx.set_base_depth(5)
    dx = torch.from_numpy(xyz).cuda()
    out = torch.zeros(len(want) + 100, dtype=torch.uint8, device="cuda")
    n = L.encode_frame(ctx, m, dx, 8, out=out)
    assert n == len(want) and out[:n].cpu().numpy().tobytes() == want
    dec = torch.zeros((len(xyz), 3), dtype=torch.int32, device="cuda")
    k = L.decode_frame(L.Context(0), m, out, length=n, out=dec)  # B comes from the stream
    assert np.array_equal(dec[:k].cpu().numpy(), sorted_unique(xyz, cfg.scan.D))
    # the model from depth 0 is what level_probs reports, whatever the base
    assert np.array_equal(L.level_probs(ctx, m, dx, 6), O.level_probs(blob, xyz, 6))


def test_batches_with_base(L):
    C, D, n_deep = 16, 9, 3
    blob = synth.make_weights(21, C, D, n_deep)
    m = L.Model(blob, 0)
    frames = [synth.random_cloud(n, D, 300 + n) for n in (1500, 700, 2600, 40)]
    ctx = L.Context(0)
    ctx.set_base_depth(3)
    _note("batch B=3")
    got, st = L.encode_batch(ctx, m, frames, 7)
    assert st == [0] * 4
    for f, g in zip(frames, got):
        assert g == O.encode(blob, f, 7, base=3)
    dec, st = L.decode_batch(ctx, m, got)
    assert st == [0] * 4
    for f, x in zip(frames, dec):
        assert np.array_equal(x, sorted_unique(f, D))
    # frames of different base depths (and version 1) in one decode call
    mixed = [got[0], O.encode(blob, frames[1], 7), O.encode(blob, frames[2], 7, base=1), got[3]]
    dec, st = L.decode_batch(L.Context(0), m, mixed)
    assert st == [0] * 4
    for f, x in zip(frames, dec):
        assert np.array_equal(x, sorted_unique(f, D))


def test_base_errors(L):
    C, D, n_deep = 16, 7, 2   # k0 = 4
    blob = synth.make_weights(5, C, D, n_deep)
    m = L.Model(blob, 0)
    xyz = synth.random_cloud(500, D, 5)
    ctx = L.Context(0)
    with pytest.raises(Exception):
        ctx.set_base_depth(-1)
    ctx.set_base_depth(5)
    with pytest.raises(L.LpccError):
        L.encode_frame(ctx, m, xyz, 6)
    ctx.set_base_depth(2)
    bs = bytearray(L.encode_frame(ctx, m, xyz, 6))
    bad = bytearray(bs)
    bad[16 + 4 * D] = 5                                      # B above k0
    with pytest.raises(L.LpccError):
        L.decode_frame(ctx, m, bytes(bad))
    bad = bytearray(bs)
    bad[16 + 4 * D + 3] ^= 1                                 # depth 0 count no longer N_0
    with pytest.raises(L.LpccError):
        L.decode_frame(ctx, m, bytes(bad))
    ctx.set_base_depth(0)                                    # back to version 1
    assert L.encode_frame(ctx, m, xyz, 6) == O.encode(blob, xyz, 6)

"""GPU parity: the gfx950 library against the CPU oracle, byte for byte.

Every test calls through the C ABI (liblpcc.so via the thin binding) and
compares with the oracle on the same seeded inputs: CDF rows of every depth,
bitstreams, decoded geometry, cross-decoding in both directions, batched
against per-frame results, device-resident buffers, and edge cases.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_25260_amd import lpcc
    lpcc.lib()
    return lpcc


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


_models = {}


def model(L, seed, C, D, n_deep, zp=False):
    key = (seed, C, D, n_deep, zp)
    if key not in _models:
        blob = synth.make_weights(seed, C, D, n_deep, zero_points=zp)
        _models[key] = (blob, L.Model(blob, 0))
    return _models[key]


def sorted_unique(xyz, D):
    u = np.unique(np.asarray(xyz, np.int32).reshape(-1, 3), axis=0)
    return u[np.argsort(O.morton(u, D))]


SMALL = [  # C, D, n_deep, n, seed, zero points
    (16, 6, 2, 400, 1, False),
    (32, 7, 3, 1500, 2, False),
    (64, 6, 2, 700, 3, False),
    (16, 5, 0, 300, 4, False),
    (16, 5, 4, 300, 5, False),
    (32, 7, 3, 900, 6, True),
    (16, 1, 0, 5, 7, False),
]


@pytest.mark.parametrize("C,D,nd,n,seed,zp", SMALL)
def test_level_probs_small(L, ctx, C, D, nd, n, seed, zp):
    blob, m = model(L, seed, C, D, nd, zp)
    xyz = synth.random_cloud(n, D, seed)
    for d in range(D):
        _note("level_probs", C, D, nd, n, seed, zp, "depth", d)
        want = O.level_probs(blob, xyz, d)
        got = L.level_probs(ctx, m, xyz, d)
        assert got.shape == want.shape
        assert np.array_equal(got, want), f"depth {d}: {np.argwhere(got != want)[:5]}"


@pytest.mark.parametrize("C,D,nd,n,seed,zp", SMALL)
def test_encode_bytes_and_round_trip_small(L, ctx, C, D, nd, n, seed, zp):
    blob, m = model(L, seed, C, D, nd, zp)
    xyz = synth.random_cloud(n, D, seed)
    for c in (4, 6, 10):
        _note("encode", C, D, nd, n, seed, zp, "c", c)
        want = O.encode(blob, xyz, c)
        got = L.encode_frame(ctx, m, xyz, c)
        assert got == want
        dec = L.decode_frame(ctx, m, got)
        assert np.array_equal(dec, sorted_unique(xyz, D))


def test_long_chunks_decode_from_lds(L, ctx):
    """Chunks of 2^12 and 2^14 nodes: payloads beyond the register window are
    read from LDS by the decoder."""
    blob, m = model(L, 8, 32, 10, 3)
    xyz = synth.random_cloud(15000, 10, 8)
    for c in (12, 14):
        _note("long chunks", c)
        want = O.encode(blob, xyz, c)
        got = L.encode_frame(ctx, m, xyz, c)
        assert got == want
        assert np.array_equal(L.decode_frame(ctx, m, got), sorted_unique(xyz, D=10))


def test_config1_all_depths_and_stream(L, ctx):
    cfg = synth.CONFIGS["cfg1"]
    blob, m = model(L, cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[0])
    for d in range(cfg.scan.D):
        _note("cfg1 level_probs depth", d)
        assert np.array_equal(L.level_probs(ctx, m, xyz, d), O.level_probs(blob, xyz, d)), d
    for c in (6, 10):
        want = O.encode(blob, xyz, c)
        got = L.encode_frame(ctx, m, xyz, c)
        assert got == want
        # cross-platform decoding in both directions
        assert np.array_equal(O.decode(blob, got), sorted_unique(xyz, cfg.scan.D))
        assert np.array_equal(L.decode_frame(ctx, m, want), sorted_unique(xyz, cfg.scan.D))


def test_config2_full_frame_bytes(L, ctx):
    cfg = synth.CONFIGS["cfg2"]
    blob, m = model(L, cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[0])
    _note("cfg2 encode", len(xyz))
    got = L.encode_frame(ctx, m, xyz, 10)
    want = O.encode(blob, xyz, 10)
    assert got == want
    dec = L.decode_frame(ctx, m, got)
    assert np.array_equal(dec, sorted_unique(xyz, cfg.scan.D))


@pytest.mark.parametrize("nd", [3, 5])
def test_threshold_variants_64beam_scene(L, ctx, nd):
    """The re-densification threshold of the paper's ablation (t = L - 3 and
    L - 5 beside the default L - 4) on a 64-beam scene, 14-level octree,
    C = 32: every fifth point of the first frame, bytes equal the oracle's."""
    cfg = synth.CONFIGS["cfg2"]
    blob, m = model(L, cfg.weight_seed, cfg.C, cfg.scan.D, nd)
    xyz = np.ascontiguousarray(synth.make_scan(cfg.scan, cfg.seeds[0])[::5])
    _note(f"cfg2 n_deep={nd}", len(xyz))
    want = O.encode(blob, xyz, 8)
    got = L.encode_frame(ctx, m, xyz, 8)
    assert got == want
    assert np.array_equal(L.decode_frame(ctx, m, got), sorted_unique(xyz, cfg.scan.D))


def test_device_resident_buffers(L, ctx):
    cfg = synth.CONFIGS["cfg1"]
    blob, m = model(L, cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[1])
    want = O.encode(blob, xyz, 8)
    dx = torch.from_numpy(xyz).cuda()
    out = torch.full((len(want) + 100,), 0x5A, dtype=torch.uint8, device="cuda")
    n = L.encode_frame(ctx, m, dx, 8, out=out)
    assert n == len(want)
    assert out[:n].cpu().numpy().tobytes() == want
    assert bool((out[n:] == 0x5A).all())  # nothing written past the stream
    dec = torch.zeros((len(xyz), 3), dtype=torch.int32, device="cuda")
    k = L.decode_frame(ctx, m, out, length=n, out=dec)
    assert np.array_equal(dec[:k].cpu().numpy(), sorted_unique(xyz, cfg.scan.D))
    cdf = torch.zeros((20000, 256), dtype=torch.int32, device="cuda")
    nn = L.level_probs(ctx, m, dx, 9, out=cdf)
    assert np.array_equal(cdf[:nn].cpu().numpy(), O.level_probs(blob, xyz, 9))


def test_device_output_capacity(L, ctx):
    """A device output shorter than the stream: LPCC_E_CAPACITY, and no byte
    at or past the given capacity is written; an exact one holds the stream."""
    cfg = synth.CONFIGS["cfg1"]
    blob, m = model(L, cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[2])
    want = O.encode(blob, xyz, 8)
    dx = torch.from_numpy(xyz).cuda()
    for cap in (len(want) - 1, len(want) // 2, 20):
        big = torch.full((len(want) + 64,), 0xC3, dtype=torch.uint8, device="cuda")
        with pytest.raises(L.LpccError) as e:
            L.encode_frame(ctx, m, dx, 8, out=big[:cap])
        assert e.value.code == L.E_CAPACITY
        assert bool((big[cap:] == 0xC3).all()), cap
    exact = torch.zeros(len(want), dtype=torch.uint8, device="cuda")
    assert L.encode_frame(ctx, m, dx, 8, out=exact) == len(want)
    assert exact.cpu().numpy().tobytes() == want


def test_batch_device_outputs(L, ctx):
    """Several frames into device outputs in one call (payloads placed on the
    device): every stream equals the oracle's, including empty frames."""
    D, C, nd = 9, 32, 3
    blob, m = model(L, 11, C, D, nd)
    frames = [synth.random_cloud(n, D, 300 + i) for i, n in enumerate([700, 0, 5, 2500, 64])]
    want = [O.encode(blob, x, 7) for x in frames]
    outs = [torch.full((len(w) + 32,), 0x77, dtype=torch.uint8, device="cuda") for w in want]
    got, st = L.encode_batch(ctx, m, [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in frames], 7,
                             outs=outs)
    assert st == [0] * len(frames)
    for f, w in enumerate(want):
        assert got[f] == len(w), f
        assert outs[f][:len(w)].cpu().numpy().tobytes() == w, f
        assert bool((outs[f][len(w):] == 0x77).all()), f


def test_batch_device_outputs_one_too_small(L, ctx):
    """One frame's device output is too short: that frame reports
    LPCC_E_CAPACITY with its required size and nothing at or past its
    capacity is written; the other frames' streams are complete."""
    D, C, nd = 9, 32, 3
    blob, m = model(L, 11, C, D, nd)
    frames = [synth.random_cloud(n, D, 400 + i) for i, n in enumerate([900, 300, 1500])]
    want = [O.encode(blob, x, 7) for x in frames]
    caps = [len(want[0]) + 8, len(want[1]) // 2, len(want[2])]
    bigs = [torch.full((c + 64,), 0x3C, dtype=torch.uint8, device="cuda") for c in caps]
    outs = [b[:c] for b, c in zip(bigs, caps)]
    got, st = L.encode_batch(ctx, m, [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in frames], 7,
                             outs=outs)
    assert st == [0, L.E_CAPACITY, 0]
    assert got[1] == len(want[1])  # the required size
    for f in (0, 2):
        assert got[f] == len(want[f])
        assert bigs[f][:len(want[f])].cpu().numpy().tobytes() == want[f], f
    for f in range(3):
        assert bool((bigs[f][caps[f]:] == 0x3C).all()), f


def test_batch_equals_per_frame(L, ctx):
    D, C, nd = 9, 32, 3
    blob, m = model(L, 11, C, D, nd)
    frames = [synth.random_cloud(n, D, 100 + i) for i, n in enumerate([500, 0, 1, 2000, 37, 900])]
    got, st = L.encode_batch(ctx, m, frames, 7)
    assert st == [0] * len(frames)
    for f, x in enumerate(frames):
        assert got[f] == O.encode(blob, x, 7), f
    dec, st = L.decode_batch(ctx, m, got)
    assert st == [0] * len(frames)
    for f, x in enumerate(frames):
        assert np.array_equal(dec[f], sorted_unique(x, D)), f


def test_edge_cases(L, ctx):
    D = 8
    blob, m = model(L, 21, 16, D, 3)
    # empty, single point, duplicates, cube corners
    for xyz in [np.zeros((0, 3), np.int32), np.array([[255, 0, 7]], np.int32),
                np.array([[1, 2, 3]] * 9 + [[0, 0, 0], [255, 255, 255]], np.int32),
                np.array([[0, 0, 0], [255, 255, 255], [0, 255, 0], [255, 0, 255]], np.int32)]:
        want = O.encode(blob, xyz, 6)
        got = L.encode_frame(ctx, m, xyz, 6)
        assert got == want
        assert np.array_equal(L.decode_frame(ctx, m, got), sorted_unique(xyz, D))
    with pytest.raises(L.LpccError) as e:
        L.encode_frame(ctx, m, np.array([[256, 0, 0]], np.int32), 6)
    assert e.value.code == L.E_INVAL
    with pytest.raises(L.LpccError) as e:
        L.encode_frame(ctx, m, np.array([[-1, 0, 0]], np.int32), 6)
    assert e.value.code == L.E_INVAL


def test_corrupt_and_wrong_model(L, ctx):
    D = 7
    blob, m = model(L, 31, 16, D, 2)
    _, m2 = model(L, 32, 16, D, 2)
    xyz = synth.random_cloud(600, D, 31)
    bs = L.encode_frame(ctx, m, xyz, 6)
    with pytest.raises(L.LpccError) as e:
        L.decode_frame(ctx, m2, bs)
    assert e.value.code == L.E_MODEL
    with pytest.raises(L.LpccError) as e:
        L.decode_frame(ctx, m, bs[:-3])
    assert e.value.code == L.E_CORRUPT
    rng = np.random.default_rng(0)
    for k in range(10):
        b2 = bytearray(bs)
        i = int(rng.integers(16 + 4 * D, len(b2)))
        b2[i] ^= 0xA5
        _note("flipped byte", i)
        try:
            out = L.decode_frame(ctx, m, bytes(b2))
            ref = O.decode(blob, bytes(b2))
            assert np.array_equal(out, ref)
        except L.LpccError as err:
            assert err.code == L.E_CORRUPT
            with pytest.raises(O.OracleError):
                O.decode(blob, bytes(b2))


def test_softmax_table_matches_oracle(L):
    assert np.array_equal(L.softmax_table(), O.lut())


def test_repeatable(L, ctx):
    cfg = synth.CONFIGS["cfg1"]
    blob, m = model(L, cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[2])
    first = L.encode_frame(ctx, m, xyz, 10)
    for _ in range(20):
        assert L.encode_frame(ctx, m, xyz, 10) == first

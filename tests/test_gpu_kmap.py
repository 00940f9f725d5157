"""GPU parity of the two ways the library builds the 3x3x3 neighbour tables
of the sparse convolutions (Sec. 3.3): a coordinate hash at every convolved
depth (mode 1), or a hash at the first convolved depth only and every later
table derived from the parent depth's table, occupancy codes and first-child
rows (mode 0, the default).  Both give the oracle's streams, decodes and CDF
rows byte for byte: per-frame and batched calls, base geometry (the chain of
tables then starts at the base depth), the schedule without cross-scale
propagation, and the deep fusion depth."""
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


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name,n", [("cfg1", 7000), ("cfg2", 20000)])
def test_kmap_modes_match_oracle(L, mode, name, n):
    cfg = synth.CONFIGS[name]
    D = cfg.scan.D
    blob = synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[2])[:n]
    print(name, n, "mode", mode, flush=True)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    ctx.set_kmap_mode(mode)
    bs = L.encode_frame(ctx, m, torch.from_numpy(xyz).cuda(), 8)
    assert bs == O.encode(blob, xyz, 8)
    assert np.array_equal(L.decode_frame(ctx, m, bs), _sorted_unique(xyz, D))
    k0 = D - cfg.n_deep - 1
    for d in (1, k0, k0 + 1, D - 1):
        assert np.array_equal(L.level_probs(ctx, m, xyz, d), O.level_probs(blob, xyz, d)), d


@pytest.mark.parametrize("mode", [0, 1])
def test_kmap_modes_with_base_depth(L, mode):
    cfg = synth.CONFIGS["cfg2"]
    D = cfg.scan.D
    blob = synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[3])[:15000]
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    ctx.set_kmap_mode(mode)
    for base in (3, 6):
        print("base", base, "mode", mode, flush=True)
        ctx.set_base_depth(base)
        bs = L.encode_frame(ctx, m, torch.from_numpy(xyz).cuda(), 8)
        assert bs == O.encode(blob, xyz, 8, base=base)
        assert np.array_equal(L.decode_frame(ctx, m, bs), _sorted_unique(xyz, D))


def test_kmap_modes_batched_and_noxfp(L):
    """Uneven batch through both modes: identical streams, equal to the
    oracle's; the same for the schedule without cross-scale propagation."""
    cfg = synth.CONFIGS["cfg2"]
    D = cfg.scan.D
    frames = [synth.make_scan(cfg.scan, s)[:k] for s, k in zip(cfg.seeds[:4], (9000, 300, 15000, 1))]
    dev = [torch.from_numpy(f).cuda() for f in frames]
    for xfp in (True, False):
        blob = synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep, xfp=xfp)
        m = L.Model(blob, 0)
        want = [O.encode(blob, f, 8) for f in frames]
        for mode in (0, 1):
            print("xfp", xfp, "mode", mode, flush=True)
            ctx = L.Context(0)
            ctx.set_kmap_mode(mode)
            outs = [torch.zeros(len(f) * 8 + 65536, dtype=torch.uint8, device="cuda") for f in frames]
            lens, st = L.encode_batch(ctx, m, dev, 8, outs=outs)
            assert st == [0] * len(frames)
            got = [bytes(o[:n].cpu().numpy()) for o, n in zip(outs, lens)]
            assert got == want
            decs, st2 = L.decode_batch(ctx, m, got)
            assert st2 == [0] * len(frames)
            for f, x in zip(frames, decs):
                assert np.array_equal(np.asarray(x), _sorted_unique(f, D))


def test_kmap_mode_errors(L):
    ctx = L.Context(0)
    for bad in (-1, 2, 7):
        with pytest.raises(Exception):
            ctx.set_kmap_mode(bad)
    ctx.set_kmap_mode(1)
    ctx.set_kmap_mode(0)


def test_kmap_modes_on_corrupt_streams(L):
    """Streams whose decoded codes claim more children than their header
    (flipped payload bytes, the wrong model): the tables derived from the
    parent depth hold only rows below the depth's node count, and both modes
    end as the oracle does (the same points, or a corrupt-stream error)."""
    cfg = synth.CONFIGS["cfg2"]
    D = cfg.scan.D
    blob = synth.make_weights(cfg.weight_seed, cfg.C, D, cfg.n_deep)
    m = L.Model(blob, 0)
    m2 = L.Model(synth.make_weights(cfg.weight_seed + 1, cfg.C, D, cfg.n_deep), 0)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[4])[:20000]
    bs = O.encode(blob, xyz, 8)
    rng = np.random.default_rng(5)
    flips = [int(rng.integers(16 + 4 * D, len(bs))) for _ in range(4)]
    for mode in (0, 1):
        ctx = L.Context(0)
        ctx.set_kmap_mode(mode)
        print("wrong model, mode", mode, flush=True)
        with pytest.raises(L.LpccError) as e:
            L.decode_frame(ctx, m2, bs)
        assert e.value.code == L.E_MODEL
        for i in flips:
            print("flipped byte", i, "mode", mode, flush=True)
            b2 = bytearray(bs)
            b2[i] ^= 0x5A
            try:
                out = L.decode_frame(ctx, m, bytes(b2))
            except L.LpccError as err:
                assert err.code == L.E_CORRUPT
                with pytest.raises(O.OracleError):
                    O.decode(blob, bytes(b2))
            else:
                assert np.array_equal(out, O.decode(blob, bytes(b2)))

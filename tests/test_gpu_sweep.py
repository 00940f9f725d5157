"""Seeded sweep of small random cases through the GPU path against the
oracle: channel width, depth, number of re-densified depths, schedule (with
or without cross-scale propagation), shared weights, zero points, layer
gains, requantisation shifts, a confident predictor head, chunk size, base
depth and neighbour-table mode drawn per case, on random clouds and scan
fragments.  Each case compares one depth's CDF rows, the stream and the
decode.  The draws are fixed (seed 2026), so a failure names its case."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth
from tests.blobs import with_fc2_bias

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_CASES = 100


def _cases():
    rng = np.random.default_rng(2026)
    out = []
    for k in range(N_CASES):
        C = int(rng.choice([16, 32, 64]))
        D = int(rng.integers(5, 13))
        nd = int(rng.integers(0, min(5, D - 1) + 1))
        xfp = bool(rng.random() < 0.8)
        shared = bool(rng.random() < 0.25)
        zp = bool(rng.random() < 0.4)
        gain = float(rng.choice([0.5, 1.0, 1.0, 2.0, 6.0]))
        shift = int(rng.choice([16, 24, 24, 30]))
        confident = bool(rng.random() < 0.2) and not shared
        cl = int(rng.integers(4, 15))
        base = int(rng.integers(0, D - nd)) if rng.random() < 0.3 else 0
        mode = int(rng.integers(0, 2))
        npts = int(rng.integers(1, 6000))
        out.append(dict(k=k, C=C, D=D, nd=nd, xfp=xfp, shared=shared, zp=zp, gain=gain, shift=shift,
                        confident=confident, cl=cl, base=base, mode=mode, npts=npts,
                        seed=int(rng.integers(1 << 30)), level=int(rng.integers(1, D))))
    return out


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_25260_amd import lpcc
    lpcc.lib()
    return lpcc


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"case{c['k']}")
def test_sweep_case(L, case):
    c = case
    print(c, flush=True)
    blob = synth.make_weights(c["seed"] % 1000, c["C"], c["D"], c["nd"], zero_points=c["zp"], gain=c["gain"],
                              shift=c["shift"], xfp=c["xfp"], shared=c["shared"])
    if c["confident"]:
        blob = with_fc2_bias(blob, c["seed"] % 255, 200000)
    xyz = synth.random_cloud(c["npts"], c["D"], c["seed"])
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    ctx.set_kmap_mode(c["mode"])
    ctx.set_base_depth(c["base"])
    dx = torch.from_numpy(xyz).cuda()
    if c["level"] >= c["base"]:
        assert np.array_equal(L.level_probs(ctx, m, dx, c["level"]), O.level_probs(blob, xyz, c["level"]))
    want = O.encode(blob, xyz, c["cl"], base=c["base"])
    assert L.encode_frame(ctx, m, dx, c["cl"]) == want
    u = np.unique(xyz, axis=0)
    assert np.array_equal(L.decode_frame(ctx, m, want), u[np.argsort(O.morton(u, c["D"]))])


def _batch_cases():
    rng = np.random.default_rng(2027)
    out = []
    for k in range(20):
        C = int(rng.choice([16, 32, 64]))
        D = int(rng.integers(5, 13))
        nd = int(rng.integers(0, min(5, D - 1) + 1))
        sizes = [int(rng.choice([0, 1, int(rng.integers(2, 5000))], p=[0.1, 0.1, 0.8]))
                 for _ in range(int(rng.integers(1, 7)))]
        out.append(dict(k=k, C=C, D=D, nd=nd, sizes=sizes, zp=bool(rng.random() < 0.4),
                        cl=int(rng.integers(4, 15)), mode=int(rng.integers(0, 2)), seed=int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("case", _batch_cases(), ids=lambda c: f"batch{c['k']}")
def test_sweep_batch(L, case):
    """Batched encode and decode of frames of uneven sizes (empty and
    one-point frames included): every stream is the oracle's per-frame
    stream, every decode the frame's sorted unique points."""
    c = case
    print(c, flush=True)
    blob = synth.make_weights(c["seed"] % 1000, c["C"], c["D"], c["nd"], zero_points=c["zp"])
    frames = [synth.random_cloud(n, c["D"], c["seed"] + i) if n else np.zeros((0, 3), np.int32)
              for i, n in enumerate(c["sizes"])]
    want = [O.encode(blob, f, c["cl"]) for f in frames]
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    ctx.set_kmap_mode(c["mode"])
    got, st = L.encode_batch(ctx, m, frames, c["cl"])
    assert st == [0] * len(frames)
    assert got == want
    decs, st2 = L.decode_batch(ctx, m, got)
    assert st2 == [0] * len(frames)
    for f, x in zip(frames, decs):
        u = np.unique(f, axis=0)
        assert np.array_equal(np.asarray(x).reshape(-1, 3), u[np.argsort(O.morton(u, c["D"]))])

"""GPU parity for confident predictor heads: one logit of every head far
above the others, so most nodes' exponent sums are at most 65281 and the
dominant entry's product E K reaches 2^31 in the frequency formula (Eq. 15).
CDF rows, streams and decodes equal the oracle's, per frame and batched.
Also saturated layers (raised multipliers: clamped activations, maximum
logits tied many times over)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth
from tests.blobs import with_fc2_bias

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


@pytest.mark.parametrize("C,D,nd,npts,sym", [(32, 10, 4, 4000, 254), (64, 12, 5, 9000, 17), (16, 9, 3, 3000, 0)])
def test_confident_head_matches_oracle(L, C, D, nd, npts, sym):
    blob = with_fc2_bias(synth.make_weights(7 + C, C, D, nd), sym, 200000)
    xyz = synth.random_cloud(npts, D, 9 + C)
    print("C", C, "D", D, "sym", sym, flush=True)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    dx = torch.from_numpy(xyz).cuda()
    k0 = D - nd - 1
    for d in (1, k0, k0 + 1, D - 1):
        assert np.array_equal(L.level_probs(ctx, m, dx, d), O.level_probs(blob, xyz, d)), d
    want = O.encode(blob, xyz, 8)
    assert L.encode_frame(ctx, m, dx, 8) == want
    assert np.array_equal(L.decode_frame(ctx, m, want), _sorted_unique(xyz, D))


def test_confident_head_batched(L):
    C, D, nd = 32, 11, 4
    blob = with_fc2_bias(synth.make_weights(3, C, D, nd), 254, 200000)
    frames = [synth.random_cloud(n, D, 40 + n) for n in (6000, 500, 12000)]
    want = [O.encode(blob, f, 8) for f in frames]
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    print("batched confident head", flush=True)
    outs = [torch.zeros(len(f) * 8 + 65536, dtype=torch.uint8, device="cuda") for f in frames]
    lens, st = L.encode_batch(ctx, m, [torch.from_numpy(f).cuda() for f in frames], 8, outs=outs)
    assert st == [0] * len(frames)
    got = [bytes(o[:n].cpu().numpy()) for o, n in zip(outs, lens)]
    assert got == want
    decs, st2 = L.decode_batch(ctx, m, got)
    assert st2 == [0] * len(frames)
    for f, x in zip(frames, decs):
        assert np.array_equal(np.asarray(x), _sorted_unique(f, D))


@pytest.mark.parametrize("gain", [4.0, 16.0])
def test_saturated_layers_match_oracle(L, gain):
    """Every layer's multiplier raised (gain 4 or 16): most activations and
    logits clamp at the int8 limits, and every node's maximum logit is tied
    many times over (the lowest index takes the remainder)."""
    C, D, nd = 32, 10, 4
    blob = synth.make_weights(5, C, D, nd, gain=gain)
    xyz = synth.random_cloud(4000, D, 21)
    print("gain", gain, flush=True)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    dx = torch.from_numpy(xyz).cuda()
    k0 = D - nd - 1
    for d in (1, k0, k0 + 1, D - 1):
        assert np.array_equal(L.level_probs(ctx, m, dx, d), O.level_probs(blob, xyz, d)), d
    want = O.encode(blob, xyz, 8)
    assert L.encode_frame(ctx, m, dx, 8) == want
    assert np.array_equal(L.decode_frame(ctx, m, want), _sorted_unique(xyz, D))

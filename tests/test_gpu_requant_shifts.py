"""GPU parity for other requantisation shifts (Eq. 14): r = 12 and 16 (small
multipliers, the 24-bit multiply-add paths with their own rounding terms)
and r = 30 and 31 (multipliers near 2^20, products beyond 32 bits: the
64-bit path, and no zero-point folding into the rounding term), with and
without zero points.  CDF rows at the shallow, fusion and deep depths,
streams and decodes equal the oracle's."""
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


@pytest.mark.parametrize("zp", [False, True])
@pytest.mark.parametrize("shift", [12, 16, 30, 31])
def test_requant_shift_matches_oracle(L, shift, zp):
    C, D, nd = 32, 10, 4
    blob = synth.make_weights(9, C, D, nd, shift=shift, zero_points=zp)
    xyz = synth.random_cloud(3000, D, 31)
    print("shift", shift, "zero points", zp, flush=True)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    dx = torch.from_numpy(xyz).cuda()
    k0 = D - nd - 1
    for d in (1, k0, k0 + 1, D - 1):
        assert np.array_equal(L.level_probs(ctx, m, dx, d), O.level_probs(blob, xyz, d)), d
    want = O.encode(blob, xyz, 8)
    assert L.encode_frame(ctx, m, dx, 8) == want
    u = np.unique(xyz, axis=0)
    assert np.array_equal(L.decode_frame(ctx, m, want), u[np.argsort(O.morton(u, D))])

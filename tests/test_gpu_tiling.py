"""Kernel variants of the gather-GEMM, child-convolution and upsampling
launches: the compacted variants (present taps / occupied children only)
with every fixed choice of 16-row blocks per wave (1, 2, 4), the dense
variants over every tap and child slot (11, 12, 14), and the autotuned
choice give the oracle's CDF rows and bitstreams byte for byte."""
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


# (C, D, n_deep, points, zero points): every width the kernels are built
# for, several 64 x rb tiles per level and ragged tails; nonzero input zero
# points exercise the per-tap corrections (present neighbours only)
CASES = [(16, 9, 3, 3000, False), (32, 10, 4, 9000, False), (64, 10, 4, 7000, False),
         (32, 9, 3, 5000, True), (64, 9, 3, 4000, True)]


@pytest.mark.parametrize("C,D,n_deep,npts,zp", CASES)
def test_fixed_tilings_match_oracle(L, C, D, n_deep, npts, zp):
    blob = synth.make_weights(11 + C, C, D, n_deep, zero_points=zp)
    xyz = synth.random_cloud(npts, D, 500 + C)
    want = O.encode(blob, xyz, 7)
    d_deep, d_shallow = D - 1, D - n_deep - 2
    p_deep, p_sh = O.level_probs(blob, xyz, d_deep), O.level_probs(blob, xyz, d_shallow)
    m = L.Model(blob, 0)
    dx = torch.from_numpy(xyz).cuda()
    for rb in (1, 2, 4, 11, 12, 14):
        ctx = L.Context(0)
        ctx.set_tiling(rb)
        print("C", C, "zp", zp, "rb", rb, flush=True)
        assert L.encode_frame(ctx, m, dx, 7) == want, f"rb={rb}"
        assert np.array_equal(L.level_probs(ctx, m, dx, d_deep), p_deep), f"rb={rb} deep"
        assert np.array_equal(L.level_probs(ctx, m, dx, d_shallow), p_sh), f"rb={rb} shallow"
        dec = L.decode_frame(ctx, m, want)
        assert len(dec) == len(np.unique(xyz, axis=0))


def test_autotuned_tiling_decides_and_matches(L):
    C, D, n_deep = 32, 11, 4
    blob = synth.make_weights(5, C, D, n_deep)
    xyz = synth.random_cloud(20000, D, 77)
    want = O.encode(blob, xyz, 8)
    m = L.Model(blob, 0)
    ctx = L.Context(0)
    ctx.set_tiling(0)
    dx = torch.from_numpy(xyz).cuda()
    for it in range(3):  # the first call times every candidate, later ones use the choice
        print("autotune call", it, flush=True)
        assert L.encode_frame(ctx, m, dx, 8) == want
        dec = L.decode_frame(ctx, m, want)
        assert len(dec) == len(np.unique(xyz, axis=0))
    table = ctx.tuning()
    assert table, "no tuned classes"
    valid = {1, 2, 4, 11, 12, 14, 101, 102, 111, 112, 114, 201, 202, 211, 212, 214}
    assert all(t["rb"] in valid for t in table), table


def test_imported_tuning_table_is_used(L):
    """A table imported into a fresh context decides its classes without
    timing: the context reports the imported variants (here each class moved
    to another valid variant), and the outputs are still the oracle's."""
    C, D, n_deep = 32, 11, 4
    blob = synth.make_weights(6, C, D, n_deep)
    xyz = synth.random_cloud(20000, D, 78)
    want = O.encode(blob, xyz, 8)
    m = L.Model(blob, 0)
    dx = torch.from_numpy(xyz).cuda()
    ctx = L.Context(0)
    print("tuning source context", flush=True)
    assert L.encode_frame(ctx, m, dx, 8) == want
    L.decode_frame(ctx, m, want)
    table = ctx.tuning()
    assert table and all(t["rb"] for t in table), table

    def other(t):
        if t["kind"] == "up":
            return 201 if t["rb"] != 201 else 202
        if t["rb"] > 100:
            return 101 if t["rb"] != 101 else 102
        return 1 if t["rb"] != 1 else 2

    moved = [dict(t, rb=other(t)) for t in table]
    ctx2 = L.Context(0)
    ctx2.set_tuning(moved)
    print("imported table", flush=True)
    assert L.encode_frame(ctx2, m, dx, 8) == want
    dec = L.decode_frame(ctx2, m, want)
    assert len(dec) == len(np.unique(xyz, axis=0))
    key = lambda t: (t["kind"], t["mode"], t["cin"], t["cout"], t["log2_rows"])
    assert {key(t): t["rb"] for t in ctx2.tuning()} == {key(t): t["rb"] for t in moved}


def test_bad_tuning_rows_rejected(L):
    ctx = L.Context(0)
    good = {"kind": "gemm", "mode": 0, "cin": 32, "cout": 32, "log2_rows": 10, "rb": 2}
    for bad in ({"rb": 3}, {"rb": 201}, {"cin": 0}, {"log2_rows": 63}, {"kind": "up", "rb": 2}):
        with pytest.raises(Exception):
            ctx.set_tuning([good, dict(good, **bad)])
    assert ctx.tuning() == []  # nothing applied by a rejected import
    ctx.set_tuning([good, dict(good, log2_rows=11, rb=0)])
    assert ctx.tuning() == [good]


def test_bad_tiling_rejected(L):
    ctx = L.Context(0)
    with pytest.raises(Exception):
        ctx.set_tiling(3)

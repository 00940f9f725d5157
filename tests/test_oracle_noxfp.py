"""Pins of the oracle's schedule without cross-scale feature propagation
(the ablation of Sec. 4.4, Table 4; blob version 2): planted weights whose
features follow from brute-force counting show that a shallow depth's
features come from the parent codes alone (embedding, ResBlock with identity
skip, upsampling) and that the deep ResBlock reads G alone; round trips for
that schedule with and without re-densified depths (n_deep = 0 is the
ablation's baseline)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth
from tests.blobs import build_blob, zeros

R = 20
UNIT = 1 << R
EMB, DOWN, CONV1, CONV2, SKIP, UP = 1, 2, 3, 4, 5, 6


def test_layer_plans_of_the_two_schedules():
    full = synth.layer_plan(16, 7, 3)
    noxfp = synth.layer_plan(16, 7, 3, xfp=False)
    k0 = 3
    # shallow depths gain an embedding of the parent codes; deep ones lose the skip layer
    assert sum(1 for L in noxfp if L[0] == EMB and L[1] <= k0) == k0
    assert not any(L[0] == SKIP for L in noxfp) and any(L[0] == SKIP for L in full)
    assert all(L[4] == 16 for L in noxfp if L[0] == CONV1)
    assert O.model_info(synth.make_weights(1, 16, 7, 3, xfp=False))[:3] == (16, 7, 3)


def test_planted_shallow_path_from_parent_codes():
    """Shallow depth d = 3 without propagation, planted weights:
    EMB at depth 2 writes popcount(X_2) into channel 0 and the constant 1 into
    channel 1; conv1 sums channel 1 over the 3x3x3 neighbourhood, conv2 passes
    it through at the centre tap, the identity skip adds the embedding; UP
    copies channels 0, 1 to every child with the parent's bits in 2..9.  So
    F_3[child] = (popcount of the parent's code, 1 + #occupied neighbours of
    the parent incl. itself, bits of the parent's code).  Nothing of depths
    0..1 enters: the depth-2 layers of the chain are zero."""
    C, D, n_deep = 12, 6, 2   # k0 = 3

    def fill(kind, depth, j, taps, cin, cout):
        p = zeros(taps, cin, cout, R)
        if depth == 3:
            if kind == EMB:
                p["W"][0, :, 0] = 1
                p["bias"][1] = 128
                p["m_pos"], p["m_neg"], p["r"] = 1, 0, 7   # (127 k + 64) >> 7 = k for k <= 8
            if kind == CONV1:
                p["W"][:, 1, 1] = 1
                p["m_neg"] = 0
            if kind == CONV2:
                p["W"][13, 1, 1] = 1
            if kind == UP:
                for o in range(8):
                    p["W"][0, 0, o * C + 0] = 1
                    p["W"][0, 1, o * C + 1] = 1
                    for b in range(8):
                        p["W"][0, C + b, o * C + 2 + b] = 1
                p["m_pos"] = UNIT
                p["m_neg"] = UNIT
        return p

    blob = build_blob(C, D, n_deep, fill, xfp=False)
    xyz = synth.random_cloud(700, D, 41)
    F3 = O.level_features(blob, xyz, 3).astype(np.int64)
    counts, V, X = O.octree(xyz, D)
    cells = np.unique(xyz >> (D - 2), axis=0)
    cells = cells[np.argsort(O.morton(cells, 2))]
    occ = {tuple(c) for c in cells}
    want = []
    for i, c in enumerate(cells):
        n = sum((c[0] + dx, c[1] + dy, c[2] + dz) in occ
                for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))
        code = int(X[2][i])
        bits = [127 if (code >> b) & 1 else 0 for b in range(8)]
        for o in range(8):
            if (code >> o) & 1:
                want.append([bin(code).count("1"), 1 + n] + bits + [0] * (C - 10))
    assert np.array_equal(F3, np.array(want))


def test_planted_deep_resblock_reads_g_alone():
    """Deep depths without propagation: EMB counts set bits at depth d-1,
    DOWN steps sum channel 0 over children; the deep ResBlock's convolutions
    are zero, so its identity skip passes G through; UP steps copy channel 0.
    The shallow UP at k0 writes 5 into F_k0, which must not appear:
    F_d[node] = (#depth-d nodes below its depth-k0 ancestor, 0, ...)."""
    C, D, n_deep = 8, 7, 3
    k0 = D - n_deep - 1

    def fill(kind, depth, j, taps, cin, cout):
        p = zeros(taps, cin, cout, R)
        if kind == UP and depth == k0:
            for o in range(8):
                p["bias"][o * C] = 5
        if depth > k0:
            if kind == EMB:
                p["W"][0, :, 0] = 1
                p["m_pos"], p["m_neg"], p["r"] = 1, 0, 7
            if kind == DOWN:
                p["W"][:, 0, 0] = 1
                p["m_neg"] = 0
            if kind == UP:
                for o in range(8):
                    p["W"][0, 0, o * C] = 1
        return p

    blob = build_blob(C, D, n_deep, fill, xfp=False)
    xyz = synth.random_cloud(400, D, 31, clustered=False)
    counts, V, X = O.octree(xyz, D)
    for d in range(k0 + 1, D):
        Fd = O.level_features(blob, xyz, d).astype(np.int64)
        anc = V[d] >> np.uint64(3 * (d - k0))
        u, cnt = np.unique(anc, return_counts=True)
        per = dict(zip(u.tolist(), cnt.tolist()))
        want0 = np.array([per[a] for a in anc.tolist()])
        assert want0.max() < 128
        assert np.array_equal(Fd[:, 0], want0), d
        assert np.all(Fd[:, 1:] == 0), d


@pytest.mark.parametrize("C,D,n_deep,n,seed", [(8, 6, 2, 300, 1), (16, 7, 0, 800, 2), (8, 8, 3, 1500, 6)])
def test_round_trip_without_propagation(C, D, n_deep, n, seed):
    blob = synth.make_weights(seed, C, D, n_deep, xfp=False)
    xyz = synth.random_cloud(n, D, seed)
    u = np.unique(xyz, axis=0)
    u = u[np.argsort(O.morton(u, D))]
    for B in (0, 1):
        bs = O.encode(blob, xyz, 6, base=B)
        assert np.array_equal(O.decode(blob, bs), u)
    # a stream of one schedule does not decode under the other's weights
    other = synth.make_weights(seed, C, D, n_deep, xfp=True)
    with pytest.raises(O.OracleError) as e:
        O.decode(other, O.encode(blob, xyz, 6))
    assert e.value.code == O.E_MODEL

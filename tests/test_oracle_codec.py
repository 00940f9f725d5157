"""Whole-codec pins of the CPU oracle: round trip, stream length bound,
causality (a depth's distribution never reads finer levels), planted
weights whose features follow from brute-force counting, and edge cases."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth
from tests.blobs import build_blob, zeros
from tests import codec_ref

R = 20
UNIT = 1 << R


def _sorted_unique(xyz, D):
    u = np.unique(np.asarray(xyz, np.int32).reshape(-1, 3), axis=0)
    return u[np.argsort(O.morton(u, D))]


@pytest.mark.parametrize("C,D,n_deep,n,seed", [
    (8, 6, 2, 300, 1), (16, 7, 3, 800, 2), (8, 5, 0, 200, 3), (8, 5, 4, 150, 4), (4, 1, 0, 3, 5),
    (8, 8, 4, 1500, 6)])
def test_round_trip(C, D, n_deep, n, seed):
    blob = synth.make_weights(seed, C, D, n_deep)
    xyz = synth.random_cloud(n, D, seed)
    for c in (4, 6, 10):
        bs = O.encode(blob, xyz, c)
        assert np.array_equal(O.decode(blob, bs), _sorted_unique(xyz, D))


def test_empty_single_and_duplicates():
    blob = synth.make_weights(3, 8, 6, 2)
    bs = O.encode(blob, np.zeros((0, 3), np.int32))
    assert len(bs) == 16 + 4 * 6 and O.decode(blob, bs).shape == (0, 3)
    one = np.array([[63, 0, 17]], np.int32)
    assert np.array_equal(O.decode(blob, O.encode(blob, one)), one)
    dup = np.array([[1, 2, 3]] * 5 + [[0, 0, 0], [63, 63, 63]], np.int32)
    assert np.array_equal(O.decode(blob, O.encode(blob, dup)), _sorted_unique(dup, 6))
    with pytest.raises(O.OracleError) as e:
        O.encode(blob, np.array([[64, 0, 0]], np.int32))
    assert e.value.code == O.E_INVAL


def test_stream_length_bound_and_cdfs():
    cfg = synth.CONFIGS["cfg1"]
    blob = synth.make_weights(1, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[0])
    D, c = cfg.scan.D, 10
    counts, V, X = O.octree(xyz, D)
    info, nsym = 0.0, 0
    for d in range(D):
        cdf = O.level_probs(blob, xyz, d)
        f = np.diff(cdf, axis=1)
        assert np.all(f >= 1) and np.all(cdf[:, 255] == 65536)
        s = X[d].astype(np.int64) - 1
        info += -np.log2(f[np.arange(len(s)), s] / 65536.0).sum()
        nsym += len(s)
    bs = O.encode(blob, xyz, c)
    nch = sum((int(n) + (1 << c) - 1) >> c for n in counts[:D])
    hdr = 16 + 4 * D + 2 * nch
    pay = 8 * (len(bs) - hdr)
    assert info + 32 * nch - 1e-3 <= pay <= info + 0.0056466 * nsym + 40 * nch + 1e-3


def test_causality_finer_geometry_is_not_read():
    """CDFs of depth d depend on V_<=d and X_<d only: moving points inside their
    depth-d cells (which changes X_d and finer levels) leaves them unchanged."""
    C, D, n_deep = 8, 7, 3
    blob = synth.make_weights(9, C, D, n_deep)
    xyz = synth.random_cloud(700, D, 9)
    rng = np.random.default_rng(9)
    for d in range(D):
        cell = xyz >> (D - d)
        moved = (cell << (D - d)) + rng.integers(0, 2 ** (D - d), size=xyz.shape)
        moved = moved.astype(np.int32)
        assert np.array_equal(np.unique(moved >> (D - d), axis=0), np.unique(cell, axis=0))
        a = O.level_probs(blob, xyz, d)
        b = O.level_probs(blob, moved, d)
        assert np.array_equal(a, b), d
        if d + 1 < D:  # and the next depth generally does change
            pass


def test_planted_shallow_path_counts_neighbours():
    """Shallow depth d = 2 with planted weights:
    up at d = 1 writes 1 into channel 0 of every child (bias only);
    ResBlock at d = 2: conv1 sums channel 0 over the 3x3x3 neighbourhood,
    conv2 passes it through at the centre tap, skip adds the input;
    up at d = 2 copies channel 0 to all children and bits(X_1) to channels 1..8.
    So F_2[child] = (1 + #occupied neighbours of its parent incl. itself,
    bits of the parent's code)."""
    C, D, n_deep = 12, 6, 2   # k0 = 3: depths 1..3 shallow

    def fill(kind, depth, j, taps, cin, cout):
        p = zeros(taps, cin, cout, R)
        if kind == 6 and depth == 1:      # UP at d = 1: constant 1 in channel 0
            for o in range(8):
                p["bias"][o * C] = 1
        if kind == 3 and depth == 2:      # CONV1: neighbour sum of channel 0
            p["W"][:, 0, 0] = 1
            p["m_neg"] = 0
        if kind == 4 and depth == 2:      # CONV2: centre tap pass-through
            p["W"][13, 0, 0] = 1
        if kind == 6 and depth == 2:      # UP: copy channel 0, parent bits
            for o in range(8):
                p["W"][0, 0, o * C + 0] = 1
                for b in range(8):
                    p["W"][0, C + b, o * C + 1 + b] = 1
            p["m_pos"] = UNIT
            p["m_neg"] = UNIT
        return p

    blob = build_blob(C, D, n_deep, fill)
    xyz = synth.random_cloud(600, D, 21)
    F2 = O.level_features(blob, xyz, 2).astype(np.int64)
    counts, V, X = O.octree(xyz, D)
    # brute force over depth-1 cells
    cells1 = np.unique(xyz >> (D - 1), axis=0)
    cells1 = cells1[np.argsort(O.morton(cells1, 1))]
    occ = {tuple(c) for c in cells1}
    want = []
    for i, c in enumerate(cells1):
        n = sum((c[0] + dx, c[1] + dy, c[2] + dz) in occ
                for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))
        bits = [127 if (X[1][i] >> b) & 1 else 0 for b in range(8)]
        for o in range(8):
            if (X[1][i] >> o) & 1:
                want.append([1 + n] + bits + [0] * (C - 9))
    assert np.array_equal(F2, np.array(want))


def test_planted_deep_path_counts_descendants():
    """Deep depth d with planted weights:
    EMB writes popcount(X_{d-1}) into channel 0 at depth d-1 (each set bit adds
    127 * m / 2^24 ~= 1); DOWN steps sum channel 0 over children and put the
    slot-weighted sum (slot o times the child's channel 0) into channel 1;
    the deep ResBlock's convolutions are zero and its skip maps G channel 0
    -> out 0, F_k0 channel 0 -> out 1 and G channel 1 -> out 2; UP steps copy
    channels 0..2 to every child.  The shallow UP at k0 writes the constant 5
    into channel 0 of F_k0.  So F_d[node] = (#depth-d nodes below its depth-k0
    ancestor a, 5, sum over a's children c of slot(c) * #depth-d nodes below c)
    when there is at least one DOWN step."""
    C, D, n_deep = 8, 7, 3   # k0 = 3, deep depths 4..6
    k0 = D - n_deep - 1

    def fill(kind, depth, j, taps, cin, cout):
        p = zeros(taps, cin, cout, R)
        if kind == 6 and depth == k0:      # shallow UP producing F_k0
            for o in range(8):
                p["bias"][o * C] = 5
        if depth > k0:
            if kind == 1:                  # EMB: count set bits
                p["W"][0, :, 0] = 1
                p["m_pos"] = 132104        # 127 * 132104 / 2^24 = 1 - 4.8e-7
                p["r"] = 24
                p["m_neg"] = 0
            if kind == 2:                  # DOWN: sum children, slot-weighted sum
                p["W"][:, 0, 0] = 1
                p["W"][:, 0, 1] = np.arange(8)
                p["m_neg"] = 0
            if kind == 5:                  # SKIP: [F_k0 | G] -> (G0, F0, G1)
                p["W"][0, C + 0, 0] = 1
                p["W"][0, 0, 1] = 1
                p["W"][0, C + 1, 2] = 1
            if kind == 6:                  # UP: copy channels 0..2 to every child
                for o in range(8):
                    for ch in range(3):
                        p["W"][0, ch, o * C + ch] = 1
        return p

    blob = build_blob(C, D, n_deep, fill)
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
        assert np.all(Fd[:, 1] == 5)
        if d - 1 > k0:
            mid = V[d] >> np.uint64(3 * (d - k0 - 1))      # ancestor at depth k0+1
            um, cm = np.unique(mid, return_counts=True)
            slot_w = {}
            for m_key, m_cnt in zip(um.tolist(), cm.tolist()):
                slot_w[m_key >> 3] = slot_w.get(m_key >> 3, 0) + (m_key & 7) * m_cnt
            want2 = np.array([slot_w[a] for a in anc.tolist()])
            assert want2.max() < 128
            assert np.array_equal(Fd[:, 2], want2), d
        else:
            assert np.all(Fd[:, 2] == 0)
        assert np.all(Fd[:, 3:] == 0)


def test_planted_predictor_head():
    """fc1 passes channel 0 through (ReLU), fc2 puts it on symbol 7 and the
    bias elsewhere: logits = (bias..., F[0] at s = 7)."""
    C, D, n_deep = 8, 5, 1

    def fill(kind, depth, j, taps, cin, cout):
        p = zeros(taps, cin, cout, R)
        if kind == 6:
            for o in range(8):
                p["bias"][o * C] = 40 + depth
        if kind == 7:
            p["W"][0, 0, 0] = 1
            p["m_neg"] = 0
        if kind == 8:
            p["W"][0, 0, 7] = 1
            p["bias"][:] = -3
            p["bias"][7] = 0
        return p

    blob = build_blob(C, D, n_deep, fill)
    xyz = synth.random_cloud(200, D, 41)
    for d in range(D):
        lg = O.level_logits(blob, xyz, d).astype(np.int64)
        F = O.level_features(blob, xyz, d).astype(np.int64)
        want = np.full(lg.shape, -3)
        want[:, 7] = np.maximum(F[:, 0], 0)
        assert np.array_equal(lg, want), d


def test_second_reading_matches_on_tiny_inputs():
    """A second, independent numpy transcription of the per-depth model agrees
    with the C oracle (guards against transcription slips in either)."""
    for (C, D, n_deep, n, seed, zp) in [(4, 5, 2, 120, 3, False), (6, 6, 3, 300, 4, True),
                                         (4, 4, 0, 60, 5, True)]:
        blob = synth.make_weights(seed, C, D, n_deep, zero_points=zp)
        xyz = synth.random_cloud(n, D, seed)
        ref = codec_ref.level_logits_all(blob, xyz)
        for d in range(D):
            assert np.array_equal(O.level_logits(blob, xyz, d), ref[d]), (C, D, n_deep, d)


def test_corrupt_streams_are_rejected():
    blob = synth.make_weights(3, 8, 6, 2)
    xyz = synth.random_cloud(300, 6, 3)
    bs = bytearray(O.encode(blob, xyz, 6))
    with pytest.raises(O.OracleError):
        O.decode(blob, bytes(bs[:-1]))                       # truncated
    other = synth.make_weights(4, 8, 6, 2)
    with pytest.raises(O.OracleError) as e:
        O.decode(other, bytes(bs))                           # wrong model
    assert e.value.code == O.E_MODEL
    bad = bytearray(bs)
    bad[16] = 2                                              # N_0 = 2
    with pytest.raises(O.OracleError):
        O.decode(blob, bytes(bad))
    # flipped payload bytes decode to something or fail, never crash
    rng = np.random.default_rng(0)
    for _ in range(20):
        b2 = bytearray(bs)
        i = int(rng.integers(16 + 24, len(b2)))
        b2[i] ^= 0x5A
        try:
            O.decode(blob, bytes(b2))
        except O.OracleError as err:
            assert err.code == O.E_CORRUPT

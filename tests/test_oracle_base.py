"""Pins of the oracle's base-geometry coding (the depths below B are coded
from the counts of their own occupancy codes, the model runs from depth B
on): the frequency rule on hand-worked counts and its special cases, B = 0
reproducing the version-1 stream, round trips for every admissible B, the
base depths' payload within range-coder overhead of their ideal length
under the transmitted counts, and malformed base tables rejected."""
import struct

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth


def _sorted_unique(xyz, D):
    u = np.unique(np.asarray(xyz, np.int32).reshape(-1, 3), axis=0)
    return u[np.argsort(O.morton(u, D))]


def test_frequency_rule_hand_example():
    # counts: code 1 three times, code 2 once (N = 4)
    # f_0 = 1 + floor(3 * 65281 / 4) = 48961, f_1 = 1 + floor(65281 / 4) = 16321,
    # 253 absent codes f = 1; total 65535, remainder 1 to the most frequent code
    c = np.zeros(255, np.uint32)
    c[0], c[1] = 3, 1
    f = np.diff(O.counts_to_cdf(c))
    assert f[0] == 48962 and f[1] == 16321 and np.all(f[2:] == 1) and f.sum() == 65536


def test_frequency_rule_special_cases():
    # all codes equally frequent: 1 + floor(65281 / 255) = 257 each, the
    # remainder 1 to the lowest code (the same as an all-equal softmax row)
    f = np.diff(O.counts_to_cdf(np.full(255, 7, np.uint32)))
    assert f[0] == 258 and np.all(f[1:] == 257)
    # a single code: it takes everything the other 254 (f = 1) leave
    c = np.zeros(255, np.uint32)
    c[254] = 9
    f = np.diff(O.counts_to_cdf(c))
    assert f[254] == 65536 - 254 and np.all(f[:254] == 1)
    # ties for the maximum: the remainder goes to the lowest of them
    c = np.zeros(255, np.uint32)
    c[[3, 7]] = 5
    f = np.diff(O.counts_to_cdf(c))
    assert f[3] == f[7] + (65536 - (255 + 2 * (5 * 65281 // 10)))
    rng = np.random.default_rng(1)
    for _ in range(50):
        c = rng.integers(0, 1 << int(rng.integers(1, 20)), 255).astype(np.uint32)
        f = np.diff(O.counts_to_cdf(c))
        assert f.sum() == 65536 and f.min() >= 1
        # floor(c 65281 / N) + 1 except the remainder at the first argmax
        N = int(c.astype(np.int64).sum()) or 1
        base = 1 + (c.astype(np.int64) * 65281) // N
        a = int(np.argmax(c))
        assert np.array_equal(np.delete(f, a), np.delete(base, a))


def test_base_zero_is_the_version_one_stream():
    blob = synth.make_weights(3, 16, 8, 2)
    xyz = synth.random_cloud(1500, 8, 11)
    assert O.encode(blob, xyz, 6, base=0) == O.encode(blob, xyz, 6)


@pytest.mark.parametrize("C,D,n_deep,n,seed", [(8, 8, 2, 1500, 11), (16, 7, 3, 900, 2), (8, 6, 0, 300, 5)])
def test_round_trip_every_base(C, D, n_deep, n, seed):
    blob = synth.make_weights(seed, C, D, n_deep)
    xyz = synth.random_cloud(n, D, seed)
    k0 = D - n_deep - 1
    want = _sorted_unique(xyz, D)
    for B in range(0, k0 + 1):
        for c in (4, 8):
            bs = O.encode(blob, xyz, c, base=B)
            assert bs[4] == (2 if B > 0 else 1) and (B == 0 or bs[16 + 4 * D] == B)
            assert np.array_equal(O.decode(blob, bs), want), (B, c)
    with pytest.raises(O.OracleError) as e:
        O.encode(blob, xyz, 8, base=k0 + 1)
    assert e.value.code == O.E_INVAL


def test_empty_and_single_point_with_base():
    blob = synth.make_weights(3, 8, 6, 2)
    bs = O.encode(blob, np.zeros((0, 3), np.int32), 6, base=2)
    assert O.decode(blob, bs).shape == (0, 3)
    one = np.array([[63, 0, 17]], np.int32)
    assert np.array_equal(O.decode(blob, O.encode(blob, one, 6, base=3)), one)


def _parse_base(bs, D):
    o = 16 + 4 * D
    B = bs[o]
    o += 1
    counts = []
    for d in range(B):
        m = bs[o]
        o += 1
        c = np.zeros(255, np.uint32)
        for _ in range(m):
            code, v = bs[o], struct.unpack_from("<I", bs, o + 1)[0]
            c[code - 1] = v
            o += 5
        counts.append(c)
    return B, counts, o


def test_base_payload_within_coder_overhead():
    """Every chunk of a base depth is within range-coder overhead of the
    ideal length of its codes under the frequencies of the transmitted
    counts, and the counts are those of the octree."""
    cfg = synth.CONFIGS["cfg1"]
    blob = synth.make_weights(1, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[0])
    D, c, Bq = cfg.scan.D, 6, 5
    bs = O.encode(blob, xyz, c, base=Bq)
    N, V, X = O.octree(xyz, D)
    B, counts, pre = _parse_base(bs, D)
    assert B == Bq
    ci = 0
    for d in range(B):
        assert np.array_equal(counts[d], np.bincount(X[d].astype(np.int64) - 1, minlength=255))
        f = np.diff(O.counts_to_cdf(counts[d]))
        s = X[d].astype(np.int64) - 1
        for k in range(0, len(s), 1 << c):
            ideal = -np.log2(f[s[k:k + (1 << c)]] / 65536.0).sum()
            ln = bs[pre + 2 * ci] | (bs[pre + 2 * ci + 1] << 8)
            n_sym = len(s[k:k + (1 << c)])
            assert ideal + 32 - 1e-3 <= 8 * ln <= ideal + 0.0056466 * n_sym + 40 + 1e-3, (d, k)
            ci += 1


def test_malformed_base_tables_rejected():
    blob = synth.make_weights(3, 8, 6, 2)  # k0 = 3
    xyz = synth.random_cloud(300, 6, 3)
    bs = bytearray(O.encode(blob, xyz, 6, base=2))
    D = 6
    o = 16 + 4 * D
    for mutate in ("b0", "bbig", "count", "order", "trunc"):
        b2 = bytearray(bs)
        if mutate == "b0":
            b2[o] = 0
        elif mutate == "bbig":
            b2[o] = 4                       # above k0
        elif mutate == "count":
            b2[o + 3] ^= 1                  # count of depth 0's only code no longer N_0
        elif mutate == "order":             # depth 1: swap two (code, count) pairs
            p = o + 1 + 1 + 5 * b2[o + 1]
            if b2[p] >= 2:
                q = p + 1
                b2[q:q + 5], b2[q + 5:q + 10] = b2[q + 5:q + 10], b2[q:q + 5]
            else:
                b2[p + 1] = 0               # code 0 is not a code
        else:
            b2 = b2[:o + 3]
        with pytest.raises(O.OracleError) as e:
            O.decode(blob, bytes(b2))
        assert e.value.code == O.E_CORRUPT, mutate

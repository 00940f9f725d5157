"""Confident predictor heads (one logit far above the rest), on the CPU.

With a dominant logit the exponent sum S of a node falls to at most 65281,
where the reciprocal K = floor(65281 2^16 / S) is at least 2^16 and the
product E K of the dominant entry (E = 2^15) reaches 2^31: the kernels'
frequency formula (Eq. 15, its division done through the reciprocal K) must
take that product unsigned.  These tests pin (a) that the
formula, with the product unsigned, equals 1 + floor(65281 E / S) over the
whole range of E and S, and that an arithmetic shift would not; and (b) that
the planted-bias blob the GPU test uses does put most nodes in that range,
so the GPU test keeps exercising it."""
import numpy as np

from oracle import oracle as O
from paper_2603_25260_amd import synth
from tests.blobs import with_fc2_bias


def kernel_freq(E, S, arithmetic=False):
    """The GPU's frequency formula on uint32 words (numpy int64 holding them)."""
    K = (65281 << 16) // S
    prod = (E * K) & 0xFFFFFFFF
    if arithmetic:
        q = (((prod ^ 0x80000000) - 0x80000000) >> 16) & 0xFFFFFFFF
    else:
        q = prod >> 16
    up = ((q & 0xFFFFFF) * S + S) & 0xFFFFFFFF
    return (q + 1 + (up <= E * 65281)) & 0xFFFFFFFF


def test_unsigned_frequency_formula_exact_over_range():
    E = np.unique(O.lut().astype(np.int64))[:, None]  # every table value, 0 .. 2^15
    S = np.unique(np.concatenate([np.arange(32768, 70000, 7), [65280, 65281, 65282],
                                  np.geomspace(65282, 255 * 32768, 4000).astype(np.int64)]))[None, :]
    want = 1 + (E * 65281) // S
    assert np.array_equal(kernel_freq(E, S), want)
    # the signed shift goes wrong exactly where E K >= 2^31, which needs S <= 65281
    bad = kernel_freq(E, S, arithmetic=True) != want
    assert bad.any()
    assert not bad[:, S[0] > 65281].any()


def test_confident_blob_reaches_small_sums():
    C, D, nd = 32, 10, 4
    blob = with_fc2_bias(synth.make_weights(7, C, D, nd), 254, 200000)
    xyz = synth.random_cloud(4000, D, 9)
    for d in (2, 5, D - 1):
        f = np.diff(O.level_probs(blob, xyz, d).astype(np.int64), axis=1)
        # f_max >= 2^15 + 256 implies S <= 65281 (the remainder is below 255)
        assert (f.max(1) >= 32768 + 256).mean() > 0.9, d
    bs = O.encode(blob, xyz, 8)
    u = np.unique(xyz, axis=0)
    assert np.array_equal(O.decode(blob, bs), u[np.argsort(O.morton(u, D))])

"""The kernels' form of the requantisation (Eq. 14): the accumulator is
clamped to the layer's [a_lo, a_hi] first and the shifted product is then
taken as a 32-bit value.  For every parameter set a weight blob may hold
(edge multipliers, shifts 0..62, extreme zero points) and for accumulators
across the whole int32 range, that form equals the oracle's requantisation,
and the 32-bit truncation never loses bits.  Host computation only."""
import ctypes
import os

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_25260_amd", "liblpcc.so")
I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblpcc.so is not built (python paper_2603_25260_amd/build.py)")
    L = ctypes.CDLL(LIB)
    L.lpcc_requant_bounds.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    return L


def bounds(lib, m_pos, m_neg, r, z):
    return bounds5(lib, m_pos, m_neg, r, z)[:4]


def bounds5(lib, m_pos, m_neg, r, z):
    out = np.zeros(5, np.int32)
    assert lib.lpcc_requant_bounds(m_pos, m_neg, r, z, out.ctypes.data) == 0
    return [int(v) for v in out]


def s24(v):
    """Low 24 bits of v as a signed value (the operand of a 24-bit multiply)."""
    v &= (1 << 24) - 1
    return v - (1 << 24) if v >= (1 << 23) else v


def wrap32(v):
    v &= (1 << 32) - 1
    return v - (1 << 32) if v >= (1 << 31) else v


def form24(acc, mp, mn, a_lo, a_hi, r, z):
    """The 24-bit form: signed 24-bit multiply-add kept to 32 bits, 32-bit shift."""
    a = min(max(acc, a_lo), a_hi)
    m = mp if a >= 0 else mn
    p = wrap32(s24(a) * s24(m) + ((1 << (r - 1)) if r > 0 else 0)) >> r
    return min(max(p + z, -128), 127)


def kernel_form(acc, mp, mn, a_lo, a_hi, r, z):
    a = min(max(acc, a_lo), a_hi)
    m = mp if a >= 0 else mn
    p = (a * m + ((1 << (r - 1)) if r > 0 else 0)) >> r  # exact (Python integers)
    assert I32_MIN <= p <= I32_MAX, (acc, a, p)
    return min(max(p + z, -128), 127)


def param_sets():
    sets = []
    m24 = int((1 << 24) / (73.6 * np.sqrt(27 * 32)))
    for z in (0, -8, 8, -128, 127):
        sets += [(m24, 0, 24, z), (m24, m24, 24, z), (m24, (m24 * 64) >> 8, 24, z)]
    for r in (0, 1, 2, 15, 31, 32, 33, 47, 61, 62):
        for m in (0, 1, 2, 255, 256, 257, 1 << 20, I32_MAX):
            sets.append((m, m // 3, r, (r * 37) % 256 - 128))
    sets += [(I32_MAX, I32_MAX, 0, 0), (I32_MAX, 0, 0, 127), (0, I32_MAX, 0, -128), (0, 0, 5, 3)]
    return sets


def accumulators(a_lo, a_hi, rng):
    base = [I32_MIN, I32_MIN + 1, -1, 0, 1, I32_MAX - 1, I32_MAX]
    for t in (a_lo, a_hi):
        base += [t + d for d in range(-2, 3)]
    base = [a for a in base if I32_MIN <= a <= I32_MAX]
    rnd = rng.integers(I32_MIN, I32_MAX, 300, dtype=np.int64).tolist()
    small = rng.integers(-5000, 5000, 300, dtype=np.int64).tolist()
    return np.array(sorted(set(base + rnd + small)), np.int64)


@pytest.mark.parametrize("m_pos,m_neg,r,z", param_sets())
def test_clamped_form_equals_oracle(lib, m_pos, m_neg, r, z):
    mp, mn, a_lo, a_hi = bounds(lib, m_pos, m_neg, r, z)
    assert a_lo <= -1 and a_hi >= 0
    rng = np.random.default_rng(m_pos * 7 + m_neg * 3 + r * 11 + z + 1000)
    acc = accumulators(a_lo, a_hi, rng)
    want = O.requant(acc, m_pos, m_neg, r, z)
    got = np.array([kernel_form(int(a), mp, mn, a_lo, a_hi, r, z) for a in acc], np.int8)
    assert np.array_equal(got, want)
    # the bounds are tight: just inside them the output is not yet saturated
    if a_hi > 0 and a_hi < I32_MAX:
        assert O.requant(np.array([a_hi - 1]), m_pos, m_neg, r, z)[0] < 127
    if a_lo < -1 and a_lo > I32_MIN:
        assert O.requant(np.array([a_lo + 1]), m_pos, m_neg, r, z)[0] > -128


def test_rejects_parameters_outside_the_blob_format(lib):
    out = np.zeros(4, np.int32)
    for args in ((-1, 0, 5, 0), (0, -1, 5, 0), (1, 1, 63, 0), (1, 1, -1, 0), (1, 1, 5, 128), (1, 1, 5, -129)):
        assert lib.lpcc_requant_bounds(*args, out.ctypes.data) == -1


@pytest.mark.parametrize("m_pos,m_neg,r,z", param_sets())
def test_24bit_form_when_flagged(lib, m_pos, m_neg, r, z):
    """Where the host flags a layer for the 24-bit multiply-add, that form
    equals the oracle on accumulators across int32, the clamp ends included."""
    mp, mn, a_lo, a_hi, rq24 = bounds5(lib, m_pos, m_neg, r, z)
    if not rq24:
        return
    rng = np.random.default_rng(m_pos * 5 + m_neg + r * 13 + z + 1000)
    acc = accumulators(a_lo, a_hi, rng)
    want = O.requant(acc, m_pos, m_neg, r, z)
    got = np.array([form24(int(a), mp, mn, a_lo, a_hi, r, z) for a in acc], np.int8)
    assert np.array_equal(got, want)


def test_24bit_flag_on_the_synthetic_logit_layers(lib):
    """The seeded logit layers (shift 24, C = 16/32/64) take the 24-bit path;
    a negative output zero point near the int8 edge pushes the product past
    int32 and keeps the 64-bit one."""
    for C in (16, 32, 64):
        m = int(int((1 << 24) / (73.6 * np.sqrt(C))) * 0.75)
        assert bounds5(lib, m, m, 24, 0)[4] == 1, C
    m = int(int((1 << 24) / (73.6 * np.sqrt(32))) * 0.75)
    assert bounds5(lib, m, m, 24, -8)[4] == 0
    assert bounds5(lib, 1 << 23, 1 << 23, 1, 0)[4] == 0

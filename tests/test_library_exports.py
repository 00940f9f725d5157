"""The C-ABI library loads without a GPU and exports every declared symbol;
its host-side exponent table equals the oracle's (no device work)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_25260_amd", "liblpcc.so")


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lpcc_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblpcc.so is not built (python paper_2603_25260_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_host_softmax_table(lib):
    out = np.zeros(256, np.int32)
    assert lib.lpcc_softmax_table(out.ctypes.data_as(ctypes.c_void_p)) == 0
    assert np.array_equal(out, O.lut())


def test_header_peek_without_device(lib):
    hdr = bytearray(16 + 4 * 3)
    hdr[0:4] = b"LPC1"
    hdr[4], hdr[5], hdr[6], hdr[7] = 1, 3, 1, 6
    hdr[12:16] = (5).to_bytes(4, "little")
    hdr[16:20] = (1).to_bytes(4, "little")
    hdr[20:24] = (2).to_bytes(4, "little")
    hdr[24:28] = (4).to_bytes(4, "little")
    hdr += bytes(2 * 3)
    D, n, ws = ctypes.c_int(), ctypes.c_int64(), ctypes.c_size_t()
    buf = (ctypes.c_uint8 * len(hdr)).from_buffer_copy(bytes(hdr))
    assert lib.lpcc_peek_header(buf, ctypes.c_size_t(len(hdr)), ctypes.byref(D), ctypes.byref(n),
                                ctypes.byref(ws)) == 0
    assert (D.value, n.value) == (3, 5)
    assert ws.value > 0  # the depth counts are present
    # 16 bytes: depth and points only, no workspace figure
    assert lib.lpcc_peek_header(buf, ctypes.c_size_t(16), ctypes.byref(D), ctypes.byref(n), ctypes.byref(ws)) == 0
    assert (D.value, n.value, ws.value) == (3, 5, 0)
    bad = (ctypes.c_uint8 * 16)(*b"XPC1" + bytes(12))
    assert lib.lpcc_peek_header(bad, ctypes.c_size_t(16), ctypes.byref(D), ctypes.byref(n), None) == -3


def test_peek_workspace_grows_with_the_frame(lib):
    """The decode workspace bound of a stream grows with its node counts and
    covers at least the node arrays and the CDF rows of its largest depth."""
    def header(D, counts):
        h = bytearray(16 + 4 * D)
        h[0:4] = b"LPC1"
        h[4], h[5], h[6], h[7] = 1, D, 2, 8
        h[12:16] = counts[D].to_bytes(4, "little")
        for d in range(D):
            h[16 + 4 * d:20 + 4 * d] = counts[d].to_bytes(4, "little")
        return bytes(h)
    small = [1, 8, 60, 400, 2000, 6000, 9000]
    big = [1, 8, 64, 500, 4000, 30000, 90000]
    out = []
    for counts in (small, big):
        h = header(6, counts)
        ws = ctypes.c_size_t()
        buf = (ctypes.c_uint8 * len(h)).from_buffer_copy(h)
        assert lib.lpcc_peek_header(buf, ctypes.c_size_t(len(h)), None, None, ctypes.byref(ws)) == 0
        out.append(ws.value)
        assert ws.value >= 512 * max(counts[:6]) + 13 * sum(counts)
    assert out[1] > out[0]


@pytest.mark.parametrize("C,D,nd,flags", [(16, 12, 4, 0), (32, 14, 4, 0), (64, 18, 5, 0), (16, 9, 3, 1),
                                          (32, 10, 4, 2), (16, 7, 0, 3), (64, 6, 5, 0)])
def test_library_weights_equal_generator(lib, C, D, nd, flags):
    """lpcc_make_weights (integer-only, in the library) writes the same bytes
    as the seeded input generator, whose multiplier uses floating point."""
    from paper_2603_25260_amd import synth
    want = synth.make_weights(7, C, D, nd, xfp=not (flags & 1), zero_points=bool(flags & 2))
    n = ctypes.c_size_t()
    assert lib.lpcc_make_weights(ctypes.c_uint64(7), C, D, nd, flags, None, ctypes.c_size_t(0), ctypes.byref(n)) == -2
    assert n.value == len(want)
    buf = (ctypes.c_uint8 * n.value)()
    assert lib.lpcc_make_weights(ctypes.c_uint64(7), C, D, nd, flags, buf, n, ctypes.byref(n)) == 0
    assert bytes(buf) == want


def test_library_weights_reject_bad_arguments(lib):
    n = ctypes.c_size_t()
    for args in ((24, 10, 2, 0), (16, 0, 0, 0), (16, 10, 10, 0), (16, 22, 2, 0), (16, 10, 2, 8)):
        C, D, nd, fl = args
        assert lib.lpcc_make_weights(ctypes.c_uint64(1), C, D, nd, fl, None, ctypes.c_size_t(0),
                                     ctypes.byref(n)) == -1, args

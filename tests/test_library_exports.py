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
        pytest.fail("liblpcc.so is not built (run __graft_entry__.build())")
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
    D, n = ctypes.c_int(), ctypes.c_int64()
    buf = (ctypes.c_uint8 * len(hdr)).from_buffer_copy(bytes(hdr))
    assert lib.lpcc_peek_header(buf, ctypes.c_size_t(len(hdr)), ctypes.byref(D), ctypes.byref(n)) == 0
    assert (D.value, n.value) == (3, 5)
    bad = (ctypes.c_uint8 * 16)(*b"XPC1" + bytes(12))
    assert lib.lpcc_peek_header(bad, ctypes.c_size_t(16), ctypes.byref(D), ctypes.byref(n)) == -3

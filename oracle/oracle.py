"""ctypes wrapper of the CPU oracle (``lpcc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the plain CPU implementation that the GPU library
is checked against.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this module.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lpcc_oracle.c")
LIB = os.path.join(HERE, "liblpcc_oracle.so")

OK, E_INVAL, E_CAPACITY, E_CORRUPT, E_MODEL, E_NOMEM = 0, -1, -2, -3, -4, -6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Wno-unused-parameter",
                               "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def _chk(st):
    if st != OK:
        raise OracleError(st)


def _xyz(xyz):
    return np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))


def lut() -> np.ndarray:
    out = np.zeros(256, np.int32)
    _chk(lib().orc_lut(_p(out)))
    return out


def morton(xyz, bits: int) -> np.ndarray:
    xyz = _xyz(xyz)
    out = np.zeros(len(xyz), np.uint64)
    _chk(lib().orc_morton(_p(xyz), ctypes.c_int64(len(xyz)), ctypes.c_int(bits), _p(out)))
    return out


def octree(xyz, D: int):
    """(counts[D+1], [V_0..V_D] uint64 keys, [X_0..X_{D-1}] uint8 codes)."""
    xyz = _xyz(xyz)
    counts = np.zeros(D + 1, np.int64)
    L = lib()
    _chk(L.orc_octree(_p(xyz), ctypes.c_int64(len(xyz)), ctypes.c_int(D), _p(counts), None, None))
    keys = np.zeros(max(1, int(counts.sum())), np.uint64)
    codes = np.zeros(max(1, int(counts[:D].sum())), np.uint8)
    _chk(L.orc_octree(_p(xyz), ctypes.c_int64(len(xyz)), ctypes.c_int(D), _p(counts), _p(keys), _p(codes)))
    V, X, ko, co = [], [], 0, 0
    for d in range(D + 1):
        V.append(keys[ko:ko + counts[d]].copy())
        ko += counts[d]
        if d < D:
            X.append(codes[co:co + counts[d]].copy())
            co += counts[d]
    return counts, V, X


def kernel_map(keys, j: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    nbr = np.zeros((len(keys), 27), np.int32)
    _chk(lib().orc_kernel_map(_p(keys), ctypes.c_int64(len(keys)), ctypes.c_int(j), _p(nbr)))
    return nbr


def requant(acc, m_pos, m_neg, r, z_out) -> np.ndarray:
    acc = np.ascontiguousarray(acc, dtype=np.int64)
    out = np.zeros(acc.shape, np.int8)
    _chk(lib().orc_requant(_p(acc), ctypes.c_int64(acc.size), ctypes.c_int32(m_pos), ctypes.c_int32(m_neg),
                           ctypes.c_int(r), ctypes.c_int(z_out), _p(out)))
    return out


def conv3(x, nbr, W, bias, m_pos, m_neg, r, z_in=0, z_out=0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.int8)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.int8)
    bias = np.ascontiguousarray(bias, dtype=np.int32)
    rows, cin = x.shape
    cout = W.shape[-1]
    y = np.zeros((rows, cout), np.int8)
    _chk(lib().orc_conv3(_p(x), _p(nbr), ctypes.c_int64(rows), ctypes.c_int(cin), ctypes.c_int(cout), _p(W),
                         _p(bias), ctypes.c_int32(m_pos), ctypes.c_int32(m_neg), ctypes.c_int(r),
                         ctypes.c_int(z_in), ctypes.c_int(z_out), _p(y)))
    return y


def logits_to_cdf(logits) -> np.ndarray:
    lg = np.ascontiguousarray(np.asarray(logits, dtype=np.int8).reshape(-1, 255))
    cdf = np.zeros((len(lg), 256), np.int32)
    _chk(lib().orc_logits_to_cdf(_p(lg), ctypes.c_int64(len(lg)), _p(cdf)))
    return cdf


def rc_encode(sym, cdf) -> bytes:
    sym = np.ascontiguousarray(sym, dtype=np.int32)
    cdf = np.ascontiguousarray(cdf, dtype=np.int32).reshape(-1, 256)
    cap = 2 * len(sym) + 16
    out = np.zeros(cap, np.uint8)
    n = ctypes.c_size_t(0)
    _chk(lib().orc_rc_encode(_p(sym), _p(cdf), ctypes.c_int64(len(sym)), _p(out), ctypes.c_size_t(cap),
                             ctypes.byref(n)))
    return out[:n.value].tobytes()


def rc_decode(data: bytes, cdf) -> np.ndarray:
    cdf = np.ascontiguousarray(cdf, dtype=np.int32).reshape(-1, 256)
    buf = np.frombuffer(data, np.uint8).copy() if len(data) else np.zeros(1, np.uint8)
    sym = np.zeros(len(cdf), np.int32)
    _chk(lib().orc_rc_decode(_p(buf), ctypes.c_size_t(len(data)), _p(cdf), ctypes.c_int64(len(cdf)), _p(sym)))
    return sym


def model_info(blob: bytes):
    C, D, nd, bid = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_uint32()
    b = np.frombuffer(blob, np.uint8)
    _chk(lib().orc_model_info(_p(b), ctypes.c_size_t(len(blob)), ctypes.byref(C), ctypes.byref(D),
                              ctypes.byref(nd), ctypes.byref(bid)))
    return C.value, D.value, nd.value, bid.value


def _level_output(blob: bytes, xyz, level: int, what: int):
    xyz = _xyz(xyz)
    C, D, _, _ = model_info(blob)
    b = np.frombuffer(blob, np.uint8)
    nn = ctypes.c_int64(0)
    L = lib()
    st = L.orc_level_output(_p(b), ctypes.c_size_t(len(blob)), _p(xyz), ctypes.c_int64(len(xyz)),
                            ctypes.c_int(level), ctypes.c_int(what), None, ctypes.c_int64(0), ctypes.byref(nn))
    if st not in (OK, E_CAPACITY):
        raise OracleError(st)
    width = {0: 256, 1: 255, 2: C}[what]
    dtype = {0: np.int32, 1: np.int8, 2: np.int8}[what]
    out = np.zeros((max(1, nn.value), width), dtype)
    _chk(L.orc_level_output(_p(b), ctypes.c_size_t(len(blob)), _p(xyz), ctypes.c_int64(len(xyz)),
                            ctypes.c_int(level), ctypes.c_int(what), _p(out), ctypes.c_int64(nn.value),
                            ctypes.byref(nn)))
    return out[:nn.value]


def level_probs(blob: bytes, xyz, level: int) -> np.ndarray:
    """CDF rows int32 [N_level, 256] of depth ``level``."""
    return _level_output(blob, xyz, level, 0)


def level_logits(blob: bytes, xyz, level: int) -> np.ndarray:
    return _level_output(blob, xyz, level, 1)


def level_features(blob: bytes, xyz, level: int) -> np.ndarray:
    return _level_output(blob, xyz, level, 2)


def encode(blob: bytes, xyz, chunk_log2: int = 10, base: int = 0) -> bytes:
    """Bitstream of one frame; the depths below ``base`` are coded from their
    own symbol counts (base = 0: every depth through the model)."""
    xyz = _xyz(xyz)
    b = np.frombuffer(blob, np.uint8)
    L = lib()
    n = ctypes.c_size_t(0)
    st = L.orc_encode_base(_p(b), ctypes.c_size_t(len(blob)), _p(xyz), ctypes.c_int64(len(xyz)),
                           ctypes.c_int(chunk_log2), ctypes.c_int(base), None, ctypes.c_size_t(0), ctypes.byref(n))
    if st not in (OK, E_CAPACITY):
        raise OracleError(st)
    out = np.zeros(max(1, n.value), np.uint8)
    _chk(L.orc_encode_base(_p(b), ctypes.c_size_t(len(blob)), _p(xyz), ctypes.c_int64(len(xyz)),
                           ctypes.c_int(chunk_log2), ctypes.c_int(base), _p(out), ctypes.c_size_t(n.value),
                           ctypes.byref(n)))
    return out[:n.value].tobytes()


def counts_to_cdf(counts) -> np.ndarray:
    """CDF (int32 [256]) of a base depth from the counts of its 255 codes."""
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint32).reshape(255))
    out = np.zeros(256, np.int32)
    _chk(lib().orc_counts_to_cdf(_p(c), _p(out)))
    return out


def peek_header(bs: bytes):
    D, n = ctypes.c_int(), ctypes.c_int64()
    buf = np.frombuffer(bs, np.uint8)
    _chk(lib().orc_peek_header(_p(buf), ctypes.c_size_t(len(bs)), ctypes.byref(D), ctypes.byref(n)))
    return D.value, n.value


def decode(blob: bytes, bs: bytes) -> np.ndarray:
    """Voxel coordinates int32 [N_D, 3] in Morton order."""
    b = np.frombuffer(blob, np.uint8)
    buf = np.frombuffer(bs, np.uint8).copy() if len(bs) else np.zeros(1, np.uint8)
    n = ctypes.c_int64(0)
    L = lib()
    st = L.orc_decode(_p(b), ctypes.c_size_t(len(blob)), _p(buf), ctypes.c_size_t(len(bs)), None,
                      ctypes.c_int64(0), ctypes.byref(n))
    if st not in (OK, E_CAPACITY):
        raise OracleError(st)
    out = np.zeros((max(1, n.value), 3), np.int32)
    _chk(L.orc_decode(_p(b), ctypes.c_size_t(len(blob)), _p(buf), ctypes.c_size_t(len(bs)), _p(out),
                      ctypes.c_int64(n.value), ctypes.byref(n)))
    return out[:n.value]

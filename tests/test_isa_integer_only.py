"""The device code is integer-only and safe to run: the gfx950 assembly of every
kernel source has no floating-point instruction (the method's arithmetic is
int8/int32/int64 only, Sec. 3.3), no register spills to scratch, and no
writes through the scalar data cache.  Compiles the kernels for gfx950 with
the library's own flags (hipcc cross-compiles without a GPU)."""
import concurrent.futures
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2603_25260_amd import build as B

KERNEL_SOURCES = ["octree.hip", "model.hip", "rc.hip"]
# any VALU/SALU opcode on f16/f32/f64 data, conversions to or from float,
# reciprocal / transcendental units
FP = re.compile(r"^\s+(v_\w*_f(16|32|64)\w*|v_cvt_\w*f(16|32|64)\w*|v_(rcp|rsq|sqrt|exp|log|sin|cos|frexp|ldexp|div)\w*"
                r"|s_\w*_f(16|32)\w*)\b")
SCALAR_WRITE = re.compile(r"^\s+s_(store|buffer_store|scratch_store|atomic|buffer_atomic|dcache_wb|dcache_discard)\w*\b")


def _asm(src, out):
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [B.HIPCC, *flags, "--cuda-device-only", "-S", "-o", out, os.path.join(B.CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


@pytest.fixture(scope="module")
def asm():
    if not os.path.exists(B.HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        with concurrent.futures.ThreadPoolExecutor(len(KERNEL_SOURCES)) as ex:
            texts = list(ex.map(lambda s: _asm(s, os.path.join(d, s + ".s")), KERNEL_SOURCES))
    return dict(zip(KERNEL_SOURCES, texts))


def _kernels(text):
    """(name, body) of every function in an assembly listing."""
    out = []
    for m in re.finditer(r"^(_Z\w+):(.*?)^\.Lfunc_end\d+:", text, re.S | re.M):
        out.append((m.group(1), m.group(2)))
    return out


def test_every_source_has_kernels(asm):
    for src, text in asm.items():
        assert len(_kernels(text)) > 0, src


def test_no_floating_point_instructions(asm):
    bad = []
    for src, text in asm.items():
        for name, body in _kernels(text):
            for line in body.split("\n"):
                if FP.match(line):
                    bad.append((src, name, line.strip()))
    assert not bad, bad[:20]


def test_no_scalar_cache_writes(asm):
    bad = []
    for src, text in asm.items():
        for name, body in _kernels(text):
            for line in body.split("\n"):
                if SCALAR_WRITE.match(line):
                    bad.append((src, name, line.strip()))
    assert not bad, bad[:20]


def test_no_scratch_spills(asm):
    for src, text in asm.items():
        sizes = re.findall(r"\.set (\w+)\.private_seg_size, (\d+)", text)
        assert sizes, src
        spilled = [(k, v) for k, v in sizes if int(v) != 0]
        assert not spilled, (src, spilled)


def test_detector_sees_float_code():
    """The patterns recognise the instructions they are meant to catch."""
    assert FP.match("\tv_cvt_f32_u32_e32 v1, v2")
    assert FP.match("\tv_rcp_iflag_f32_e32 v1, v2")
    assert FP.match("\tv_max_f64 v[0:1], v[2:3], 0")
    assert not FP.match("\tv_mul_u32_u24_e32 v1, s2, v3")
    assert not FP.match("\tv_mfma_i32_16x16x64_i8 a[0:3], v[0:3], v[4:7], 0")
    assert SCALAR_WRITE.match("\ts_store_dword s0, s[2:3], 0x0")
    assert not SCALAR_WRITE.match("\ts_load_dword s0, s[2:3], 0x0")

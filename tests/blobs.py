"""Hand-built weight blobs for planted-weight tests (blob format only, no codec arithmetic)."""
import struct

import numpy as np

from paper_2603_25260_amd import synth


def build_blob(C, D, n_deep, fill, xfp=True):
    """Blob whose layer (kind, depth, j) gets the arrays ``fill(kind, depth, j, taps, cin, cout)``
    returns: dict with W [taps, cin, cout] int8, bias [cout] int32, m_pos, m_neg, r, z_in, z_out.
    ``xfp = False``: the schedule without cross-scale propagation (blob version 2)."""
    plan = synth.layer_plan(C, D, n_deep, xfp)
    out = bytearray(struct.pack("<6IQ", synth.BLOB_MAGIC, 1 if xfp else 2, C, D, n_deep, len(plan), 0))
    for (kind, depth, j, taps, cin, cout) in plan:
        p = fill(kind, depth, j, taps, cin, cout)
        W = np.asarray(p["W"], np.int8).reshape(taps, cin, cout)
        b = np.asarray(p["bias"], np.int32).reshape(cout)
        out += struct.pack("<6I2iI2i", kind, depth, j, taps, cin, cout, p["m_pos"], p["m_neg"], p["r"],
                           p.get("z_in", 0), p.get("z_out", 0))
        out += b.tobytes() + W.tobytes()
        while len(out) % 4:
            out += b"\0"
    return bytes(out)


def zeros(taps, cin, cout, r=20):
    """A layer computing 0 (zero weights and bias, unit gain)."""
    return {"W": np.zeros((taps, cin, cout)), "bias": np.zeros(cout), "m_pos": 1 << r, "m_neg": 1 << r, "r": r}


def with_fc2_bias(blob, sym, bias):
    """The same (unshared) blob with output ``sym`` of every predictor head
    (FC2) given bias ``bias``: a confident head whose logit ``sym`` sits at
    the top of the int8 range far above the others."""
    b = bytearray(blob)
    _, ver, _, _, _, nl, _ = struct.unpack_from("<6IQ", b, 0)
    assert not ver & synth.SHARED
    off = struct.calcsize("<6IQ")
    rec = struct.calcsize("<6I2iI2i")
    for _ in range(nl):
        kind, _, _, taps, cin, cout = struct.unpack_from("<6I", b, off)
        off += rec
        if kind == synth.FC2:
            struct.pack_into("<i", b, off + 4 * sym, bias)
        off += 4 * cout + taps * cin * cout
        off += -off % 4
    return bytes(b)

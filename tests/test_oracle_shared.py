"""Level-aware parameter sharing (the future work named in the last paragraph
of Sec. S2, "Detailed Model Structure": neural blocks whose parameters are
shared across octree levels).  Reading: the layers of one role share one
int8 weight tensor across depths (the predictor's two layers at every depth;
per kind the shallow depths d <= k0 and the deep depths d > k0 apart) while
every layer keeps its own bias and requantisation, which is what makes a
shared block level-aware.  A shared blob stores each tensor once and every
record names the layer whose weights it uses.

Pins (CPU):
* sharing is a storage form: the shared blob and the unshared blob holding
  the owners' weights in every record give the same CDF rows at every depth,
  and the same stream payload;
* the blob size follows from the layer list (owners store weights, the rest
  an index);
* the weights really are shared (equal tensors within a role) while the
  biases stay per depth;
* the library's generator writes the same bytes as the seeded generator;
* the second numpy transcription of the model gives the oracle's logits on a
  shared blob;
* both parsers reject an owner index that points forward, at a layer of
  another shape, or at a layer that does not own its weights.
"""
import struct

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth
from tests.codec_ref import level_logits_all, parse_blob


def _records(blob):
    """(header, [(fixed 44 bytes, owner, bias bytes, W bytes or None)])"""
    version = struct.unpack_from("<I", blob, 4)[0]
    n_layers = struct.unpack_from("<I", blob, 20)[0]
    off, recs = 32, []
    for li in range(n_layers):
        fixed = blob[off:off + 44]
        kind, depth, j, taps, cin, cout = struct.unpack_from("<6I", blob, off)
        off += 44
        owner = li
        if version & 0x100:
            owner = struct.unpack_from("<I", blob, off)[0]
            off += 4
        bias = blob[off:off + 4 * cout]
        off += 4 * cout
        W = None
        if owner == li:
            W = blob[off:off + taps * cin * cout]
            off += taps * cin * cout
        off = (off + 3) & ~3
        recs.append((fixed, owner, bias, W))
    assert off == len(blob)
    return blob[:32], recs


def _expand(blob):
    """The unshared blob with every record holding its owner's weights."""
    head, recs = _records(blob)
    version = struct.unpack_from("<I", head, 4)[0] & 0xFF
    out = bytearray(head[:4] + struct.pack("<I", version) + head[8:])
    for fixed, owner, bias, W in recs:
        out += fixed + bias + (W if W is not None else recs[owner][3])
        while len(out) % 4:
            out += b"\0"
    return bytes(out)


CASES = [(16, 7, 3, True, False), (16, 8, 4, False, False), (32, 7, 2, True, True)]


@pytest.mark.parametrize("C,D,nd,xfp,zp", CASES)
def test_shared_equals_expanded(C, D, nd, xfp, zp):
    shared = synth.make_weights(5, C, D, nd, xfp=xfp, zero_points=zp, shared=True)
    expanded = _expand(shared)
    # the expanded blob is the unshared draw with the owners' weights copied in
    plain = synth.make_weights(5, C, D, nd, xfp=xfp, zero_points=zp)
    assert len(expanded) == len(plain)
    assert expanded != plain  # the shared weights replace per-depth ones
    xyz = synth.random_cloud(600, D, 11)
    for d in range(D):
        assert np.array_equal(O.level_probs(shared, xyz, d), O.level_probs(expanded, xyz, d)), d
    a, b = O.encode(shared, xyz, 6), O.encode(expanded, xyz, 6)
    hs = 16 + 4 * D  # magic, version, D, n_deep, c, blob id, N_D, the depth counts
    assert a[:8] == b[:8] and a[12:] == b[12:]  # only the blob id differs
    assert len(a) > hs
    dec = O.decode(shared, a)
    u = np.unique(xyz, axis=0)
    assert np.array_equal(dec, u[np.argsort(O.morton(u, D))])


def test_shared_blob_size_and_roles():
    C, D, nd = 32, 10, 4
    k0 = D - nd - 1
    blob = synth.make_weights(1, C, D, nd, shared=True)
    plan = synth.layer_plan(C, D, nd)
    owner = synth.weight_owners(C, D, nd)
    want = 32
    for li, (kind, depth, j, taps, cin, cout) in enumerate(plan):
        want += 48 + 4 * cout + (taps * cin * cout if owner[li] == li else 0)
        want = (want + 3) & ~3
    assert len(blob) == want
    assert len(blob) < len(synth.make_weights(1, C, D, nd)) / 3
    _, _, _, L = parse_blob(blob)
    fc1 = [L[(synth.FC1, d, d)] for d in range(D)]
    assert all(np.array_equal(f["W"], fc1[0]["W"]) for f in fc1)
    assert len({f["b"].tobytes() for f in fc1}) == D  # level-aware: per-depth biases
    shallow_up = [L[(synth.UP, d, d - 1)]["W"] for d in range(1, k0 + 1)]
    deep_up = [L[(synth.UP, d, j)]["W"] for d in range(k0 + 1, D) for j in range(k0, d)]
    assert all(np.array_equal(w, shallow_up[0]) for w in shallow_up)
    assert all(np.array_equal(w, deep_up[0]) for w in deep_up)
    assert not np.array_equal(shallow_up[0], deep_up[0])  # shallow and deep roles apart
    downs = [L[(synth.DOWN, d, j)]["W"] for d in range(k0 + 2, D) for j in range(d - 1, k0, -1)]
    assert len(downs) > 1 and all(np.array_equal(w, downs[0]) for w in downs)


@pytest.mark.parametrize("C,D,nd,xfp,zp", CASES)
def test_library_generator_matches(C, D, nd, xfp, zp):
    from paper_2603_25260_amd import lpcc
    want = synth.make_weights(1, C, D, nd, xfp=xfp, zero_points=zp, shared=True)
    assert lpcc.make_weights(1, C, D, nd, xfp=xfp, zero_points=zp, shared=True) == want


def test_numpy_transcription_on_shared_blob():
    C, D, nd = 16, 6, 2
    blob = synth.make_weights(3, C, D, nd, shared=True)
    xyz = synth.random_cloud(150, D, 4)
    ref = level_logits_all(blob, xyz)
    for d in range(D):
        assert np.array_equal(np.asarray(ref[d]), O.level_logits(blob, xyz, d)), d


def _with_owner(blob, li, owner):
    """Rewrite the owner index of record li (records keep their lengths only
    when li and the new owner both reference; used on referencing records)."""
    head, recs = _records(blob)
    out = bytearray(head)
    for k, (fixed, own, bias, W) in enumerate(recs):
        out += fixed + struct.pack("<I", owner if k == li else own) + bias + (W if W is not None else b"")
        while len(out) % 4:
            out += b"\0"
    return bytes(out)


def test_bad_owner_rejected():
    from paper_2603_25260_amd import lpcc
    C, D, nd = 16, 7, 3
    blob = synth.make_weights(1, C, D, nd, shared=True)
    plan = synth.layer_plan(C, D, nd)
    owner = synth.weight_owners(C, D, nd)
    refs = [i for i in range(len(plan)) if owner[i] != i]
    li = refs[0]
    fc2 = [i for i, p in enumerate(plan) if p[0] == synth.FC2]
    bad = [
        _with_owner(blob, li, li + 1),  # forward reference
        _with_owner(blob, fc2[1], owner[[i for i, p in enumerate(plan) if p[0] == synth.FC1][0]]),  # other shape
        _with_owner(blob, fc2[2], fc2[1]),  # a layer that does not own its weights
    ]
    xyz = synth.random_cloud(100, D, 1)
    for b in bad:
        with pytest.raises(O.OracleError):
            O.level_probs(b, xyz, 0)
        with pytest.raises(lpcc.LpccError):
            lpcc.Model(b, 0)

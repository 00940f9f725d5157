"""Seeded synthetic inputs: spinning-LiDAR scans and random-init integer weight blobs.

This module holds no part of the codec's arithmetic.  It only draws inputs that
both the GPU library and the CPU oracle consume:

* ``make_scan(cfg, seed)`` casts the rays of a spinning multi-beam LiDAR into a
  scene (ground plane, axis-aligned boxes, an enclosing wall), adds range noise
  and dropout, and quantises the hits to int32 voxel coordinates in
  ``[0, 2**D)**3``.  The paper's datasets (KITTI, Ford; Sec. 4.1) are not
  available; these scans stand in for them with the same structure (rings of
  points, ground, box-like obstacles) and comparable point counts.
* ``make_weights(seed, C, D, n_deep)`` writes the weight blob: one record per
  layer of the per-depth model (int8 weights, int32 bias, multiply/shift
  requantisation parameters, zero points; Sec. 3.3, Eq. 12-14).  Values come
  from SplitMix64 (Steele, Lea & Flood, 2014), a counter-based generator, so
  the blob is a pure function of its arguments.

The blob layout (little-endian) is::

    u32 magic 'LPCW', u32 version=1, u32 C, u32 D, u32 n_deep, u32 n_layers,
    u64 seed
    n_layers records:
      u32 kind, u32 depth, u32 j, u32 taps, u32 cin, u32 cout,
      i32 m_pos, i32 m_neg, u32 r, i32 z_in, i32 z_out,
      [version flag 0x100 (shared weights): u32 owner],
      i32 bias[cout], i8 W[taps][cin][cout] (only when the layer owns its
      weights), zero padding to 4 bytes

Layer kinds and their order per coded depth d (k0 = D - n_deep - 1):

* d = 0: FC1, FC2
* 1 <= d <= k0: CONV1 (27 x C -> C), CONV2 (27 x C -> C), UP (C+8 -> 8C), FC1, FC2
* d > k0: EMB (8 -> C), DOWN j = d-1 .. k0+1 (8 x C -> C), CONV1 (27 x 2C -> C),
  CONV2, SKIP (2C -> C), UP j = k0 .. d-1, FC1, FC2
"""
from __future__ import annotations

import dataclasses
import math
import struct

import numpy as np

# ----------------------------------------------------------------------------
# Layer kinds (shared vocabulary of the blob format)
# ----------------------------------------------------------------------------
EMB, DOWN, CONV1, CONV2, SKIP, UP, FC1, FC2 = 1, 2, 3, 4, 5, 6, 7, 8
KIND_NAMES = {EMB: "emb", DOWN: "down", CONV1: "conv1", CONV2: "conv2",
              SKIP: "skip", UP: "up", FC1: "fc1", FC2: "fc2"}
# activation folded into the requantisation multiplier for negative inputs
ACT_RELU, ACT_IDENT, ACT_PRELU = 0, 1, 2
KIND_ACT = {EMB: ACT_RELU, DOWN: ACT_RELU, CONV1: ACT_RELU, CONV2: ACT_IDENT,
            SKIP: ACT_IDENT, UP: ACT_PRELU, FC1: ACT_RELU, FC2: ACT_IDENT}

BLOB_MAGIC = 0x5743504C  # b"LPCW"
N_SYMBOLS = 255


def layer_plan(C: int, D: int, n_deep: int, xfp: bool = True):
    """List of (kind, depth, j, taps, cin, cout) in blob order.

    ``xfp = False`` is the ablation without cross-scale feature propagation
    (blob version 2): the features of depth d come from the codes of depth
    d-1 alone (an embedding of X_{d-1}, a ResBlock with identity skip, the
    upsampling), and the deep ResBlock reads G alone (C -> C, identity skip,
    no skip layer).  With n_deep = 0 as well it is the ablation's baseline."""
    if not (1 <= D <= 21):
        raise ValueError("D must be in [1, 21]")
    if not (0 <= n_deep <= D - 1):
        raise ValueError("n_deep must be in [0, D-1]")
    k0 = D - n_deep - 1
    plan = []
    for d in range(D):
        if d == 0:
            pass
        elif d <= k0:
            if not xfp:
                plan.append((EMB, d, d - 1, 1, 8, C))
            plan += [(CONV1, d, 0, 27, C, C), (CONV2, d, 0, 27, C, C),
                     (UP, d, d - 1, 1, C + 8, 8 * C)]
        else:
            plan.append((EMB, d, d - 1, 1, 8, C))
            for j in range(d - 1, k0, -1):
                plan.append((DOWN, d, j, 8, C, C))
            if xfp:
                plan += [(CONV1, d, k0, 27, 2 * C, C), (CONV2, d, k0, 27, C, C),
                         (SKIP, d, k0, 1, 2 * C, C)]
            else:
                plan += [(CONV1, d, k0, 27, C, C), (CONV2, d, k0, 27, C, C)]
            for j in range(k0, d):
                plan.append((UP, d, j, 1, C + 8, 8 * C))
        plan += [(FC1, d, d, 1, C, C), (FC2, d, d, 1, C, N_SYMBOLS)]
    return plan


# ----------------------------------------------------------------------------
# SplitMix64, counter form: output k (k >= 1) = mix(seed + k * gamma)
# ----------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, start: int, n: int) -> np.ndarray:
    """Outputs start+1 .. start+n of SplitMix64 seeded with ``seed``."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


SHARED = 0x100  # version flag: layers may take their weights from an earlier layer


def weight_owners(C: int, D: int, n_deep: int, xfp: bool = True):
    """Level-aware parameter sharing: for every layer of the plan, the index
    of the layer whose weights it uses.  Layers of one role share one weight
    tensor across depths: the predictor's two layers at every depth, and per
    kind the layers of the shallow depths (d <= k0) and those of the deep
    depths (d > k0) apart (their inputs differ: [S | bits] vs [Z | bits],
    F vs [F_k0 | G]).  The first layer of a role in blob order owns the
    weights; every layer keeps its own bias and requantisation, which is what
    makes a shared block level-aware (a one-hot level input through a linear
    layer is exactly a per-level bias)."""
    k0 = D - n_deep - 1
    owner, first = [], {}
    for i, (kind, depth, j, taps, cin, cout) in enumerate(layer_plan(C, D, n_deep, xfp)):
        role = (kind,) if kind in (FC1, FC2) else (kind, depth > k0)
        owner.append(first.setdefault(role, i))
    return owner


def make_weights(seed: int, C: int, D: int, n_deep: int, *,
                 zero_points: bool = False, gain: float = 1.0,
                 shift: int = 24, xfp: bool = True, shared: bool = False) -> bytes:
    """Random-init integer weight blob for channel width C and D levels.

    W ~ uniform integers in [-127, 127]; bias uniform in [-4096, 4096];
    m_pos chosen so that a layer roughly keeps the spread of its input
    (``gain`` / (73.6 * sqrt(fan_in)) at shift ``shift``); ReLU layers get
    m_neg = 0, identity layers m_neg = m_pos, PReLU layers (slope 64/256)
    m_neg = (m_pos * 64) >> 8.  With ``zero_points`` every layer also gets
    input/output zero points in [-8, 8] (to exercise that part of Eq. 13-14).
    With ``shared`` the blob shares weights across depths (``weight_owners``;
    version flag SHARED): each record carries a u32 owner index after z_out
    and holds weights only when it owns them.  The draws are the same as for
    the unshared blob, so a shared blob equals the unshared one with every
    layer's weights replaced by its owner's.
    """
    plan = layer_plan(C, D, n_deep, xfp)
    owner = weight_owners(C, D, n_deep, xfp) if shared else list(range(len(plan)))
    out = bytearray()
    out += struct.pack("<6IQ", BLOB_MAGIC, (1 if xfp else 2) | (SHARED if shared else 0), C, D, n_deep, len(plan),
                       seed)
    ctr = 0
    for li, (kind, depth, j, taps, cin, cout) in enumerate(plan):
        nW = taps * cin * cout
        u = splitmix64(seed, ctr, nW + cout + 2)
        ctr += nW + cout + 2
        hi = (u >> np.uint64(33)).astype(np.int64)
        W = (hi[:nW] % 255 - 127).astype(np.int8)
        b = (hi[nW:nW + cout] % 8193 - 4096).astype(np.int32)
        fan_in = taps * cin
        m_pos = int(math.floor((1 << shift) * gain / (73.6 * math.sqrt(fan_in))))
        if kind == FC2:
            m_pos = int(m_pos * 0.75)  # logits mostly inside the int8 range
        act = KIND_ACT[kind]
        m_neg = 0 if act == ACT_RELU else (m_pos if act == ACT_IDENT else (m_pos * 64) >> 8)
        if zero_points:
            z_in = int(hi[nW + cout] % 17) - 8
            z_out = int(hi[nW + cout + 1] % 17) - 8
        else:
            z_in = z_out = 0
        out += struct.pack("<6I2iI2i", kind, depth, j, taps, cin, cout,
                           m_pos, m_neg, shift, z_in, z_out)
        if shared:
            out += struct.pack("<I", owner[li])
        out += b.tobytes()
        if owner[li] == li:
            out += W.tobytes()
        while len(out) % 4:
            out += b"\0"
    return bytes(out)


# ----------------------------------------------------------------------------
# Synthetic spinning-LiDAR scans
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class ScanSpec:
    beams: int
    elev_deg: tuple          # (min, max), beams evenly spaced over it
    azimuths: int
    boxes: int
    r_max: float             # metres; an enclosing wall stands just inside it
    D: int                   # octree levels
    voxel: float             # metres per voxel
    noise: float = 0.02      # range noise sigma, metres
    dropout: float = 0.10    # per-ray dropout probability
    ground_z: float = -1.7


@dataclasses.dataclass(frozen=True)
class CodecConfig:
    name: str
    scan: ScanSpec
    C: int
    n_deep: int
    seeds: tuple
    weight_seed: int = 1


ELEV_BY_BEAMS = {16: (-15.0, 15.0), 32: (-30.0, 10.0), 64: (-24.8, 2.0), 128: (-25.0, 15.0)}

CONFIGS = {
    # 16-beam scan, 12-level octree, C=16
    "cfg1": CodecConfig("16beam_D12_C16",
                        ScanSpec(16, (-15.0, 15.0), 1024, 20, 80.0, 12, 160.0 / 4096),
                        C=16, n_deep=4, seeds=tuple(range(1001, 1017))),
    # 64-beam scan, 14-level octree at 1 cm, C=32
    "cfg2": CodecConfig("64beam_D14_C32",
                        ScanSpec(64, (-24.8, 2.0), 2048, 60, 80.0, 14, 0.01),
                        C=32, n_deep=4, seeds=tuple(range(2001, 2009))),
    # 128-beam scan, 18-level octree at 1 mm, C=64, 5 deep levels
    "cfg4": CodecConfig("128beam_D18_C64",
                        ScanSpec(128, (-25.0, 15.0), 2048, 60, 120.0, 18, 0.001),
                        C=64, n_deep=5, seeds=tuple(range(4001, 4009))),
}


def batch_scan_spec(seed: int, D: int = 14, voxel: float = 0.01) -> ScanSpec:
    """Per-frame scene of the uneven batch: beams in {16,32,64}, 1024-2048
    azimuth steps, 20-60 boxes, all drawn from ``seed``."""
    rng = np.random.default_rng(seed)
    beams = int(rng.choice([16, 32, 64]))
    az = int(rng.integers(1024, 2049))
    boxes = int(rng.integers(20, 61))
    return ScanSpec(beams, ELEV_BY_BEAMS[beams], az, boxes, 80.0, D, voxel)


def fleet_spec(n_sensors: int, seed: int, depths=(14, 15, 16, 17, 18), beams=(16, 32, 64, 128)):
    """(beams, D) of every simulated sensor of a serving fleet, drawn from ``seed``."""
    rng = np.random.default_rng(seed)
    return [(int(rng.choice(beams)), int(rng.choice(depths))) for _ in range(n_sensors)]


def fleet_model(D: int):
    """(C, D, n_deep) of the model a fleet sensor of depth D uses: C = 32 up
    to 16 levels, 64 beyond; four re-densified depths."""
    return (32 if D <= 16 else 64), D, 4


def fleet_scan_spec(beams: int, D: int, azimuths: int = 2048) -> ScanSpec:
    """Scene of one fleet sensor: its beam count, 40 boxes, voxel 163.84 m / 2^D."""
    return ScanSpec(beams, ELEV_BY_BEAMS[beams], azimuths, 40, 80.0, D, 163.84 / (2 ** D))


def fleet_frame_seed(seed: int, sensor: int, k: int) -> int:
    """Scan seed of frame k of sensor ``sensor`` in the fleet drawn from ``seed``."""
    return seed + 1 + 100 * sensor + k


def _scene(spec: ScanSpec, rng: np.random.Generator):
    """Axis-aligned boxes standing on the ground: (lo[3], hi[3]) arrays."""
    n = spec.boxes
    box_range = 0.6 * spec.r_max
    centres = np.zeros((n, 2))
    k = 0
    while k < n:
        c = rng.uniform(-box_range, box_range, size=2)
        if np.hypot(c[0], c[1]) >= 3.0 + 6.0:
            centres[k] = c
            k += 1
    half = rng.uniform(1.0, 6.0, size=(n, 2))
    height = rng.uniform(1.5, 15.0, size=n)
    lo = np.stack([centres[:, 0] - half[:, 0], centres[:, 1] - half[:, 1],
                   np.full(n, spec.ground_z)], axis=1)
    hi = np.stack([centres[:, 0] + half[:, 0], centres[:, 1] + half[:, 1],
                   spec.ground_z + height], axis=1)
    return lo, hi


def make_points(spec: ScanSpec, seed: int) -> np.ndarray:
    """Float64 [n, 3] hit points in metres (sensor at the origin)."""
    rng = np.random.default_rng(seed)
    lo, hi = _scene(spec, rng)
    elev = np.deg2rad(np.linspace(spec.elev_deg[0], spec.elev_deg[1], spec.beams))
    az = 2.0 * np.pi * np.arange(spec.azimuths) / spec.azimuths
    E, A = np.meshgrid(elev, az, indexing="ij")
    dirs = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1).reshape(-1, 3)
    nr = dirs.shape[0]
    t = np.full(nr, np.inf)
    # ground plane
    dz = dirs[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(dz < -1e-9, spec.ground_z / dz, np.inf)
    t = np.minimum(t, tg)
    # enclosing cylindrical wall just inside r_max
    r_wall = 0.95 * spec.r_max
    horiz = np.hypot(dirs[:, 0], dirs[:, 1])
    with np.errstate(divide="ignore"):
        tw = np.where(horiz > 1e-9, r_wall / horiz, np.inf)
    t = np.minimum(t, tw)
    # boxes: slab test (direction components of exactly 0 get a huge inverse)
    safe = np.where(np.abs(dirs) < 1e-12, 1e-12, dirs)
    inv = 1.0 / safe
    for b in range(lo.shape[0]):
        t1 = lo[b][None, :] * inv
        t2 = hi[b][None, :] * inv
        tn = np.minimum(t1, t2)
        tf = np.maximum(t1, t2)
        tmin = np.maximum(np.maximum(tn[:, 0], tn[:, 1]), tn[:, 2])
        tmax = np.minimum(np.minimum(tf[:, 0], tf[:, 1]), tf[:, 2])
        hit = (tmax >= tmin) & (tmin > 0.0) & (tmin < t)
        t = np.where(hit, tmin, t)
    valid = np.isfinite(t) & (t <= spec.r_max)
    keep = valid & (rng.random(nr) >= spec.dropout)
    rng_noise = rng.normal(0.0, spec.noise, size=nr)
    r = t + rng_noise
    pts = dirs * r[:, None]
    return pts[keep]


def quantise(points: np.ndarray, D: int, voxel: float) -> np.ndarray:
    """Voxel coordinates: floor((p + 2^(D-1) * voxel) / voxel), clamped."""
    v = np.floor((points + (2 ** (D - 1)) * voxel) / voxel)
    v = np.clip(v, 0, 2 ** D - 1)
    return v.astype(np.int32)


def make_scan(spec: ScanSpec, seed: int) -> np.ndarray:
    """int32 [n, 3] voxel coordinates of one synthetic scan (duplicates kept)."""
    return np.ascontiguousarray(quantise(make_points(spec, seed), spec.D, spec.voxel))


def random_cloud(n: int, D: int, seed: int, *, clustered: bool = True) -> np.ndarray:
    """Small random voxel sets for unit tests: clustered blobs or uniform."""
    rng = np.random.default_rng(seed)
    side = 2 ** D
    if n == 0:
        return np.zeros((0, 3), np.int32)
    if not clustered:
        return rng.integers(0, side, size=(n, 3)).astype(np.int32)
    n_cent = max(1, n // 32)
    cent = rng.integers(0, side, size=(n_cent, 3))
    pick = rng.integers(0, n_cent, size=n)
    spread = max(1, side // 64)
    pts = cent[pick] + rng.integers(-spread, spread + 1, size=(n, 3))
    return np.clip(pts, 0, side - 1).astype(np.int32)

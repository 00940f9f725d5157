"""The benchmark's algorithmic-work counts against the oracle: node counts per
depth and present 3x3x3 neighbour pairs (self included) from bench.octree_stats
equal the oracle's octree and neighbour tables, and bench.expected_decode is
the oracle's Morton order of the unique voxels."""
import numpy as np
import pytest

import bench
from oracle import oracle as O
from paper_2603_25260_amd import synth


@pytest.mark.parametrize("name,n", [("cfg1", None), ("cfg2", 20000)])
def test_octree_stats_match_oracle(name, n):
    cfg = synth.CONFIGS[name]
    D = cfg.scan.D
    k0 = D - cfg.n_deep - 1
    xyz = synth.make_scan(cfg.scan, cfg.seeds[0])[:n]
    N, P = bench.octree_stats(xyz, D, k0)
    counts, V, _ = O.octree(xyz, D)
    assert list(N) == list(counts)
    assert [int(p) for p in P] == [int((O.kernel_map(V[j], j) >= 0).sum()) for j in range(k0 + 1)]


def test_expected_decode_is_morton_order():
    xyz = synth.random_cloud(3000, 9, 7)
    u = np.unique(xyz, axis=0)
    assert np.array_equal(bench.expected_decode(xyz, 9), u[np.argsort(O.morton(u, 9))])


def test_frame_work_closed_form_single_voxel():
    # one voxel: one node per depth, one pair (itself) per depth
    D, C, nd = 6, 16, 2
    N, P = bench.octree_stats(np.array([[5, 9, 33]], np.int32), D, D - nd - 1)
    assert list(N) == [1] * (D + 1) and list(P) == [1] * (D - nd)
    w = bench.frame_work(N, P, C, D, nd)
    k0 = D - nd - 1
    assert w["conv"]["macs"] == k0 * 2 * C * C + nd * 3 * C * C
    assert w["predict"]["macs"] == D * (C * C + 255 * C)
    assert w["up"]["macs"] == (k0 + sum(d - k0 for d in range(k0 + 1, D))) * (C + 8) * C


def test_source_digest_ignores_comments_only():
    """The profiled-traffic table is tied to the library's code: a comment or
    blank-line edit keeps the digest's input, any code edit changes it."""
    a = "int f(int x) {  // doubles\n  return 2 * x;\n}\n"
    b = "// a new note\nint f(int x) {\n\n  return 2 * x;   // still doubles\n}\n"
    c = "int f(int x) {\n  return 3 * x;\n}\n"
    assert bench.code_lines(a) == bench.code_lines(b)
    assert bench.code_lines(a) != bench.code_lines(c)
    assert len(bench.library_sources_digest()) == 16

"""Graph mode: the launch batches of every call are captured into HIP graphs
and replayed (executable graphs updated in place between calls).  Every
replay must give the eager path's bytes and points, with eager work and
synchronisations of the program in between, for frames of different sizes
(new instantiation) and of the same size (in-place update), and for batches."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_25260_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_25260_amd import lpcc
    lpcc.lib()
    return lpcc


def _sorted_unique(xyz, D):
    u = np.unique(xyz, axis=0)
    return u[np.argsort(O.morton(u, D))]


def test_graph_replays_match_eager(L):
    C, D, n_deep = 32, 11, 4
    blob = synth.make_weights(9, C, D, n_deep)
    m = L.Model(blob, 0)
    eager = L.Context(0)
    eager.set_tiling(1)
    g = L.Context(0)
    g.set_tiling(1)  # fixed tiles: every call of a shape has the same launch sequence
    g.set_graphs(True)
    frames = [synth.random_cloud(n, D, 40 + i) for i, n in enumerate((6000, 6000, 2500, 9000))]
    want = [O.encode(blob, f, 8) for f in frames[:2]]
    for rep in range(3):
        for i, f in enumerate(frames):
            print("graph replay", rep, "frame", i, flush=True)
            dx = torch.from_numpy(f).cuda()
            ref = L.encode_frame(eager, m, dx, 8)          # eager work in between
            torch.cuda.synchronize()
            got = L.encode_frame(g, m, dx, 8)
            assert got == ref, f"encode rep {rep} frame {i}"
            if i < 2:
                assert got == want[i]
            dec = L.decode_frame(g, m, got)
            assert np.array_equal(dec, _sorted_unique(f, D)), f"decode rep {rep} frame {i}"
    st = g.graph_stats()
    print(st, flush=True)
    assert st["instantiated"] >= 1 and st["updated"] >= 1


def test_graph_batches_match_eager(L):
    C, D, n_deep = 16, 10, 3
    blob = synth.make_weights(3, C, D, n_deep)
    m = L.Model(blob, 0)
    frames = [torch.from_numpy(synth.random_cloud(n, D, 70 + n)).cuda() for n in (1500, 4000, 700, 2600)]
    eager = L.Context(0)
    ref, st = L.encode_batch(eager, m, frames, 7)
    assert st == [0] * 4
    g = L.Context(0)
    g.set_graphs(True)
    for rep in range(3):
        print("graph batch", rep, flush=True)
        got, st = L.encode_batch(g, m, frames, 7)
        assert st == [0] * 4 and got == ref
        dec, st = L.decode_batch(g, m, got)
        assert st == [0] * 4
        for f, x in zip(frames, dec):
            assert np.array_equal(x, _sorted_unique(f.cpu().numpy(), D))
        torch.cuda.synchronize()

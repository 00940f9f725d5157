"""The allocation-free encode entry point (lpcc_encode_frame_noalloc, static
device workspace) against lpcc_encode_frame on the same context: identical
bytes on two calls in a row, the second with a smaller input, for host and
device inputs and outputs; no device memory taken by its calls; a frame whose
workspace exceeds the static block is refused with LPCC_E_NOMEM before any
work, and the entry point stays usable afterwards."""
import numpy as np
import pytest

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


def _noalloc_dev(L, ctx, m, dx, want_len, cl):
    out = torch.full((want_len + 4096,), 0xA5, dtype=torch.uint8, device="cuda")
    n = L.encode_frame_noalloc(ctx, m, dx, out, cl)
    assert bool((out[n:] == 0xA5).all()), "bytes written past the stream"
    return bytes(out[:n].cpu().numpy())


@pytest.mark.parametrize("name,n_small", [("cfg1", 3000), ("cfg2", 20000)])
def test_noalloc_equals_encode_frame(L, name, n_small):
    cfg = synth.CONFIGS[name]
    m = L.Model(synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), 0)
    ctx = L.Context(0)
    big = synth.make_scan(cfg.scan, cfg.seeds[0])
    small = np.ascontiguousarray(big[::max(1, len(big) // n_small)][:n_small])
    cl = 8
    frames = [big, small]  # second call with the smaller input
    devs = [torch.from_numpy(f).cuda() for f in frames]
    want = [L.encode_frame(ctx, m, d, cl) for d in devs]
    held, _ = ctx.workspace()
    print(f"{name}: {len(big)} and {len(small)} points; context workspace {held} bytes", flush=True)
    # warm calls (device and host buffers): nothing new is loaded afterwards
    assert _noalloc_dev(L, ctx, m, devs[1], len(want[1]), cl) == want[1]
    warm = np.zeros(len(want[1]) + 64, np.uint8)
    assert warm[:L.encode_frame_noalloc(ctx, m, frames[1], warm, cl)].tobytes() == want[1]
    outs = [torch.zeros(len(w) + 4096, dtype=torch.uint8, device="cuda") for w in want]
    hout = [np.zeros(len(w) + 64, np.uint8) for w in want]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    lens = []
    for d, o in zip(devs, outs):
        lens.append(L.encode_frame_noalloc(ctx, m, d, o, cl))
    hlens = []
    for f, o in zip(frames, hout):  # host input and host output
        hlens.append(L.encode_frame_noalloc(ctx, m, f, o, cl))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, f"device memory changed by {free0 - free1} bytes"
    for i, w in enumerate(want):
        assert bytes(outs[i][:lens[i]].cpu().numpy()) == w, (name, i)
        assert hout[i][:hlens[i]].tobytes() == w, (name, i)
    # again in the opposite order: the block keeps the last call's contents
    assert _noalloc_dev(L, ctx, m, devs[0], len(want[0]), cl) == want[0]
    assert _noalloc_dev(L, ctx, m, devs[1], len(want[1]), cl) == want[1]


def test_noalloc_refuses_oversized_frame(L):
    cfg = synth.CONFIGS["cfg1"]
    m = L.Model(synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), 0)
    ctx = L.Context(0)
    # 24M points: the octree phase alone needs more than the static block
    huge = np.zeros((24_000_000, 3), np.int32)
    out = np.zeros(1 << 20, np.uint8)
    with pytest.raises(L.LpccError) as ei:
        L.encode_frame_noalloc(ctx, m, huge, out, 8)
    assert ei.value.code == L.E_NOMEM
    assert "static block" in str(ei.value)
    xyz = synth.make_scan(cfg.scan, cfg.seeds[1])
    want = L.encode_frame(ctx, m, xyz, 8)
    got = np.zeros(len(want) + 64, np.uint8)
    n = L.encode_frame_noalloc(ctx, m, xyz, got, 8)
    assert got[:n].tobytes() == want

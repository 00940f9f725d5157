"""Serving: continuous batching through lpcc_server_*.  Every result equals the
same job run alone (byte for byte); a small memory budget forces admission
control; jobs from several models and both kinds mix in flight."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_25260_amd import lpcc
    lpcc.lib()
    return lpcc


def test_served_equals_alone_small_fleet(L):
    from paper_2603_25260_amd import serve
    print("serving: 6 sensors, 2 s", flush=True)
    rep = serve.run(duration_s=2.0, n_sensors=6, rate_hz=20.0, seed=77, slots=3, max_batch=3, chunk_log2=8,
                    frames_per_sensor=2, verify=True, depths=(10, 11, 12), beams=(16, 32), azimuths=1024,
                    realtime=False)
    sys.stdout.write(f"{rep}\n")
    assert rep["requests"] > 0 and rep["ok"] == rep["requests"]
    assert rep["mismatches_vs_alone"] == 0
    assert rep["encode_jobs"] > 0 and rep["decode_jobs"] > 0


def test_admission_with_small_budget(L):
    """A budget that holds about one job at a time still completes everything,
    with results equal to the isolated calls."""
    from paper_2603_25260_amd import serve
    print("serving: tight budget", flush=True)
    rep = serve.run(duration_s=1.0, n_sensors=4, rate_hz=20.0, seed=78, slots=3, max_batch=4, chunk_log2=8,
                    frames_per_sensor=1, verify=True, depths=(10, 11), beams=(16,), azimuths=1024,
                    hbm_budget=48 << 20, realtime=False)
    sys.stdout.write(f"{rep}\n")
    assert rep["ok"] == rep["requests"] and rep["mismatches_vs_alone"] == 0
    assert 0 < rep["bytes_peak"] <= rep["budget_bytes"] == 48 << 20


def test_context_budget(L):
    """A context capped below what a frame needs fails with LPCC_E_NOMEM and
    stays usable; with room it encodes the same stream, and its workspace
    never exceeds the cap."""
    from paper_2603_25260_amd import synth
    D, C = 10, 16
    blob = synth.make_weights(3, C, D, 3)
    m = L.Model(blob, 0)
    xyz = synth.random_cloud(3000, D, 31)
    tight = L.Context(0, hbm_budget=1 << 20)
    with pytest.raises(L.LpccError) as e:
        L.encode_frame(tight, m, xyz, 8)
    assert e.value.code == L.E_NOMEM and "budget" in str(e.value)
    ref = L.encode_frame(L.Context(0), m, xyz, 8)
    roomy = L.Context(0, hbm_budget=64 << 20)
    assert L.encode_frame(roomy, m, xyz, 8) == ref == O.encode(blob, xyz, 8)
    held, peak = roomy.workspace()
    assert 0 < held <= peak <= 64 << 20


def test_served_streams_match_oracle(L):
    """Streams produced by the server decode with the CPU oracle."""
    from paper_2603_25260_amd import synth
    D, C = 9, 16
    blob = synth.make_weights(5, C, D, 3)
    m = L.Model(blob, 0)
    srv = L.Server([m], 0, slots=2, max_batch=2)
    frames = [synth.random_cloud(n, D, 900 + n) for n in (300, 1200, 50, 800)]
    outs = [np.zeros(64 * len(f) + 4096, np.uint8) for f in frames]
    tk = [srv.submit(0, 0, f, o, chunk_log2=6) for f, o in zip(frames, outs)]
    srv.drain()
    done = {d["ticket"]: d for d in srv.poll(16)}
    for t, f, o in zip(tk, frames, outs):
        d = done[t]
        assert d["status"] == 0
        bs = o[:d["out_len"]].tobytes()
        assert bs == O.encode(blob, f, 6)
    srv.close()

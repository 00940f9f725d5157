"""Write tests/golden/digests.json: sha256 digests of CPU-oracle outputs for
full-size synthetic frames, so that GPU tests and the benchmark can check
frames whose oracle run takes minutes.  Calls only the oracle and the seeded
input generator.

    python tests/golden/make_digests.py               # every entry (CPU-tens of minutes)
    python tests/golden/make_digests.py streams cfg3  # one group, merged into the file

Entries:
* ``levels``: for (workload, seed) pairs, the int32 CDF rows of every depth
  (level_probs) and the encoded stream at chunk size 2^8;
* ``streams``: the encoded stream (chunk size 2^8) of every frame of every
  workload: the 16-beam, 64-beam and 128-beam scans of their seed lists, the
  32 uneven frames of the batching workload (seeds 3001-3032, 64-beam model),
  and one frame of each of the 24 sensors of the serving fleet (fleet seed
  5000, each sensor with the model of its depth).
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2603_25260_amd import synth  # noqa: E402

LEVEL_JOBS = [("cfg4", 4001), ("cfg2", 2002)]
CHUNK = 8
FLEET_SEED, FLEET_SENSORS, FLEET_FRAMES = 5000, 24, 1
BATCH_SEEDS = tuple(range(3001, 3033))
PATH = os.path.join(HERE, "digests.json")


def sha(b):
    return hashlib.sha256(b).hexdigest()


def frame_of(group, key):
    """(blob arguments (seed, C, D, n_deep), xyz) of one stream entry."""
    if group in ("cfg1", "cfg2", "cfg4"):
        cfg = synth.CONFIGS[group]
        return (cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), synth.make_scan(cfg.scan, int(key))
    if group == "cfg3":
        cfg = synth.CONFIGS["cfg2"]
        s = int(key)
        return (cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep), synth.make_scan(synth.batch_scan_spec(s), s)
    if group == "fleet":
        i, k = (int(v) for v in key.split("_"))
        beams, D = synth.fleet_spec(FLEET_SENSORS, FLEET_SEED)[i]
        C, D, nd = synth.fleet_model(D)
        xyz = synth.make_scan(synth.fleet_scan_spec(beams, D), synth.fleet_frame_seed(FLEET_SEED, i, k))
        return (1, C, D, nd), xyz
    raise KeyError(group)


def stream_keys(group):
    if group in ("cfg1", "cfg2", "cfg4"):
        return [str(s) for s in synth.CONFIGS[group].seeds]
    if group == "cfg3":
        return [str(s) for s in BATCH_SEEDS]
    if group == "fleet":
        return [f"{i}_{k}" for i in range(FLEET_SENSORS) for k in range(FLEET_FRAMES)]
    raise KeyError(group)


def one(task):
    kind, group, key, what = task
    if kind == "streams":
        (ws, C, D, nd), xyz = frame_of(group, key)
        blob = synth.make_weights(ws, C, D, nd)
        bs = O.encode(blob, xyz, CHUNK)
        return task, {"sha256": sha(bs), "bytes": len(bs), "points": int(len(xyz)), "C": C, "D": D}
    cfg = synth.CONFIGS[group]
    blob = synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, int(key))
    if what == "stream":
        bs = O.encode(blob, xyz, CHUNK)
        return task, {"sha256": sha(bs), "bytes": len(bs), "points": int(len(xyz))}
    cdf = O.level_probs(blob, xyz, what)
    return task, {"sha256": sha(cdf.astype("<i4").tobytes()), "rows": int(cdf.shape[0])}


def main(argv):
    O.build()
    out = json.load(open(PATH)) if os.path.exists(PATH) else {}
    tasks = []
    want_kind = argv[0] if argv else None
    want_groups = set(argv[1:])
    if want_kind in (None, "levels"):
        for name, seed in LEVEL_JOBS:
            if want_groups and name not in want_groups:
                continue
            tasks.append(("levels", name, str(seed), "stream"))
            tasks += [("levels", name, str(seed), d) for d in range(synth.CONFIGS[name].scan.D)]
    if want_kind in (None, "streams"):
        for group in ("cfg1", "cfg2", "cfg3", "cfg4", "fleet"):
            if want_groups and group not in want_groups:
                continue
            tasks += [("streams", group, k, None) for k in stream_keys(group)]
    # longest first (deep octrees, wide models), so the pool drains evenly
    def cost(t):
        return 1 if t[0] == "levels" else {"cfg4": 3, "fleet": 2}.get(t[1], 1)
    tasks.sort(key=cost, reverse=True)
    with mp.Pool(int(os.environ.get("DIGEST_WORKERS", min(8, os.cpu_count() or 1)))) as pool:
        for (kind, group, key, what), val in pool.imap_unordered(one, tasks):
            if kind == "levels":
                e = out.setdefault(group, {}).setdefault(key, {"levels": {}})
                if what == "stream":
                    e["stream_c8"] = val
                else:
                    e["levels"][str(what)] = val
            else:
                out.setdefault("streams", {}).setdefault(group, {})[key] = val
            print(kind, group, key, what, flush=True)
            json.dump(out, open(PATH + ".tmp", "w"), indent=1, sort_keys=True)
            os.replace(PATH + ".tmp", PATH)


if __name__ == "__main__":
    main(sys.argv[1:])

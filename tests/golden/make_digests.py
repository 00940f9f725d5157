"""Write tests/golden/digests.json: sha256 digests of CPU-oracle outputs for
full-size synthetic frames, so that GPU tests can check frames whose oracle
run takes minutes.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_digests.py            # all entries (several CPU-minutes)

Entries: for each (workload, seed): the encoded stream (chunk size 2^8) and
the int32 CDF rows of every depth (level_probs), as sha256 of the raw bytes.
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

JOBS = [("cfg4", 4001), ("cfg2", 2002)]
CHUNK = 8


def sha(b):
    return hashlib.sha256(b).hexdigest()


def one(task):
    name, seed, what = task
    cfg = synth.CONFIGS[name]
    blob = synth.make_weights(cfg.weight_seed, cfg.C, cfg.scan.D, cfg.n_deep)
    xyz = synth.make_scan(cfg.scan, seed)
    if what == "stream":
        bs = O.encode(blob, xyz, CHUNK)
        return name, seed, what, {"sha256": sha(bs), "bytes": len(bs), "points": int(len(xyz))}
    cdf = O.level_probs(blob, xyz, what)
    return name, seed, what, {"sha256": sha(cdf.astype("<i4").tobytes()), "rows": int(cdf.shape[0])}


def main():
    O.build()
    tasks = []
    for name, seed in JOBS:
        D = synth.CONFIGS[name].scan.D
        tasks.append((name, seed, "stream"))
        tasks += [(name, seed, d) for d in range(D)]
    out = {}
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        for name, seed, what, val in pool.imap_unordered(one, tasks):
            e = out.setdefault(name, {}).setdefault(str(seed), {"levels": {}})
            if what == "stream":
                e["stream_c8"] = val
            else:
                e["levels"][str(what)] = val
            print(name, seed, what, flush=True)
    json.dump(out, open(os.path.join(HERE, "digests.json"), "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()

"""Writes tests/golden/digests_<workload>.npz: for every directed pair of a
full-size workload, the digest of the oracle's matches (tests/digests.py)
and its match count.  It calls only the oracle (the matcher of Sec. 2.3.1
steps (1)-(4)) and the seeded input generator.  Run from the repository
root, e.g.:

    python tests/golden/make_digests.py strips knn-200x40000 grid-5000x10000

Workloads (the generator's defaults; L = 6, m = 8, K = 8, t_r = 4/5):
  strips            500 images, 2k-20k features, 5,554 pairs
  knn-200x40000     200 images x 40,000 features, 2,000 pairs
  grid-5000x10000   5,000 images x 10,000 features, 101,824 pairs
  grid-1200x10000   12 x 100 grid of 10,000-feature images
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2505_22089_amd import synth  # noqa: E402
from tests.digests import golden_path, match_counts, pair_digests  # noqa: E402

WORKLOADS = {
    "strips": lambda: synth.config3(),
    "knn-200x40000": lambda: synth.config4(),
    "grid-5000x10000": lambda: synth.config5(progress=lambda m: print("  gen", m, flush=True)),
    "grid-1200x10000": lambda: synth.config5(rows=12, cols=100),
}


def log(msg):
    print("[%s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)


def make(name: str, chunk: int = 2048) -> None:
    log("%s: generating" % name)
    wl = WORKLOADS[name]()
    log("%s: %d images, %d pairs; hashing" % (name, len(wl.images), len(wl.pairs)))
    H = O.hash_workload(wl)
    P = len(wl.pairs)
    dig = np.empty(P, np.uint64)
    cnt = np.empty(P, np.int64)
    t0 = time.time()
    for p0 in range(0, P, chunk):
        p1 = min(P, p0 + chunk)
        out, offs, _, _ = O.match_pairs(H, wl.pairs[p0:p1], wl.L, wl.m, wl.K, wl.ratio)
        dig[p0:p1] = pair_digests(out, offs)
        cnt[p0:p1] = match_counts(out, offs)
        log("%s: %d / %d pairs (%.0f pairs/s)" % (name, p1, P, p1 / (time.time() - t0)))
    meta = dict(workload=name, images=str(len(wl.images)), pairs=str(P), L=str(wl.L), m=str(wl.m),
                K=str(wl.K), ratio="%d/%d" % tuple(wl.ratio), matches=str(int(cnt.sum())),
                oracle_threads=str(O.max_threads()))
    np.savez_compressed(golden_path(name), digests=dig, matches=cnt.astype(np.int32),
                        pairs=np.asarray(wl.pairs, np.int32),
                        meta_keys=np.array(list(meta.keys())), meta_vals=np.array(list(meta.values())))
    log("%s: written %s (%d matches)" % (name, golden_path(name), int(cnt.sum())))


if __name__ == "__main__":
    names = sys.argv[1:] or ["strips", "knn-200x40000", "grid-5000x10000"]
    for n in names:
        if n not in WORKLOADS:
            sys.exit("unknown workload %s (one of %s)" % (n, ", ".join(WORKLOADS)))
    for n in names:
        make(n)

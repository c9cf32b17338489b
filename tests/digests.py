"""Per-pair digests of match outputs, so that every pair of a large workload
can be compared with stored expected values without storing the matches.

A pair's digest is the first 8 bytes of BLAKE2b over its int32 outputs
(little-endian, one per query row, db row or -1), read as a little-endian
uint64.  No part of the matching is computed here."""
import hashlib
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def pair_digests(out: np.ndarray, offs: np.ndarray) -> np.ndarray:
    out = np.ascontiguousarray(out, dtype="<i4")
    offs = np.asarray(offs, dtype=np.int64)
    dig = np.empty(len(offs) - 1, dtype=np.uint64)
    mv = memoryview(out).cast("B")
    for p in range(len(offs) - 1):
        h = hashlib.blake2b(mv[4 * int(offs[p]):4 * int(offs[p + 1])], digest_size=8).digest()
        dig[p] = np.frombuffer(h, dtype="<u8")[0]
    return dig


def match_counts(out: np.ndarray, offs: np.ndarray) -> np.ndarray:
    ok = np.concatenate([[0], np.cumsum(np.asarray(out) >= 0)])
    offs = np.asarray(offs, dtype=np.int64)
    return (ok[offs[1:]] - ok[offs[:-1]]).astype(np.int64)


def golden_path(name: str) -> str:
    return os.path.join(GOLDEN, "digests_%s.npz" % name)


def load_golden(name: str):
    """(digests, match counts, pairs, meta dict) stored for a workload."""
    with np.load(golden_path(name), allow_pickle=False) as z:
        meta = dict(zip(z["meta_keys"].tolist(), z["meta_vals"].tolist()))
        return z["digests"], z["matches"], z["pairs"], meta

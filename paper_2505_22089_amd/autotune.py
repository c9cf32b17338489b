"""Autotuner for the batched match launch.

Chooses chm_tuning for a store and a pair list by timing the batched plan on
the device: which match kernel serves which pairs (query major, bucket
major, and the db-image size from which bucket major takes over), the
bucket-major group size, and the query-major launch shape (queries per work
item, work-group size, LDS staging of the db codes, persistent work-groups
per compute unit, tail fraction, item size of launches without LDS staging).

The search is coordinate descent from the library's defaults: each field in
turn takes each of its candidate values with the others fixed, and the
fastest value is kept before the next field is tried.  Any tuning gives
identical results: every timed candidate's output is compared with the
first one's and a mismatch raises.  Winners are cached in a JSON file keyed
by the device name, a hash of the loaded library (a rebuilt kernel never
reuses an old winner) and the workload shape, so later runs skip the search.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import chm

# candidate values per field, in the order the search visits the fields
SEARCH: List[Tuple[str, List[int]]] = [
    ("match_kernel", [chm.KERNEL_QUERY_MAJOR, chm.KERNEL_BUCKET_MAJOR]),
    ("bm_min_db_feats", [0, 6144, 10176, 20000]),
    ("group_queries", [32768, 65536, 98304, 196608]),
    ("queries_per_item", [1024, 2048, 3072, 4096]),
    ("wg_threads", [256, 1024]),
    ("lds_codes", [0, 1]),
    ("grid_per_cu", [1, 2, 4]),
    ("tail_percent", [0, 4, 8, 16]),
    ("hbm_item_queries", [256, 512, 1024]),
]

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "chm_autotune.json")

_LIB_HASH: Optional[str] = None


def library_hash() -> str:
    """sha256 (16 hex digits) of the loaded libchm.so."""
    global _LIB_HASH
    if _LIB_HASH is None:
        chm.lib()
        h = hashlib.sha256()
        with open(chm.LIB_PATH, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _LIB_HASH = h.hexdigest()[:16]
    return _LIB_HASH


def _bucket(v: float) -> int:
    return int(round(np.log2(max(1.0, float(v))) * 2))


def shape_key(store: "chm.Store", pairs: np.ndarray) -> str:
    import torch
    dev = torch.cuda.get_device_name(0)
    nq = np.array([store.feats[int(q)] for q in pairs[:, 0]], dtype=np.float64)
    nd = np.array([store.feats[int(d)] for d in pairs[:, 1]], dtype=np.float64)
    c = store.cfg
    return "%s|lib %s|L%d m%d K%d|P%d|q%d|d%d|dmin%d|dmax%d" % (
        dev, library_hash(), c.num_tables, c.bucket_bits, c.top_k, _bucket(len(pairs)),
        _bucket(nq.mean() if len(nq) else 1), _bucket(nd.mean() if len(nd) else 1),
        _bucket(nd.min() if len(nd) else 1), _bucket(nd.max() if len(nd) else 1))


def _time_plan(store, pairs, offs, out, reps: int) -> float:
    import torch
    plan = chm.Plan(store, pairs, offs, out, None, chm.MATCH_BATCHED)
    try:
        plan.execute()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.execute()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps
    finally:
        plan.close()


def tune(store: "chm.Store", pairs: np.ndarray, reps: int = 5, cache: Optional[str] = DEFAULT_CACHE,
         search: Optional[List[Tuple[str, List[int]]]] = None, verbose: bool = False,
         report: Optional[dict] = None) -> Dict[str, int]:
    """Picks and applies the fastest tuning for this store and pair list;
    returns it (every chm_tuning field).  report, if given, receives the
    default's and the winner's plan times (ms), the number of tunings timed
    and whether the cache answered."""
    import torch
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    key = shape_key(store, pairs)
    table = {}
    if cache and os.path.exists(cache):
        try:
            table = json.load(open(cache))
        except (OSError, ValueError):
            table = {}
    if key in table:
        best = table[key]["tuning"]
        store.set_tuning(**best)
        if report is not None:
            report.update(cached=True, best_ms=table[key]["ms"], default_ms=table[key].get("default_ms"),
                          timed=0)
        return store.tuning_dict()
    offs = chm.out_offsets(store, pairs)
    total = max(1, int(offs[-1]))
    out = torch.empty(total, dtype=torch.int32, device=store.arena.device)
    ref = None
    tried: Dict[str, float] = {}

    def run(t: Dict[str, int]) -> float:
        nonlocal ref
        k = json.dumps(t, sort_keys=True)
        if k in tried:
            return tried[k]
        store.set_tuning(**t)
        out.fill_(-7)
        ms = _time_plan(store, pairs, offs, out, reps) * 1e3
        o = out.cpu().numpy()
        if ref is None:
            ref = o
        elif not np.array_equal(o, ref):
            raise RuntimeError("tuning %s changed the matches" % t)
        tried[k] = ms
        if verbose:
            print("autotune %s: %.3f ms" % (t, ms), flush=True)
        return ms

    best = store.tuning_dict()
    best_ms = default_ms = run(best)
    for field, values in (search or SEARCH):
        for v in values:
            cand = dict(best, **{field: int(v)})
            ms = run(cand)
            if ms < best_ms:
                best, best_ms = cand, ms
    store.set_tuning(**best)
    if report is not None:
        report.update(cached=False, best_ms=best_ms, default_ms=default_ms, timed=len(tried))
    if cache:
        table[key] = {"tuning": best, "ms": best_ms, "default_ms": default_ms,
                      "tried": [{"tuning": json.loads(k), "ms": v} for k, v in sorted(tried.items(), key=lambda x: x[1])]}
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            tmp = cache + ".tmp"
            json.dump(table, open(tmp, "w"), indent=1)
            os.replace(tmp, cache)
        except OSError:
            pass
    return store.tuning_dict()

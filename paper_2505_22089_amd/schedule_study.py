"""Host-to-device traffic of pair schedules under a GPU residency cap.

Counts the descriptor bytes each schedule copies host -> HBM for a view
graph, for three ways of walking the pairs:

* naive: both images of every pair are loaded for that pair and freed
  after it (no residency at all);
* sequential: pairs in list order, images kept resident until the cap
  forces the least recently used one out (a load/free list);
* graph partition: the images, in GPS order, are cut into parts of at most
  half the cap; part A is loaded once for its internal pairs, then every
  part B that shares pairs with A is streamed through the other half (the
  part-pair schedule of graph-partition methods);
* MBR: the block schedule of Sec. 2.2 / Algorithm 1 (GPS order, segments of
  Size_blk images, block rows), computed by the library's scheduler.

Only image sizes and the pair list are needed, so full-size view graphs
(5,000 images, ~10^5 pairs) are studied without generating descriptors.
Run: python -m paper_2505_22089_amd.schedule_study
"""
from __future__ import annotations

import argparse
import json
from collections import OrderedDict
from typing import Dict, List, Sequence

import numpy as np

from . import chm, synth


def naive_bytes(pairs: np.ndarray, desc_bytes: Sequence[int]) -> int:
    return int(sum(desc_bytes[q] + desc_bytes[d] for q, d in pairs))


def sequential_lru(pairs: np.ndarray, slot_bytes: Sequence[int], desc_bytes: Sequence[int],
                   cap: int) -> Dict[str, int]:
    """Pairs in order; a missing image is loaded, evicting least recently
    used images (never the other image of the current pair) until it fits."""
    res: "OrderedDict[int, None]" = OrderedDict()
    used = loaded_bytes = loads = peak = 0
    for q, d in pairs:
        for i in (int(q), int(d)):
            if i in res:
                res.move_to_end(i)
                continue
            while used + slot_bytes[i] > cap:
                victim = next(v for v in res if v not in (int(q), int(d)))
                used -= slot_bytes[victim]
                del res[victim]
            res[i] = None
            used += slot_bytes[i]
            loaded_bytes += desc_bytes[i]
            loads += 1
            peak = max(peak, used)
    return {"h2d_bytes": loaded_bytes, "loads": loads, "resident_peak": peak}


def graph_partition(n: int, pairs: np.ndarray, slot_bytes: Sequence[int], desc_bytes: Sequence[int],
                    cap: int) -> Dict[str, object]:
    """Part-pair schedule over GPS-ordered parts of at most cap / 2 bytes.
    Returns traffic and checks: every pair once, residency within cap."""
    edges = np.unique(np.sort(np.asarray(pairs, dtype=np.int32).reshape(-1, 2), axis=1), axis=0)
    order = chm.gps_order(n, edges, list(range(n)))
    part_of = np.empty(n, np.int64)
    parts: List[List[int]] = [[]]
    used = 0
    for v in order:
        if parts[-1] and used + slot_bytes[v] > cap // 2:
            parts.append([])
            used = 0
        parts[-1].append(int(v))
        part_of[v] = len(parts) - 1
        used += slot_bytes[v]
    by_parts: Dict[tuple, List[int]] = {}
    for p, (q, d) in enumerate(np.asarray(pairs).reshape(-1, 2)):
        a, b = sorted((int(part_of[q]), int(part_of[d])))
        by_parts.setdefault((a, b), []).append(p)
    loaded = loads = peak = 0
    done = np.zeros(len(pairs), np.int64)
    for a in range(len(parts)):
        partners = sorted(b for (x, b) in by_parts if x == a and b != a)
        if (a, a) not in by_parts and not partners:
            continue
        bytes_a = sum(slot_bytes[v] for v in parts[a])
        loaded += sum(desc_bytes[v] for v in parts[a])
        loads += len(parts[a])
        peak = max(peak, bytes_a)
        for p in by_parts.get((a, a), []):
            done[p] += 1
        for b in partners:
            loaded += sum(desc_bytes[v] for v in parts[b])
            loads += len(parts[b])
            peak = max(peak, bytes_a + sum(slot_bytes[v] for v in parts[b]))
            for p in by_parts[(a, b)]:
                done[p] += 1
    return {"h2d_bytes": int(loaded), "loads": int(loads), "parts": len(parts), "resident_peak": int(peak),
            "every_pair_once": bool((done == 1).all())}


def mbr(n: int, pairs: np.ndarray, slot_bytes: Sequence[int], desc_bytes: Sequence[int], cap: int,
        blk: int) -> Dict[str, object]:
    s = chm.schedule_mbr(n, pairs, slot_bytes, cap, blk)
    loads = [i for st in s.steps for i in st["load"]]
    return {"h2d_bytes": int(sum(desc_bytes[i] for i in loads)), "loads": len(loads),
            "steps": len(s.steps), "iterations": s.iterations, "fallback_pairs": s.fallback_pairs,
            "dims": s.dims}


# ---------------------------------------------------------------- step lists
# The same schedules as explicit steps (evict, load, pairs) that the
# library runs on the device (chm.schedule_from_steps + chm.run_schedule).

def naive_steps(pairs: np.ndarray) -> List[dict]:
    """One step per pair: its images loaded for it and freed after it (the
    sequential per-pair strategy, with re-upload)."""
    steps, res = [], []
    for p, (q, d) in enumerate(np.asarray(pairs).reshape(-1, 2)):
        need = sorted({int(q), int(d)})
        steps.append({"evict": res, "load": need, "pairs": [p]})
        res = need
    return steps


def lru_steps(pairs: np.ndarray, slot_bytes: Sequence[int], cap: int) -> List[dict]:
    """Pairs in list order with a load/free list: a pair whose images are
    resident (or fit beside the resident set) joins the current step; one
    that needs room closes it, and the next step first frees the least
    recently used images (never the pair's own) until its images fit."""
    res: "OrderedDict[int, None]" = OrderedDict()
    used = 0
    steps: List[dict] = []
    cur = {"evict": [], "load": [], "pairs": []}
    for p, (q, d) in enumerate(np.asarray(pairs).reshape(-1, 2)):
        q, d = int(q), int(d)
        need = [i for i in dict.fromkeys((q, d)) if i not in res]
        if used + sum(slot_bytes[i] for i in need) > cap:
            if cur["pairs"]:
                steps.append(cur)
            cur = {"evict": [], "load": [], "pairs": []}
            while used + sum(slot_bytes[i] for i in need) > cap:
                victim = next(v for v in res if v not in (q, d))
                used -= slot_bytes[victim]
                del res[victim]
                cur["evict"].append(victim)
        for i in need:
            res[i] = None
            used += slot_bytes[i]
            cur["load"].append(i)
        for i in (q, d):
            res.move_to_end(i)
        cur["pairs"].append(p)
    if cur["pairs"]:
        steps.append(cur)
    return steps


def partition_steps(n: int, pairs: np.ndarray, slot_bytes: Sequence[int], cap: int) -> List[dict]:
    """The part-pair schedule of graph_partition() as steps: part A is
    loaded with its internal pairs, then each partner part B in turn (the
    previous B freed first); A is freed before the next part A."""
    edges = np.unique(np.sort(np.asarray(pairs, dtype=np.int32).reshape(-1, 2), axis=1), axis=0)
    order = chm.gps_order(n, edges, list(range(n)))
    part_of = np.empty(n, np.int64)
    parts: List[List[int]] = [[]]
    used = 0
    for v in order:
        if parts[-1] and used + slot_bytes[v] > cap // 2:
            parts.append([])
            used = 0
        parts[-1].append(int(v))
        part_of[v] = len(parts) - 1
        used += slot_bytes[v]
    by_parts: Dict[tuple, List[int]] = {}
    for p, (q, d) in enumerate(np.asarray(pairs).reshape(-1, 2)):
        a, b = sorted((int(part_of[q]), int(part_of[d])))
        by_parts.setdefault((a, b), []).append(p)
    steps: List[dict] = []
    resident: List[int] = []
    for a in range(len(parts)):
        partners = sorted(b for (x, b) in by_parts if x == a and b != a)
        if (a, a) not in by_parts and not partners:
            continue
        steps.append({"evict": resident, "load": list(parts[a]), "pairs": by_parts.get((a, a), [])})
        resident = list(parts[a])
        prev: List[int] = []
        for b in partners:
            steps.append({"evict": prev, "load": list(parts[b]), "pairs": by_parts[(a, b)]})
            prev = list(parts[b])
        resident = resident + prev
    return steps


def steps_h2d(steps: Sequence[dict], desc_bytes: Sequence[int]) -> int:
    return int(sum(desc_bytes[i] for s in steps for i in s["load"]))


def grid_graph(rows: int = 50, cols: int = 100, seed: int = 1005) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.concatenate([synth.band_grid_pairs(rows, cols, 1, 3), synth.cross_links(rng, rows, cols)])


def study(name: str, n: int, pairs: np.ndarray, feats: np.ndarray, caps_gb: List[float],
          blks: List[int]) -> List[dict]:
    cfg = chm.config()
    slot = [chm.image_bytes(cfg, int(f)) + 256 for f in feats]
    desc = [int(f) * 128 for f in feats]
    floor = int(sum(desc))
    out = []
    for cap_gb in caps_gb:
        cap = int(cap_gb * (1 << 30))
        row = {"workload": name, "cap_GB": cap_gb, "images": n, "pairs": int(len(pairs)),
               "floor_bytes": floor, "naive_bytes": naive_bytes(pairs, desc),
               "sequential": sequential_lru(pairs, slot, desc, cap),
               "graph_partition": graph_partition(n, pairs, slot, desc, cap), "mbr": {}}
        for blk in blks:
            row["mbr"][blk] = mbr(n, pairs, slot, desc, cap, blk)
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--caps", default="16,2")
    ap.add_argument("--blks", default="50,100,200,400,800")
    a = ap.parse_args()
    caps = [float(c) for c in a.caps.split(",")]
    blks = [int(b) for b in a.blks.split(",")]
    rows = []
    pairs = grid_graph()
    rows += study("grid-50x100 x 10000", 5000, pairs, np.full(5000, 10000), caps, blks)
    strips = synth.offset_grid_pairs(25, 20, synth.STRIP_12)
    rng = np.random.default_rng(1003)
    feats = np.round(np.exp(rng.uniform(np.log(2000), np.log(20000), 500))).astype(np.int64)
    rows += study("strips-25x20 x LU(2k-20k)", 500, strips, feats, [c / 8 for c in caps], blks)
    for r in rows:
        print(json.dumps(r))


if __name__ == "__main__":
    main()

"""Plain-Python oracle of the MBR (matrix band reduction) block schedule.

Test infrastructure only.  Follows Sec. 2.2 steps (1)-(5) (initialisation,
permute order, schedule blocks, matrix update, termination), Algorithm 1 of
Sec. 2.4 (load / match / free per block row) and Algorithm 2 of Appendix A
(Gibbs-Poole-Stockmeyer ordering).  Readings where the text is silent:

* GPS runs per connected component of the symmetric view graph (self pairs
  ignored for adjacency); components are numbered consecutively in order of
  their smallest image id.
* Pseudo-peripheral pair: start at the minimum-degree node (ties: smallest
  id); take v = minimum-degree node of the last level of L(u) (ties: smallest
  id); if L(v) is deeper, restart from v, else return (u, v).
* Combined level structure (Gibbs, Poole and Stockmeyer, 1976): node w gets
  (i, j) = (level in L(u), depth - level in L(v)); nodes with i == j are fixed
  at level i; the remaining nodes form connected components, taken largest
  first (ties: smallest id); each whole component goes to its L(u) levels or
  its reversed L(v) levels, whichever gives the smaller maximum width among
  the levels it adds to (ties: the level structure of smaller width, then L(u)).
* Numbering: level 0 sorted by (degree, id); level i > 0 sorted by (smallest
  number of a neighbour in level i-1, degree, id); nodes are numbered level
  by level.
* Size_blk counts images.  Segments are consecutive runs of the permuted
  order holding at most Size_blk images, closed early when the next image
  would take the segment above half the memory cap (so two neighbouring
  segments always fit).  Block row r is the window of segments r, r+1, ...
  as long as their bytes fit in the cap; it processes every remaining pair
  with one end in segment r and the other in the window.  Images are loaded
  when a pair of the row first needs them (only what is not resident) and
  every resident image outside the row's window is freed first.
* An iteration that processes no pair falls back to one pair per step.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple


class CapacityError(ValueError):
    pass


def symmetric_adjacency(n: int, edges: Sequence[Tuple[int, int]]) -> List[List[int]]:
    """M_sym = M or M^T as sorted neighbour lists (Sec. 2.2 step (1))."""
    nb = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            nb[a].add(b)
            nb[b].add(a)
    return [sorted(s) for s in nb]


def level_structure(adj: List[List[int]], root: int) -> List[List[int]]:
    """Breadth-first level structure L(root) of root's component."""
    seen = {root}
    levels = [[root]]
    while True:
        nxt = []
        for w in levels[-1]:
            for x in adj[w]:
                if x not in seen:
                    seen.add(x)
                    nxt.append(x)
        if not nxt:
            return [sorted(l) for l in levels]
        levels.append(nxt)


def pseudo_peripheral_pair(adj, comp: List[int]):
    """Algorithm 2, procedure PseudoPeripheralNodeSelection."""
    u = min(comp, key=lambda w: (len(adj[w]), w))
    Lu = level_structure(adj, u)
    while True:
        v = min(Lu[-1], key=lambda w: (len(adj[w]), w))
        Lv = level_structure(adj, v)
        if len(Lv) > len(Lu):
            u, Lu = v, Lv
            continue
        return u, v, Lu, Lv


def _width(levels: List[List[int]]) -> int:
    return max(len(l) for l in levels)


def combined_levels(adj, Lu, Lv) -> List[List[int]]:
    """Algorithm 2, GpsOrdering: combine L(u) and L(v) into one level structure."""
    k = len(Lu) - 1
    li = {w: i for i, l in enumerate(Lu) for w in l}
    lj = {w: k - i for i, l in enumerate(Lv) for w in l}
    nodes = sorted(li)
    width = [0] * (k + 1)
    level = {}
    for w in nodes:
        if li[w] == lj[w]:
            level[w] = li[w]
            width[li[w]] += 1
    rest = [w for w in nodes if w not in level]
    rest_set = set(rest)
    comps = []
    seen = set()
    for s in rest:
        if s in seen:
            continue
        seen.add(s)
        comp, dq = [], deque([s])
        while dq:
            w = dq.popleft()
            comp.append(w)
            for x in adj[w]:
                if x in rest_set and x not in seen:
                    seen.add(x)
                    dq.append(x)
        comps.append(sorted(comp))
    comps.sort(key=lambda c: (-len(c), c[0]))
    wu, wv = _width(Lu), _width(Lv)
    for comp in comps:
        add_i = [0] * (k + 1)
        add_j = [0] * (k + 1)
        for w in comp:
            add_i[li[w]] += 1
            add_j[lj[w]] += 1
        h0 = max(width[i] + add_i[i] for i in range(k + 1) if add_i[i] > 0)
        l0 = max(width[i] + add_j[i] for i in range(k + 1) if add_j[i] > 0)
        use_u = h0 < l0 or (h0 == l0 and wu <= wv)
        for w in comp:
            lv = li[w] if use_u else lj[w]
            level[w] = lv
            width[lv] += 1
    out = [[] for _ in range(k + 1)]
    for w in nodes:
        out[level[w]].append(w)
    return out


def gps_order(adj: List[List[int]], nodes: Sequence[int]) -> List[int]:
    """Permutation (list of node ids in new order) of the given nodes, component by component."""
    nodes = sorted(nodes)
    node_set = set(nodes)
    sub = {w: [x for x in adj[w] if x in node_set] for w in nodes}
    order: List[int] = []
    seen = set()
    for s in nodes:
        if s in seen:
            continue
        comp = [s]
        seen.add(s)
        dq = deque([s])
        while dq:
            w = dq.popleft()
            for x in sub[w]:
                if x not in seen:
                    seen.add(x)
                    comp.append(x)
                    dq.append(x)
        comp.sort()
        if len(comp) == 1:
            order.append(comp[0])
            continue
        u, v, Lu, Lv = pseudo_peripheral_pair(sub, comp)
        levels = combined_levels(sub, Lu, Lv)
        number: Dict[int, int] = {}
        for i, lev in enumerate(levels):
            if i == 0:
                keyed = sorted(lev, key=lambda w: (len(sub[w]), w))
            else:
                prev = set(levels[i - 1])
                inf = len(nodes) + len(order) + 1

                def key(w):
                    ns = [number[x] for x in sub[w] if x in prev]
                    return (min(ns) if ns else inf, len(sub[w]), w)
                keyed = sorted(lev, key=key)
            for w in keyed:
                number[w] = len(order)
                order.append(w)
    return order


def bandwidth(order: Sequence[int], edges: Sequence[Tuple[int, int]]) -> int:
    pos = {w: i for i, w in enumerate(order)}
    bw = 0
    for a, b in edges:
        if a in pos and b in pos:
            bw = max(bw, abs(pos[a] - pos[b]))
    return bw


@dataclass
class Step:
    evict: List[int] = field(default_factory=list)
    load: List[int] = field(default_factory=list)
    pairs: List[int] = field(default_factory=list)


@dataclass
class Schedule:
    steps: List[Step]
    dims: List[int]            # MBR matrix dimension at the start of each iteration
    bandwidths: List[int]      # bandwidth of the permuted matrix per iteration
    iterations: int
    fallback_pairs: int        # pairs handled one per step after a stalled iteration


def schedule_mbr(n_images: int, pairs: Sequence[Tuple[int, int]], image_bytes: Sequence[int],
                 cap_bytes: int, blk_images: int) -> Schedule:
    """Sec. 2.2 steps (1)-(5) with the block-row pipeline of Sec. 2.3.2."""
    pairs = [(int(a), int(b)) for a, b in pairs]
    if blk_images < 1:
        raise ValueError("blk_images must be >= 1")
    for a, b in pairs:
        if not (0 <= a < n_images and 0 <= b < n_images):
            raise ValueError("pair references an image out of range")
        if image_bytes[a] + (image_bytes[b] if b != a else 0) > cap_bytes:
            raise CapacityError("a pair does not fit in the memory cap")
    # undirected cells of M_sym and the directed pairs behind each
    cell_pairs: Dict[Tuple[int, int], List[int]] = {}
    for p, (a, b) in enumerate(pairs):
        cell_pairs.setdefault((min(a, b), max(a, b)), []).append(p)
    remaining = set(cell_pairs)
    resident: List[int] = []
    steps: List[Step] = []
    dims, bws = [], []
    iterations = 0
    fallback = 0
    half = cap_bytes / 2.0

    while remaining:
        iterations += 1
        active = sorted({w for c in remaining for w in c})
        dims.append(len(active))
        edges = sorted(remaining)
        adj = symmetric_adjacency(n_images, edges)
        order = gps_order(adj, active)
        bws.append(bandwidth(order, edges))
        pos = {w: i for i, w in enumerate(order)}
        # segments of the permuted order
        seg_of = {}
        seg_bounds: List[Tuple[int, int]] = []
        start, nbytes = 0, 0
        for i, w in enumerate(order):
            if i > start and (i - start == blk_images or nbytes + image_bytes[w] > half):
                seg_bounds.append((start, i))
                start, nbytes = i, 0
            nbytes += image_bytes[w]
        seg_bounds.append((start, len(order)))
        seg_bytes = [sum(image_bytes[order[i]] for i in range(s, e)) for s, e in seg_bounds]
        for si, (s, e) in enumerate(seg_bounds):
            for i in range(s, e):
                seg_of[order[i]] = si
        # cells grouped by the segment of their lower-positioned end
        by_seg: Dict[int, List[Tuple[int, int]]] = {}
        for c in edges:
            lo = min(pos[c[0]], pos[c[1]])
            by_seg.setdefault(seg_of[order[lo]], []).append(c)
        processed = 0
        for r in range(len(seg_bounds)):
            e, tot = r, seg_bytes[r]
            while e + 1 < len(seg_bounds) and tot + seg_bytes[e + 1] <= cap_bytes:
                e += 1
                tot += seg_bytes[e]
            win_lo, win_hi = seg_bounds[r][0], seg_bounds[e][1]
            cells = [c for c in by_seg.get(r, [])
                     if win_lo <= pos[c[0]] < win_hi and win_lo <= pos[c[1]] < win_hi]
            if not cells:
                continue
            step = Step()
            keep = [w for w in resident if w in pos and win_lo <= pos[w] < win_hi]
            keep_set = set(keep)
            step.evict = sorted(w for w in resident if w not in keep_set)
            resident = keep
            need = sorted({w for c in cells for w in c})
            step.load = [w for w in need if w not in keep_set]
            resident = resident + step.load
            step.pairs = sorted(p for c in cells for p in cell_pairs[c])
            steps.append(step)
            for c in cells:
                remaining.discard(c)
            processed += len(cells)
        if processed == 0:
            # stalled: one pair per step for whatever remains
            for c in sorted(remaining):
                step = Step()
                need = sorted(set(c))
                step.evict = sorted(w for w in resident if w not in need)
                resident = [w for w in resident if w in need]
                step.load = [w for w in need if w not in set(resident)]
                resident = resident + step.load
                step.pairs = sorted(cell_pairs[c])
                steps.append(step)
                fallback += len(step.pairs)
            remaining.clear()
    return Schedule(steps=steps, dims=dims, bandwidths=bws, iterations=iterations,
                    fallback_pairs=fallback)

"""Pins of the MBR schedule oracle (Sec. 2.2, Algorithm 1, Appendix A).

* every pair is processed exactly once and only while both images are resident;
* residency never exceeds the cap and loads never repeat a resident image;
* the matrix dimension never grows and every iteration makes progress, so the
  matrix empties (the paper reports the dimension shrinking for dataset 1);
* level-by-level numbering obeys bandwidth <= 2w - 1 (w = widest level);
* GPS beats a random relabelling, gives bandwidth 1 on a path, and at most
  one above the optimum min(R, C) on an R x C grid.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import reverse_cuthill_mckee

from oracle import mbr
from paper_2505_22089_amd import synth


def check_schedule(n, pairs, sizes, cap, sched):
    resident = set()
    seen = []
    for st in sched.steps:
        for w in st.evict:
            assert w in resident
            resident.discard(w)
        for w in st.load:
            assert w not in resident
            resident.add(w)
        assert sum(sizes[w] for w in resident) <= cap
        for p in st.pairs:
            a, b = pairs[p]
            assert a in resident and b in resident
        seen.extend(st.pairs)
    assert sorted(seen) == list(range(len(pairs)))
    used = {int(w) for pr in pairs for w in pr}
    assert sum(len(st.load) for st in sched.steps) >= len(used)
    assert all(x >= y for x, y in zip(sched.dims, sched.dims[1:]))
    cells = {(min(a, b), max(a, b)) for a, b in pairs}
    assert sched.iterations <= max(1, len(cells))


def random_graph(rng, n, p_edge):
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p_edge]
    return np.array(pairs, dtype=np.int32).reshape(-1, 2)


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_every_pair_once_within_cap(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    pairs = random_graph(rng, n, float(rng.uniform(0.02, 0.3)))
    sizes = rng.integers(1, 10, size=n).tolist()
    cap = max(sizes) * 2 + int(rng.integers(0, 30))
    blk = int(rng.integers(1, 8))
    sched = mbr.schedule_mbr(n, pairs, sizes, cap, blk)
    check_schedule(n, pairs, sizes, cap, sched)


def test_band_grid_single_iteration_loads_each_image_once():
    rng = np.random.default_rng(1)
    pairs = np.concatenate([synth.band_grid_pairs(10, 30, 1, 3), synth.cross_links(rng, 10, 30)])
    sizes = [10] * 300
    sched = mbr.schedule_mbr(300, pairs, sizes, 10 * 200, 40)
    check_schedule(300, pairs, sizes, 2000, sched)
    assert sched.iterations == 1
    assert sum(len(s.load) for s in sched.steps) == 300


def test_tight_cap_needs_several_iterations():
    rng = np.random.default_rng(2)
    pairs = random_graph(rng, 80, 0.05)
    sizes = [1] * 80
    sched = mbr.schedule_mbr(80, pairs, sizes, 6, 3)
    check_schedule(80, pairs, sizes, 6, sched)
    assert sched.iterations > 1 and sched.dims[-1] < sched.dims[0]


def level_numbering_bound(adj, comp):
    u, v, Lu, Lv = mbr.pseudo_peripheral_pair(adj, comp)
    levels = mbr.combined_levels(adj, Lu, Lv)
    # every edge joins equal or adjacent levels (a valid level structure)
    lv = {w: i for i, l in enumerate(levels) for w in l}
    for w in comp:
        for x in adj[w]:
            assert abs(lv[w] - lv[x]) <= 1
    return max(len(l) for l in levels)


@pytest.mark.parametrize("seed", range(5))
def test_gps_bandwidth_within_level_bound(seed):
    rng = np.random.default_rng(100 + seed)
    n = 70
    pairs = random_graph(rng, n, 0.06)
    edges = sorted({(min(a, b), max(a, b)) for a, b in pairs})
    adj = mbr.symmetric_adjacency(n, edges)
    order = mbr.gps_order(adj, range(n))
    assert sorted(order) == list(range(n))
    # per component: bandwidth <= 2w - 1
    pos = {w: i for i, w in enumerate(order)}
    seen = set()
    for s in range(n):
        if s in seen or not adj[s]:
            seen.add(s)
            continue
        comp = sorted(mbr.level_structure(adj, s)[0] + [x for l in mbr.level_structure(adj, s)[1:] for x in l])
        seen.update(comp)
        w = level_numbering_bound(adj, comp)
        bw = max(abs(pos[a] - pos[b]) for a in comp for b in adj[a])
        assert bw <= 2 * w - 1
        assert sorted(pos[x] for x in comp) == list(range(min(pos[x] for x in comp),
                                                           min(pos[x] for x in comp) + len(comp)))


def test_gps_path_and_grid_and_random_relabelling():
    n = 30
    path = [(i, i + 1) for i in range(n - 1)]
    perm = np.random.default_rng(0).permutation(n)
    edges = [(int(perm[a]), int(perm[b])) for a, b in path]
    adj = mbr.symmetric_adjacency(n, edges)
    assert mbr.bandwidth(mbr.gps_order(adj, range(n)), edges) == 1
    R, C = 7, 12
    grid = [(r * C + c, r * C + c + 1) for r in range(R) for c in range(C - 1)] + \
           [(r * C + c, (r + 1) * C + c) for r in range(R - 1) for c in range(C)]
    adj = mbr.symmetric_adjacency(R * C, grid)
    gbw = mbr.bandwidth(mbr.gps_order(adj, range(R * C)), grid)
    # the grid's optimum is min(R, C); corner-rooted diagonal levels of width
    # min(R, C) numbered in a consistent order cost at most one more
    assert min(R, C) <= gbw <= min(R, C) + 1
    rng = np.random.default_rng(1)
    for _ in range(5):
        p = rng.permutation(R * C)
        assert gbw <= mbr.bandwidth(list(p), grid)
    # reported beside SciPy's reverse Cuthill-McKee (not asserted beyond sanity)
    rows = [a for a, b in grid] + [b for a, b in grid]
    cols = [b for a, b in grid] + [a for a, b in grid]
    A = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(R * C, R * C))
    rcm = reverse_cuthill_mckee(A, symmetric_mode=True)
    assert gbw <= mbr.bandwidth(list(rcm), grid) + min(R, C)


def test_disconnected_components_are_consecutive():
    edges = [(5, 9), (9, 7), (0, 3), (3, 2), (11, 12)]
    adj = mbr.symmetric_adjacency(13, edges)
    order = mbr.gps_order(adj, [0, 2, 3, 5, 7, 9, 11, 12, 4])
    assert set(order[:3]) == {0, 2, 3}
    assert order[3] == 4
    assert set(order[4:7]) == {5, 7, 9}
    assert set(order[7:]) == {11, 12}


def test_self_pairs_and_directed_duplicates():
    pairs = np.array([[0, 0], [0, 1], [1, 0], [2, 1], [3, 3]], dtype=np.int32)
    sizes = [1, 1, 1, 1]
    sched = mbr.schedule_mbr(4, pairs, sizes, 2, 1)
    check_schedule(4, pairs, sizes, 2, sched)
    step_of = {p: k for k, st in enumerate(sched.steps) for p in st.pairs}
    assert step_of[1] == step_of[2]     # both directions of one cell go together


def test_empty_and_capacity_errors():
    s = mbr.schedule_mbr(3, np.zeros((0, 2), np.int32), [1, 1, 1], 2, 1)
    assert s.steps == [] and s.dims == []
    with pytest.raises(mbr.CapacityError):
        mbr.schedule_mbr(2, [(0, 1)], [3, 3], 5, 1)
    with pytest.raises(ValueError):
        mbr.schedule_mbr(2, [(0, 2)], [1, 1], 5, 1)

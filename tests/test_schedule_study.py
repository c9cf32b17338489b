"""Host-only schedule study: traffic counts of the three pair schedules."""
import numpy as np

from paper_2505_22089_amd import schedule_study as S
from paper_2505_22089_amd import synth


def test_naive_counts_both_images_per_pair():
    pairs = np.array([[0, 1], [1, 2], [0, 2]], np.int32)
    assert S.naive_bytes(pairs, [10, 20, 30]) == 30 + 50 + 40


def test_sequential_lru_loads_each_image_once_when_everything_fits():
    pairs = np.array([[0, 1], [1, 2], [2, 0], [0, 1]], np.int32)
    r = S.sequential_lru(pairs, [1, 1, 1], [5, 6, 7], cap=3)
    assert r == {"h2d_bytes": 18, "loads": 3, "resident_peak": 3}


def test_sequential_lru_evicts_least_recently_used_not_the_partner():
    # cap of two images: pair (0,2) must evict 1 (least recent other than 0)
    pairs = np.array([[0, 1], [0, 2], [1, 2]], np.int32)
    r = S.sequential_lru(pairs, [1, 1, 1], [1, 1, 1], cap=2)
    # loads: 0, 1, then 2 (evicts 1), then 1 (evicts 0)
    assert r["loads"] == 4 and r["resident_peak"] == 2


def test_mbr_reaches_the_floor_on_a_path_with_room():
    n = 40
    pairs = np.array([[i, i + 1] for i in range(n - 1)], np.int32)
    slot = [100] * n
    desc = [64] * n
    r = S.mbr(n, pairs, slot, desc, cap=20 * 100, blk=4)
    assert r["h2d_bytes"] == n * 64 and r["loads"] == n and r["fallback_pairs"] == 0


def test_mbr_never_beats_the_floor_and_never_exceeds_naive_on_a_grid():
    rng = np.random.default_rng(0)
    pairs = np.concatenate([synth.band_grid_pairs(6, 12, 1, 3), synth.cross_links(rng, 6, 12)])
    n = 72
    slot = [10] * n
    desc = [8] * n
    for cap in (200, 120, 60):
        r = S.mbr(n, pairs, slot, desc, cap=cap, blk=4)
        assert n * 8 <= r["h2d_bytes"] <= S.naive_bytes(pairs, desc)


def test_quality_scoring_counts_planted_tracks():
    from paper_2505_22089_amd import quality_study as Q

    class W:
        tracks = [np.array([5, 6, -1, 7]), np.array([6, 9, 5])]
    pairs = np.array([[0, 1]], np.int32)
    offs = np.array([0, 4], np.int64)
    # query 0 (track 5) -> db 2 (track 5): right; query 1 (track 6) -> db 1 (track 9): wrong;
    # query 2 (no track) -> db 0: wrong; query 3 (track 7, absent from db) -> none
    out = np.array([2, 1, 0, -1], np.int32)
    r = Q._score(W, pairs, offs, out)
    assert r == {"matches": 3, "precision": 1 / 3, "recall": 1 / 2}
    keep = [np.array([True, False, False, True])]
    r = Q._score(W, pairs, offs, out, keep)
    assert r == {"matches": 1, "precision": 1.0, "recall": 1 / 2}


def test_graph_partition_covers_every_pair_once_within_the_cap():
    rng = np.random.default_rng(1)
    pairs = np.concatenate([synth.band_grid_pairs(6, 12, 1, 3), synth.cross_links(rng, 6, 12)])
    n = 72
    slot = [10] * n
    desc = [8] * n
    for cap in (200, 120, 60):
        r = S.graph_partition(n, pairs, slot, desc, cap)
        assert r["every_pair_once"] and r["resident_peak"] <= cap
        assert n * 8 <= r["h2d_bytes"] <= S.naive_bytes(pairs, desc)
    # everything fits in one part: each image is loaded once
    r = S.graph_partition(n, pairs, slot, desc, 2 * n * 10)
    assert r["parts"] == 1 and r["h2d_bytes"] == n * 8


def _grid(rows=6, cols=12):
    rng = np.random.default_rng(0)
    return np.concatenate([synth.band_grid_pairs(rows, cols, 1, 3), synth.cross_links(rng, rows, cols)])


def test_step_lists_are_valid_library_schedules_with_the_counted_traffic():
    """The step lists of the per-pair, load/free-list and graph-partition
    schedules pass the library's residency replay (every pair once, images
    resident, cap kept) and copy exactly the bytes the counters report."""
    from paper_2505_22089_amd import chm
    pairs = _grid()
    n = 72
    rng = np.random.default_rng(3)
    slot = [int(v) for v in rng.integers(8, 14, n)]
    desc = [s * 7 for s in slot]
    for cap in (60, 150, 10 ** 6):
        lru = S.lru_steps(pairs, slot, cap)
        assert S.steps_h2d(lru, desc) == S.sequential_lru(pairs, slot, desc, cap)["h2d_bytes"]
        part = S.partition_steps(n, pairs, slot, cap)
        assert S.steps_h2d(part, desc) == S.graph_partition(n, pairs, slot, desc, cap)["h2d_bytes"]
        for steps in (lru, part, S.naive_steps(pairs)):
            sch = chm.schedule_from_steps(n, pairs, slot, cap, steps)
            chm.schedule_free(sch)
    assert S.steps_h2d(S.naive_steps(pairs), desc) == S.naive_bytes(pairs, desc)


def test_schedule_from_steps_rejects_broken_residency():
    from paper_2505_22089_amd import chm
    pairs = np.array([[0, 1], [1, 2]], np.int32)
    slot = [10, 10, 10]
    ok = [{"evict": [], "load": [0, 1], "pairs": [0]}, {"evict": [0], "load": [2], "pairs": [1]}]
    chm.schedule_free(chm.schedule_from_steps(3, pairs, slot, 20, ok))
    bad = [
        [{"evict": [], "load": [0, 1, 2], "pairs": [0, 1]}],                                  # above the cap
        [{"evict": [], "load": [0, 1], "pairs": [0, 1]}],                                     # image 2 absent
        [{"evict": [], "load": [0, 1], "pairs": [0]}, {"evict": [2], "load": [], "pairs": [1]}],  # evicts absent
        [{"evict": [], "load": [0, 1], "pairs": [0]}, {"evict": [], "load": [1], "pairs": [1]}],  # reloads 1
        [{"evict": [], "load": [0, 1], "pairs": [0, 0]}],                                     # pair twice
        [{"evict": [], "load": [0, 1], "pairs": [0]}],                                        # pair 1 missing
    ]
    for steps in bad:
        try:
            chm.schedule_from_steps(3, pairs, slot, 20, steps)
        except chm.ChmError as e:
            assert e.status == -1
        else:
            raise AssertionError("accepted %s" % steps)

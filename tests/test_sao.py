"""SAO local constraint (Sec. 2.3.3): pins of the oracle, then the library's
host implementation against the oracle, bit for bit.

The pins do not retype the oracle: the edit distance is checked on textbook
values, the cyclic distance on its defining invariances and on brute force
over both rotations, the angular order against atan2, the neighbour search
against SciPy's k-d tree, and whole scores on exact similarity transforms
(which keep every neighbourhood's cyclic order) and on a mirror image (which
reverses it).
"""
import ctypes as C

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import sao as S
from paper_2505_22089_amd import chm, synth


# ------------------------------------------------------------------ oracle pins

@pytest.mark.parametrize("a,b,d", [("kitten", "sitting", 3), ("flaw", "lawn", 2), ("", "abc", 3),
                                   ("abc", "abc", 0), ("intention", "execution", 5)])
def test_levenshtein_textbook_values(a, b, d):
    assert S.levenshtein(list(a), list(b)) == d
    assert S.levenshtein(list(b), list(a)) == d


def test_cyclic_edit_distance_invariances():
    rng = np.random.default_rng(0)
    for _ in range(300):
        n = int(rng.integers(1, 8))
        a = [int(v) for v in rng.integers(0, 5, n)]
        b = [int(v) for v in rng.integers(0, 5, n)]
        k = int(rng.integers(0, n))
        c = S.cyclic_edit_distance(a, b)
        assert S.cyclic_edit_distance(a, a[k:] + a[:k]) == 0
        assert c == S.cyclic_edit_distance(b, a)                      # symmetric
        assert c == S.cyclic_edit_distance(a[k:] + a[:k], b)          # rotation-invariant
        assert c <= S.levenshtein(a, b) and c <= n
        # rotating one sequence suffices (the library relies on it)
        assert c == min(S.levenshtein(a, b[j:] + b[:j]) for j in range(n))


def test_angular_order_is_atan2_order():
    rng = np.random.default_rng(1)
    for _ in range(200):
        pts = rng.integers(-1000, 1000, size=(12, 2))
        ang = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * np.pi)
        s = np.sort(ang)
        if (pts == 0).all(axis=1).any() or np.min(np.diff(s)) < 1e-9:
            continue
        order = S.angular_order((0, 0), [tuple(p) for p in pts], list(range(12)))
        assert order == list(np.argsort(ang, kind="stable"))


def test_nearest_matches_kdtree():
    rng = np.random.default_rng(2)
    pts = rng.integers(0, 100000, size=(400, 2))
    labels = np.arange(400)
    tree = cKDTree(pts.astype(np.float64))
    for a in range(0, 400, 37):
        dist, idx = tree.query(pts[a].astype(np.float64), k=7)
        assert len(set(np.round(dist[1:] ** 2).astype(np.int64))) == 6  # no ties here
        assert S.nearest(pts[a], pts, labels, a, 6) == list(idx[1:])


def _identity_matches(n):
    return np.arange(n, dtype=np.int32)


def _similar(pts, quarter_turns, scale, shift):
    x, y = pts[:, 0].astype(np.int64), pts[:, 1].astype(np.int64)
    for _ in range(quarter_turns):
        x, y = -y, x
    return np.stack([scale * x + shift[0], scale * y + shift[1]], axis=1)


def test_similarity_scores_zero_and_mirror_does_not():
    rng = np.random.default_rng(3)
    P = rng.integers(0, 50000, size=(150, 2))
    for turns, scale in ((0, 1), (1, 2), (2, 3), (3, 1)):
        Q = _similar(P, turns, scale, (777, -4242))
        ced, out = S.sao_pair(P, Q, _identity_matches(150), 6)
        assert (ced == 0).all() and (out == np.arange(150)).all()
    M = P.copy()
    M[:, 0] = -M[:, 0]  # mirror: every angular order reverses
    ced, _ = S.sao_pair(P, M, _identity_matches(150), 6)
    assert np.mean(ced > 0) > 0.9


def test_small_match_counts():
    P = np.array([[0, 0], [10, 0], [0, 10]], np.int64)
    ced, out = S.sao_pair(P, P, np.array([-1, -1, -1]), 6)
    assert (ced == -1).all() and (out == -1).all()
    ced, out = S.sao_pair(P, P, np.array([-1, 2, -1]), 6)  # one match: N = 0, kept
    assert list(ced) == [-1, 0, -1] and list(out) == [-1, 2, -1]


# ------------------------------------------------------------------ library vs oracle

def _pair_case(seed, n_q=300, n_d=280, frac=0.6, outliers=0.25, dup=0.05, spread=30000):
    rng = np.random.default_rng(seed)
    kq = rng.integers(0, spread, size=(n_q, 2)).astype(np.int32)
    kd = rng.integers(-spread, spread, size=(n_d, 2)).astype(np.int32)
    match = np.where(rng.random(n_q) < frac, rng.integers(0, n_d, n_q), -1).astype(np.int32)
    # geometrically consistent part: db keypoint = quarter turn of the query keypoint
    good = (match >= 0) & (rng.random(n_q) >= outliers)
    kd[match[good]] = _similar(kq[good], 1, 1, (5, 7)).astype(np.int32)
    # some queries share a db row (several matches on one db keypoint)
    d = (match >= 0) & (rng.random(n_q) < dup)
    if d.any() and (match >= 0).any():
        match[d] = match[match >= 0][0]
    return kq, kd, match


@pytest.mark.parametrize("nn,th", [(6, (1, 2)), (1, (0, 1)), (8, (1, 3)), (12, (2, 3))])
def test_library_matches_oracle(nn, th):
    cases = [_pair_case(s) for s in range(4)]
    cases.append(_pair_case(9, n_q=40, frac=0.05))            # a handful of matches
    cases.append(_pair_case(10, n_q=50, frac=0.0))            # none
    kps, pairs, parts = [], [], []
    for kq, kd, m in cases:
        pairs.append((len(kps), len(kps) + 1))
        kps += [kq, kd]
        parts.append(m)
    offs = np.concatenate([[0], np.cumsum([len(m) for m in parts])]).astype(np.int64)
    allm = np.concatenate(parts)
    out, ced = chm.sao_filter(kps, np.array(pairs), offs, allm, nn, th, n_threads=3, want_ced=True)
    for p, (kq, kd, m) in enumerate(cases):
        rc, rf = S.sao_pair(kq, kd, m, nn, th)
        assert np.array_equal(ced[offs[p]:offs[p + 1]], rc), p
        assert np.array_equal(out[offs[p]:offs[p + 1]], rf), p


def test_library_neighbour_count_limits():
    # N = min(n_neighbors, M - 1): a pair with 20 matches and n_neighbors 32
    kq, kd, m = _pair_case(13, n_q=60, frac=0.34)
    assert 10 < int((m >= 0).sum()) < 33
    out, ced = chm.sao_filter([kq, kd], np.array([[0, 1]]), np.array([0, len(m)], np.int64), m, 32,
                              (1, 2), want_ced=True)
    rc, rf = S.sao_pair(kq, kd, m, 32, (1, 2))
    assert np.array_equal(ced, rc) and np.array_equal(out, rf)
    # the full 32 neighbours: zero on similarity transforms, positive on a mirror
    rng = np.random.default_rng(14)
    P = rng.integers(0, 1 << 20, size=(400, 2)).astype(np.int32)
    pairs, offs, ident = np.array([[0, 1], [0, 2]]), np.array([0, 400, 800], np.int64), np.arange(400)
    Q = _similar(P, 3, 2, (-99, 12345)).astype(np.int32)
    Mi = P.copy()
    Mi[:, 1] = -Mi[:, 1]
    out, ced = chm.sao_filter([P, Q, Mi], pairs, offs, np.concatenate([ident, ident]), 32, (1, 2),
                              want_ced=True)
    assert (ced[:400] == 0).all() and np.array_equal(out[:400], ident)
    assert np.mean(ced[400:] > 0) > 0.9


def test_library_on_synthetic_workload_with_repeated_texture():
    wl = synth.config2(n_images=5, n_feats=600, k=2, repeat_frac=0.3)
    kps = synth.keypoints(wl)
    rng = np.random.default_rng(4)
    parts = []
    for q, d in wl.pairs:  # planted-track matches plus a tenth at random rows
        tq, td = wl.tracks[q], wl.tracks[d]
        pos = {int(t): i for i, t in enumerate(td) if t >= 0}
        m = np.array([pos.get(int(t), -1) for t in tq], np.int32)
        r = rng.random(len(m)) < 0.1
        m[r] = rng.integers(0, len(td), int(r.sum()))
        parts.append(m)
    offs = np.concatenate([[0], np.cumsum([len(m) for m in parts])]).astype(np.int64)
    out, ced = chm.sao_filter(kps, wl.pairs, offs, np.concatenate(parts), 6, (1, 2), want_ced=True)
    for p in (0, len(wl.pairs) - 1):
        q, d = wl.pairs[p]
        rc, rf = S.sao_pair(kps[q], kps[d], parts[p], 6, (1, 2))
        assert np.array_equal(ced[offs[p]:offs[p + 1]], rc)
        assert np.array_equal(out[offs[p]:offs[p + 1]], rf)


def test_library_filters_in_place():
    kq, kd, m = _pair_case(11)
    kps = [kq, kd]
    ptrs = (C.c_void_p * 2)(*[k.ctypes.data for k in kps])
    nf = np.array([len(kq), len(kd)], np.int32)
    pairs = np.array([[0, 1]], np.int32)
    offs = np.array([0, len(m)], np.int64)
    buf = m.copy()
    st = chm.lib().chm_sao_filter(1, pairs.ctypes.data, C.cast(ptrs, C.c_void_p), nf.ctypes.data, 2,
                                  offs.ctypes.data, buf.ctypes.data, 6, 1, 2, 1, buf.ctypes.data, None)
    assert st == 0
    assert np.array_equal(buf, S.sao_pair(kq, kd, m, 6, (1, 2))[1])


def test_library_rejects_bad_input():
    kq, kd, m = _pair_case(12)
    offs = np.array([0, len(m)], np.int64)
    pairs = np.array([[0, 1]])
    bad = m.copy()
    bad[np.argmax(bad >= 0)] = len(kd)
    with pytest.raises(chm.ChmError, match="db row"):
        chm.sao_filter([kq, kd], pairs, offs, bad)
    far = kq.copy()
    far[np.argmax(m >= 0), 0] = 1 << 30
    with pytest.raises(chm.ChmError, match="coordinate"):
        chm.sao_filter([far, kd], pairs, offs, m)
    for nn in (0, 33):
        with pytest.raises(chm.ChmError, match="n_neighbors"):
            chm.sao_filter([kq, kd], pairs, offs, m, n_neighbors=nn)
    with pytest.raises(chm.ChmError, match="offsets"):
        chm.sao_filter([kq, kd], pairs, np.array([0, len(m) - 1], np.int64), m[:-1])
    with pytest.raises(chm.ChmError, match="image"):
        chm.sao_filter([kq, kd], np.array([[0, 2]]), offs, m)


def test_device_entry_rejects_bad_arguments_before_any_gpu_call():
    """Argument checks of chm_sao_filter_device run on the host and return
    before anything is enqueued (no device is needed to see them)."""
    L = chm.lib()
    pairs = np.array([[0, 1]], np.int32)
    nf = np.array([10, 10], np.int32)
    offs = np.array([0, 10], np.int64)
    fake = (C.c_void_p * 2)(256, 512)  # never dereferenced on these paths
    kp = C.cast(fake, C.c_void_p)

    def call(nn=6, num=1, den=2, match=4096, out=8192, work=1 << 20, work_bytes=1 << 30, offsets=offs):
        return L.chm_sao_filter_device(1, pairs.ctypes.data, kp, nf.ctypes.data, 2, offsets.ctypes.data,
                                       match, nn, num, den, out, None, work, work_bytes, None)
    assert call(nn=9) == -1
    assert call(den=0) == -1
    assert call(out=4096) == -1                        # output aliases the matches
    assert call(work=(1 << 20) + 16) == -1             # misaligned work buffer
    assert call(offsets=np.array([0, 9], np.int64)) == -1
    need = chm.sao_work_bytes(1, 10)
    assert call(work_bytes=need - 1) == -3             # CHM_E_CAPACITY
    assert chm.sao_work_bytes(400, 8000) < (1 << 30)


def _golden(name):
    import os
    lines = [l for l in open(os.path.join(os.path.dirname(__file__), "golden", name)) if not l.startswith("#")]
    return [np.array([int(v) for v in l.split()]) for l in lines]


def test_stored_sao_values_still_hold_for_oracle_and_library():
    from tests.golden import make_golden as G
    kq, kd, match = G.sao_case()
    ced, filt = _golden("sao_60.txt")
    rc, rf = S.sao_pair(kq, kd, match, 6, (1, 2))
    assert np.array_equal(rc, ced) and np.array_equal(rf, filt)
    out, lc = chm.sao_filter([kq, kd], np.array([[0, 1]]), np.array([0, 60], np.int64), match, 6, (1, 2),
                             want_ced=True)
    assert np.array_equal(lc, ced) and np.array_equal(out, filt)
    # the random matches are all rejected, most of the transformed ones kept
    assert (filt[45:] == -1).all() and (filt[:45] >= 0).mean() > 0.7

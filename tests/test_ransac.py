"""RANSAC global verification (Sec. 2.3.3): pins of the oracle, then the
library's host implementation against it, match for match.

Pins: a hypothesis through two matches of an exact similarity makes every
match of that similarity an inlier at threshold 0 (and only those); the
residual test equals the floating-point distance away from the threshold
boundary; the hypothesis index rule picks two distinct matches; a planted
similarity with outliers is recovered.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import ransac as R
from paper_2505_22089_amd import chm, synth


def _similarity(P, z, t):
    """q = z p + t with z = a + ib integer, exact in integers."""
    a, b = z
    x, y = P[:, 0].astype(np.int64), P[:, 1].astype(np.int64)
    return np.stack([a * x - b * y + t[0], b * x + a * y + t[1]], axis=1)


def test_exact_similarity_is_all_inliers_at_zero_threshold():
    rng = np.random.default_rng(0)
    P = rng.integers(-5000, 5000, size=(60, 2))
    Q = _similarity(P, (3, -2), (700, -11))
    Q[50:] += rng.integers(1, 40, size=(10, 2))   # the last ten are off the model
    for i, j in ((0, 1), (5, 49), (49, 0)):
        mask = R.inliers_of(P, Q, i, j, 0)
        assert mask[:50].all() and not mask[50:].any()
    assert R.inliers_of(P, Q, 3, 3, 0) is None      # p_i = p_j: no model


def test_residual_test_matches_float_distance():
    rng = np.random.default_rng(1)
    P = rng.integers(-3000, 3000, size=(200, 2))
    Q = rng.integers(-3000, 3000, size=(200, 2))
    for _ in range(20):
        i, j = rng.choice(200, 2, replace=False)
        thr = int(rng.integers(1, 4000))
        mask = R.inliers_of(P, Q, i, j, thr)
        p, q = P.astype(float), Q.astype(float)
        dp, dq = complex(*(p[j] - p[i])), complex(*(q[j] - q[i]))
        z = dq / dp
        pred = z * ((p[:, 0] - p[i, 0]) + 1j * (p[:, 1] - p[i, 1])) + complex(*q[i])
        dist = np.abs((q[:, 0] + 1j * q[:, 1]) - pred)
        clear = np.abs(dist - thr) > 1e-6 * max(thr, 1)
        assert np.array_equal(mask[clear], (dist <= thr)[clear])


def test_hypothesis_rule_picks_two_distinct_matches():
    words = synth.ransac_words(1, 500, seed=3)[0]
    for M in (2, 3, 7, 1000):
        for u, v in words:
            i = int(u) % M
            j = int(v) % (M - 1)
            j += 1 if j >= i else 0
            assert 0 <= i < M and 0 <= j < M and i != j


def test_planted_similarity_with_outliers_is_recovered():
    rng = np.random.default_rng(2)
    n = 400
    kq = rng.integers(-20000, 20000, size=(n, 2)).astype(np.int32)
    kd = _similarity(kq, (2, 1), (-300, 900)).astype(np.int32)
    match = np.arange(n, dtype=np.int32)
    bad = rng.random(n) < 0.4
    match[bad] = rng.permutation(n)[: bad.sum()]
    match[bad & (match == np.arange(n))] = -1
    words = synth.ransac_words(1, 64, seed=4)[0]
    out, best = R.ransac_pair(kq, kd, match, words, thr=0, min_inliers=10)
    good = match == np.arange(n)
    assert best == good.sum()
    assert np.array_equal(out >= 0, good)


# ------------------------------------------------------------------ library vs oracle

def _case(seed, n_q=250, n_d=240, frac=0.7, outliers=0.3, noise=3, spread=40000):
    rng = np.random.default_rng(seed)
    kq = rng.integers(-spread, spread, size=(n_q, 2)).astype(np.int32)
    kd = rng.integers(-spread, spread, size=(n_d, 2)).astype(np.int32)
    match = np.where(rng.random(n_q) < frac, rng.integers(0, n_d, n_q), -1).astype(np.int32)
    good = (match >= 0) & (rng.random(n_q) >= outliers)
    kd[match[good]] = (_similarity(kq[good], (1, 1), (55, -7)) +
                       rng.integers(-noise, noise + 1, size=(int(good.sum()), 2))).astype(np.int32)
    return kq, kd, match


@pytest.mark.parametrize("thr,min_inl,iters", [(8, 8, 48), (0, 2, 16), (200, 30, 5), (5, 1000, 20)])
def test_library_matches_oracle(thr, min_inl, iters):
    cases = [_case(s) for s in range(4)]
    cases.append(_case(9, n_q=30, frac=0.1))            # a few matches
    cases.append(_case(10, n_q=40, frac=0.0))           # none
    cases.append(_case(11, n_q=20, frac=0.06))          # one or two
    kps, pairs, parts = [], [], []
    for kq, kd, m in cases:
        pairs.append((len(kps), len(kps) + 1))
        kps += [kq, kd]
        parts.append(m)
    offs = np.concatenate([[0], np.cumsum([len(m) for m in parts])]).astype(np.int64)
    words = synth.ransac_words(len(pairs), iters, seed=thr + iters)
    out, best = chm.ransac_filter(kps, np.array(pairs), offs, np.concatenate(parts), words, thr, min_inl,
                                  n_threads=3)
    for p, (kq, kd, m) in enumerate(cases):
        ro, rb = R.ransac_pair(kq, kd, m, words[p], thr, min_inl)
        assert np.array_equal(out[offs[p]:offs[p + 1]], ro), p
        assert best[p] == rb, p


def test_library_on_synthetic_workload_with_repeated_texture():
    wl = synth.config2(n_images=5, n_feats=600, k=2, repeat_frac=0.3)
    kps = synth.keypoints(wl)
    rng = np.random.default_rng(6)
    parts = []
    for q, d in wl.pairs:
        tq, td = wl.tracks[q], wl.tracks[d]
        pos = {int(t): i for i, t in enumerate(td) if t >= 0}
        m = np.array([pos.get(int(t), -1) for t in tq], np.int32)
        r = rng.random(len(m)) < 0.15
        m[r] = rng.integers(0, len(td), int(r.sum()))
        parts.append(m)
    offs = np.concatenate([[0], np.cumsum([len(m) for m in parts])]).astype(np.int64)
    words = synth.ransac_words(len(wl.pairs), 64)
    out, best = chm.ransac_filter(kps, wl.pairs, offs, np.concatenate(parts), words, 64, 8)
    for p in range(len(wl.pairs)):
        q, d = wl.pairs[p]
        ro, rb = R.ransac_pair(kps[q], kps[d], parts[p], words[p], 64, 8)
        assert np.array_equal(out[offs[p]:offs[p + 1]], ro) and best[p] == rb


def test_library_filters_in_place_and_rejects_bad_input():
    kq, kd, m = _case(12)
    words = synth.ransac_words(1, 32, seed=7)
    kps = [kq, kd]
    ptrs = (C.c_void_p * 2)(*[k.ctypes.data for k in kps])
    nf = np.array([len(kq), len(kd)], np.int32)
    pairs = np.array([[0, 1]], np.int32)
    offs = np.array([0, len(m)], np.int64)
    buf = m.copy()
    st = chm.lib().chm_ransac_filter(1, pairs.ctypes.data, C.cast(ptrs, C.c_void_p), nf.ctypes.data, 2,
                                     offs.ctypes.data, buf.ctypes.data, words.ctypes.data, 32, 8, 8, 1,
                                     buf.ctypes.data, None)
    assert st == 0
    assert np.array_equal(buf, R.ransac_pair(kq, kd, m, words[0], 8, 8)[0])
    far = kq.copy()
    far[np.argmax(m >= 0)] = (1 << 19, 0)
    with pytest.raises(chm.ChmError, match="coordinate"):
        chm.ransac_filter([far, kd], pairs, offs, m, words, 8)
    bad = m.copy()
    bad[np.argmax(bad >= 0)] = len(kd)
    with pytest.raises(chm.ChmError, match="db row"):
        chm.ransac_filter([kq, kd], pairs, offs, bad, words, 8)
    with pytest.raises(chm.ChmError, match="thr"):
        chm.ransac_filter([kq, kd], pairs, offs, m, words, 1 << 20)

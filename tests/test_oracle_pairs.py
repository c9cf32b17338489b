"""Pins of the oracle's multi-pair driver (``orc_match_pairs``).

Every full-size parity check compares the HIP path with this driver, so it is
pinned twice on the CPU:

* it equals the single-pair routine called pair by pair and concatenated
  (matches, top-K keys and candidate counts), on pair lists that repeat
  pairs, hold self pairs and empty and one-feature images, with one and with
  several threads (one thread reuses its scratch for every pair, so a stale
  candidate stamp or an offset slip between pairs shows);
* independently of the single-pair routine, its top-K keys equal the dense
  formulation of steps (1)-(3) of Sec. 2.3.1 (the candidate set is every db
  point sharing a bucket in some table, ranked by (Hamming distance, index))
  and its matches equal exact 2-NN + ratio test over those K candidates with
  SciPy's distances.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from paper_2505_22089_amd import synth

L, M = 6, 8
SIZES = [0, 1, 37, 120, 64, 300, 1, 9]


@pytest.fixture(scope="module")
def images(orc):
    rng = np.random.default_rng(21)
    base = synth.sift_like(rng, 200)
    X = []
    for k, n in enumerate(SIZES):
        # half of each image are noisy copies of a shared pool, so pairs have
        # real matches as well as distractors
        c = min(n, n // 2)
        part = synth.noisy_copy(rng, base[rng.choice(200, size=c, replace=False)]) if c else base[:0]
        X.append(np.concatenate([part, synth.sift_like(rng, n - c)])[rng.permutation(n)])
    X.append(X[3].copy())  # an identical copy of an image, as a separate image
    W = synth.projection_weights(42, 128 + L * M)
    mu = synth.centring_vector(X)
    H = [orc.hash_image(x, W, mu, L, M) for x in X]
    return X, H


def pair_list(n_images, seed):
    rng = np.random.default_rng(seed)
    p = [(3, 3), (5, 2), (0, 4), (4, 0), (1, 5), (5, 1), (6, 1), (1, 6), (0, 0), (8, 3), (3, 8)]
    p += [tuple(int(v) for v in rng.integers(0, n_images, 2)) for _ in range(25)]
    p += [(5, 2), (5, 2), (2, 5)]  # repeated pairs, both directions
    return np.array(p, np.int32)


def per_pair(orc, H, pairs, K, ratio, single, whole):
    outs, keys, total = [], [], 0
    for q, d in pairs:
        o, t, nc = orc.match_pair(H[q], H[d], L, M, K, ratio, want_topk=True, accept_single=single,
                                  whole_last_bucket=whole)
        outs.append(o)
        keys.append(t)
        total += nc
    return np.concatenate(outs), np.concatenate(keys), total


@pytest.mark.parametrize("K,ratio,single,whole", [(8, (4, 5), False, False), (2, (1, 1), False, False),
                                                  (1, (4, 5), True, False), (3, (99, 100), False, True),
                                                  (32, (2, 3), True, True)])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_match_pairs_equals_single_pairs_concatenated(orc, images, K, ratio, single, whole, threads):
    X, H = images
    pairs = pair_list(len(H), seed=K + threads)
    ref_out, ref_keys, ref_nc = per_pair(orc, H, pairs, K, ratio, single, whole)
    prev = orc.max_threads()
    orc.set_threads(threads)
    try:
        out, offs, topk, nc = orc.match_pairs(H, pairs, L, M, K, ratio, want_topk=True, accept_single=single,
                                              whole_last_bucket=whole)
    finally:
        orc.set_threads(prev)
    expect_offs = np.concatenate([[0], np.cumsum([X[q].shape[0] for q in pairs[:, 0]])])
    assert np.array_equal(offs, expect_offs)
    assert np.array_equal(out, ref_out)
    assert np.array_equal(topk, ref_keys)
    assert nc == ref_nc
    assert (out >= 0).sum() > 20  # the list has real matches


def test_match_pairs_equals_dense_formulation(orc, images):
    """One thread, so every pair reuses the same candidate stamps."""
    X, H = images
    K = 4
    pairs = pair_list(len(H), seed=5)
    prev = orc.max_threads()
    orc.set_threads(1)
    try:
        out, offs, topk, nc = orc.match_pairs(H, pairs, L, M, K, (4, 5), want_topk=True)
    finally:
        orc.set_threads(prev)
    total = 0
    for p, (q, d) in enumerate(pairs):
        hq, hd = H[q], H[d]
        qi = [sum(int(w) << (32 * k) for k, w in enumerate(c)) for c in hq.codes]
        di = [sum(int(w) << (32 * k) for k, w in enumerate(c)) for c in hd.codes]
        D = cdist(X[q].astype(np.float64), X[d].astype(np.float64), "sqeuclidean").astype(np.int64) \
            if X[q].shape[0] and X[d].shape[0] else None
        for i in range(X[q].shape[0]):
            cand = np.nonzero((hq.ids[i][None, :] == hd.ids).any(axis=1))[0]
            total += len(cand)
            ranked = sorted((bin(qi[i] ^ di[j]).count("1"), int(j)) for j in cand)[:K]
            expect = [(h << 24) | j for h, j in ranked] + [0xFFFFFFFF] * (K - len(ranked))
            assert list(topk[offs[p] + i]) == expect, (p, i)
            m = -1
            if len(ranked) >= 2:
                by_dist = sorted(ranked, key=lambda hj: (D[i, hj[1]], hj[1]))
                d1, d2 = D[i, by_dist[0][1]], D[i, by_dist[1][1]]
                if 25 * d1 < 16 * d2:
                    m = by_dist[0][1]
            assert out[offs[p] + i] == m, (p, i)
    assert nc == total

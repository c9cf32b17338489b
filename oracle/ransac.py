"""Plain RANSAC global verification of a pair's matches (Sec. 2.3.3).

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg import it; the product path never does.

Model: a 2D similarity q = z * (p - p_i) + q_i in complex notation, fixed by
two correspondences (i, j): z = (q_j - q_i) / (p_j - p_i).  For a third
match k the residual is r_k = (q_k - q_i) - z * (p_k - p_i); k is an inlier
when |r_k| <= thr.  With D = |p_j - p_i|^2 and w = (q_j - q_i) * conj(p_j -
p_i) (so z = w / D) the test is |D (q_k - q_i) - w (p_k - p_i)|^2 <=
D^2 thr^2, exact in integers.

Hypotheses: iteration t draws two random words (u_t, v_t) (inputs, not drawn
here); with M matches, i = u_t mod M and j = v_t mod (M - 1), j += 1 when
j >= i, so i != j.  A sample with p_i = p_j is skipped (no model).  The best
hypothesis has the most inliers; ties keep the earlier one.  The pair is
verified when that count reaches min_inliers; its verified matches are the
best hypothesis' inliers, the others (and every match of an unverified
pair) become -1.  Fewer than two matches: nothing is verified.

Readings (the paper names RANSAC without its model or parameters): the
synthetic views are similarity transforms of a plane, so the model is a
similarity; the iteration count, threshold and minimum inlier count are
parameters.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def inliers_of(P: np.ndarray, Q: np.ndarray, i: int, j: int, thr: int) -> np.ndarray:
    """Inlier mask of the similarity through matches i and j (None if p_i = p_j)."""
    pix, piy = int(P[i, 0]), int(P[i, 1])
    qix, qiy = int(Q[i, 0]), int(Q[i, 1])
    dpx, dpy = int(P[j, 0]) - pix, int(P[j, 1]) - piy
    dqx, dqy = int(Q[j, 0]) - qix, int(Q[j, 1]) - qiy
    D = dpx * dpx + dpy * dpy
    if D == 0:
        return None
    wr, wi = dqx * dpx + dqy * dpy, dqy * dpx - dqx * dpy   # w = dq * conj(dp)
    lim = D * D * thr * thr
    mask = np.zeros(len(P), bool)
    for k in range(len(P)):
        ex, ey = int(P[k, 0]) - pix, int(P[k, 1]) - piy
        fx, fy = int(Q[k, 0]) - qix, int(Q[k, 1]) - qiy
        rx = D * fx - (wr * ex - wi * ey)
        ry = D * fy - (wr * ey + wi * ex)
        mask[k] = rx * rx + ry * ry <= lim
    return mask


def ransac_pair(kp_q: np.ndarray, kp_d: np.ndarray, match: np.ndarray, words: np.ndarray,
                thr: int, min_inliers: int) -> Tuple[np.ndarray, int]:
    """(verified matches per query row, inlier count of the best hypothesis)."""
    match = np.asarray(match)
    rows = np.nonzero(match >= 0)[0]
    M = len(rows)
    out = np.full(len(match), -1, np.int32)
    if M < 2:
        return out, 0
    P = np.asarray(kp_q, dtype=np.int64)[rows]
    Q = np.asarray(kp_d, dtype=np.int64)[match[rows]]
    best, best_mask = -1, None
    for u, v in np.asarray(words, dtype=np.uint64).reshape(-1, 2):
        i = int(u) % M
        j = int(v) % (M - 1)
        j += 1 if j >= i else 0
        mask = inliers_of(P, Q, i, j, thr)
        if mask is None:
            continue
        c = int(mask.sum())
        if c > best:
            best, best_mask = c, mask
    if best_mask is None or best < min_inliers:
        return out, max(best, 0)
    out[rows[best_mask]] = match[rows[best_mask]]
    return out, best

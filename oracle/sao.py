"""Plain SAO local geometric constraint (Sec. 2.3.3, Fig. 4).

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg import it; the product path never does.

For one directed image pair with initial matches i -> m(i) (query row i,
db row m(i), -1 for none), every match is scored as follows:

* its keypoints are p_i in the query image and q_i = db keypoint m(i);
* N = min(n_neighbors, M - 1), with M the number of matches of the pair;
* O_p: the N other matches whose query keypoints are nearest to p_i (squared
  Euclidean distance, ties by the smaller match label = query row);
  O_q: the N other matches whose db keypoints are nearest to q_i (a db
  keypoint matched by several queries is one point per match);
* each list is put in angular order around its centre: counter-clockwise
  from the +x axis, angles in [0, 2 pi); a neighbour on the centre itself
  comes first; equal angles by distance, then label;
* the dissimilarity is CED(labels of O_p, labels of O_q) / N, where CED is
  the cyclic edit distance: the smallest Levenshtein distance (unit insert,
  delete and substitute costs) over all rotations of both sequences;
* a match is kept when that score is at most the threshold num / den, i.e.
  CED * den <= num * N (N = 0 keeps the match with CED 0).

Coordinates are integers (any unit, |x|, |y| < 2^30), so every distance and
every angular comparison is exact.

Readings (the paper leaves them open): the neighbour set is the exact
Euclidean k-nearest set (the paper derives it from a Delaunay graph, a search
structure for the same neighbours); the default N = 6 follows its figure; the
threshold is a parameter, default 1/2.
"""
from __future__ import annotations

import functools
from typing import List, Optional, Sequence, Tuple

import numpy as np


def levenshtein(a: Sequence[int], b: Sequence[int]) -> int:
    """Textbook dynamic programme with unit costs."""
    n, m = len(a), len(b)
    prev = list(range(m + 1))
    for i in range(1, n + 1):
        cur = [i] + [0] * m
        for j in range(1, m + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[m]


def cyclic_edit_distance(a: Sequence[int], b: Sequence[int]) -> int:
    """Minimum Levenshtein distance over every rotation of a and of b."""
    a, b = list(a), list(b)
    best = levenshtein(a, b)
    for i in range(len(a)):
        for j in range(len(b)):
            best = min(best, levenshtein(a[i:] + a[:i], b[j:] + b[:j]))
    return best


def _half(v: Tuple[int, int]) -> int:
    """-1 for the zero vector, 0 for angles in [0, pi), 1 for [pi, 2 pi)."""
    x, y = v
    if x == 0 and y == 0:
        return -1
    return 0 if (y > 0 or (y == 0 and x > 0)) else 1


def angle_cmp(u: Tuple[int, int, int, int], v: Tuple[int, int, int, int]) -> int:
    """Order of (dx, dy, d2, label) entries: angle, then distance, then label."""
    hu, hv = _half(u[:2]), _half(v[:2])
    if hu != hv:
        return -1 if hu < hv else 1
    if hu >= 0:
        cross = u[0] * v[1] - u[1] * v[0]
        if cross != 0:
            return -1 if cross > 0 else 1
    if u[2] != v[2]:
        return -1 if u[2] < v[2] else 1
    return (u[3] > v[3]) - (u[3] < v[3])


def angular_order(centre: Tuple[int, int], pts: Sequence[Tuple[int, int]],
                  labels: Sequence[int]) -> List[int]:
    entries = []
    for (x, y), lab in zip(pts, labels):
        dx, dy = int(x) - int(centre[0]), int(y) - int(centre[1])
        entries.append((dx, dy, dx * dx + dy * dy, int(lab)))
    entries.sort(key=functools.cmp_to_key(angle_cmp))
    return [e[3] for e in entries]


def nearest(centre: Tuple[int, int], pts: np.ndarray, labels: np.ndarray, own: int,
            n: int) -> List[int]:
    """Indices (into pts) of the n nearest points other than label `own`,
    by squared distance, ties by label (int64: exact below 2^30)."""
    pts = np.asarray(pts, dtype=np.int64)
    labels = np.asarray(labels, dtype=np.int64)
    d2 = (pts[:, 0] - int(centre[0])) ** 2 + (pts[:, 1] - int(centre[1])) ** 2
    keep = np.nonzero(labels != own)[0]
    order = keep[np.lexsort((labels[keep], d2[keep]))]
    return [int(k) for k in order[:n]]


def sao_pair(kp_q: np.ndarray, kp_d: np.ndarray, match: np.ndarray, n_neighbors: int = 6,
             threshold: Tuple[int, int] = (1, 2),
             only_rows: Optional[Sequence[int]] = None) -> Tuple[np.ndarray, np.ndarray]:
    """(CED per query row, -1 where unmatched; filtered matches).  With
    only_rows, just those query rows are scored (the others stay -1)."""
    match = np.asarray(match)
    rows = np.nonzero(match >= 0)[0]
    M = len(rows)
    N = min(n_neighbors, M - 1) if M else 0
    P = np.asarray(kp_q, dtype=np.int64)[rows]
    Q = np.asarray(kp_d, dtype=np.int64)[match[rows]]
    ced = np.full(len(match), -1, np.int64)
    out = np.full(len(match), -1, np.int32)
    num, den = threshold
    wanted = None if only_rows is None else set(int(r) for r in only_rows)
    for a, i in enumerate(rows):
        if wanted is not None and int(i) not in wanted:
            continue
        if N == 0:
            ced[i] = 0
        else:
            kp = nearest(P[a], P, rows, int(i), N)
            kq = nearest(Q[a], Q, rows, int(i), N)
            op = angular_order(P[a], [tuple(P[k]) for k in kp], rows[kp])
            oq = angular_order(Q[a], [tuple(Q[k]) for k in kq], rows[kq])
            ced[i] = cyclic_edit_distance(op, oq)
        if ced[i] * den <= num * N:
            out[i] = match[i]
    return ced, out


def sao_pairs(kps: Sequence[np.ndarray], pairs: np.ndarray, offs: np.ndarray, out: np.ndarray,
              n_neighbors: int = 6, threshold: Tuple[int, int] = (1, 2),
              which: Optional[Sequence[int]] = None):
    """sao_pair over the listed pairs (all by default); returns per pair
    (ced, filtered) for the pairs in `which`."""
    res = []
    for p in (range(len(pairs)) if which is None else which):
        q, d = pairs[p]
        res.append(sao_pair(kps[q], kps[d], out[offs[p]:offs[p + 1]], n_neighbors, threshold))
    return res

"""Seeded synthetic workloads for cascade-hashing matching.

This module only draws inputs: descriptors, view graphs (directed image pairs),
the random projection matrix and the centring vector.  It holds none of the
matching arithmetic, and both the HIP path and the CPU oracle take its output
as plain arrays.

The paper's UAV datasets (Table 1), their SIFT features and retrieved pairs
(Table 3) are not available, so these stand-ins copy their shape: 128-d uint8
SIFT-like descriptors with at most a few thousand to tens of thousands of
features per image (Sec. 3.4.1 caps features at 8,192), sparse, near-banded view
graphs (Fig. 9/10) and about 10-17 pairs per image (Table 3 / Table 1).

Recipe
------
* SIFT-like descriptor: z = |N(0, 40^2)|^128 in float64, x = clip(rint(512 z /
  ||z||_2), 0, 255) as uint8 (rint is round-half-even).
* Noisy copy of x: clip(rint(x + sigma * N(0, 1)), 0, 255), sigma = 8 unless
  stated, the normal draws in float32, not renormalised.
* Multi-image workloads use a footprint/track model: image centres in the
  plane, square footprints of side F, a global set of tracks (position + base
  descriptor) with uniform density; an image observes the tracks inside its
  footprint as noisy copies (at most ``cap_frac`` of its feature count,
  subsampled when more fall inside) and fills the rest with fresh draws, rows
  shuffled.  F is chosen by bisection on the analytic mean overlap
  |shared| / min(N_q, N_d) over the listed pairs; the realised overlap is
  measured and reported in ``Workload.meta``.
* Projection matrix: z = default_rng(seed).standard_normal((R, 128)) rounded
  once, float64 -> bfloat16 with round-to-nearest-even, magnitudes below 2^-16
  flushed to +0; returned as bf16 bit patterns (uint16).
* Centring vector mu: per dimension, the round-half-up integer mean over every
  descriptor of the workload, computed in int64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

DIM = 128
CODE_BITS = 128
SEED_W = 42


def sift_like(rng: np.random.Generator, n: int) -> np.ndarray:
    """n SIFT-like uint8 descriptors (half-normal, L2-normalised to 512)."""
    z = np.abs(rng.normal(0.0, 40.0, size=(n, DIM)))
    nrm = np.sqrt(np.einsum("ij,ij->i", z, z))[:, None]
    nrm[nrm == 0] = 1.0
    x = np.rint(512.0 * z / nrm)
    return np.clip(x, 0, 255).astype(np.uint8)


def noisy_copy(rng: np.random.Generator, x: np.ndarray, sigma: float = 8.0) -> np.ndarray:
    """Noisy copies of the rows of x (Gaussian sigma, re-clipped to 0..255)."""
    noise = rng.standard_normal(size=x.shape, dtype=np.float32) * np.float32(sigma)
    y = np.rint(x.astype(np.float32) + noise)
    return np.clip(y, 0, 255).astype(np.uint8)


def projection_weights(seed: int = SEED_W, rows: int = 176, dim: int = DIM) -> np.ndarray:
    """bfloat16 bit patterns (uint16, rows x dim) of a seeded Gaussian matrix."""
    z = np.random.default_rng(seed).standard_normal((rows, dim))
    mant, expo = np.frexp(z)                      # z = mant * 2**expo, 0.5 <= |mant| < 1
    q = np.ldexp(np.rint(mant * 256.0), expo - 8)  # 8 significant bits, ties to even
    q[np.abs(q) < 2.0 ** -16] = 0.0
    q = q + 0.0                                   # -0 -> +0
    if not np.all(np.abs(q) < 32.0):
        raise ValueError("projection weight magnitude out of range")
    bits = (q.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return bits


def centring_vector(images: List[np.ndarray]) -> np.ndarray:
    """Round-half-up integer mean of all descriptors, per dimension (uint8)."""
    tot = np.zeros(DIM, dtype=np.int64)
    n = 0
    for x in images:
        tot += x.astype(np.int64).sum(axis=0)
        n += x.shape[0]
    if n == 0:
        return np.zeros(DIM, dtype=np.uint8)
    return ((2 * tot + n) // (2 * n)).astype(np.uint8)


@dataclass
class Workload:
    name: str
    images: List[np.ndarray]
    pairs: np.ndarray                 # (P, 2) int32, directed (query image, db image)
    W: np.ndarray                     # (R, 128) uint16 bf16 bits
    mu: np.ndarray                    # (128,) uint8
    L: int = 6
    m: int = 8
    K: int = 8
    ratio: tuple = (4, 5)
    tracks: Optional[List[np.ndarray]] = None   # per image, track id per row (-1 fresh)
    gt: Optional[np.ndarray] = None             # (G, 2) planted (row in A, row in B), pair 0
    centres: Optional[np.ndarray] = None
    track_pos: Optional[np.ndarray] = None      # (T, 2) plane position of each track
    meta: Dict = field(default_factory=dict)

    @property
    def n_feats(self) -> np.ndarray:
        return np.array([x.shape[0] for x in self.images], dtype=np.int64)


# ---------------------------------------------------------------- view graphs

def knn_pairs(centres: np.ndarray, k: int) -> np.ndarray:
    """Directed pairs i -> each of its k nearest centres (ties by smaller id)."""
    n = len(centres)
    d2 = ((centres[:, None, :] - centres[None, :, :]) ** 2).sum(-1)
    out = []
    for i in range(n):
        order = np.lexsort((np.arange(n), d2[i]))
        nb = [j for j in order if j != i][:k]
        out.extend((i, j) for j in nb)
    return np.array(out, dtype=np.int32).reshape(-1, 2)


def offset_grid_pairs(rows: int, cols: int, offsets) -> np.ndarray:
    """Directed pairs on a rows x cols grid (id = r*cols + c) for each offset (dr, dc)."""
    out = []
    for r in range(rows):
        for c in range(cols):
            for dr, dc in offsets:
                rr, cc = r + dr, c + dc
                if 0 <= rr < rows and 0 <= cc < cols:
                    out.append((r * cols + c, rr * cols + cc))
    return np.array(out, dtype=np.int32).reshape(-1, 2)


STRIP_12 = [(0, 1), (0, -1), (0, 2), (0, -2), (1, 0), (-1, 0),
            (1, 1), (1, -1), (-1, 1), (-1, -1), (2, 0), (-2, 0)]


def band_grid_pairs(rows: int, cols: int, max_dr: int, max_dc: int) -> np.ndarray:
    offs = [(dr, dc) for dr in range(-max_dr, max_dr + 1) for dc in range(-max_dc, max_dc + 1)
            if (dr, dc) != (0, 0)]
    return offset_grid_pairs(rows, cols, offs)


def cross_links(rng: np.random.Generator, rows: int, cols: int, lo: int = 3, hi: int = 6) -> np.ndarray:
    """One oblique directed link per image to a strip lo..hi rows away."""
    out = []
    for r in range(rows):
        for c in range(cols):
            choices = [rr for rr in range(rows) if lo <= abs(rr - r) <= hi]
            if not choices:
                continue
            rr = int(choices[rng.integers(len(choices))])
            cc = int(np.clip(c + rng.integers(-3, 4), 0, cols - 1))
            out.append((r * cols + c, rr * cols + cc))
    return np.array(out, dtype=np.int32).reshape(-1, 2)


# ---------------------------------------------------------------- track model

def _expected_overlap(F, centres, feats, pairs, cap_frac):
    nbar = feats.mean()
    q, d = pairs[:, 0], pairs[:, 1]
    dx = np.abs(centres[q, 0] - centres[d, 0])
    dy = np.abs(centres[q, 1] - centres[d, 1])
    seen = cap_frac * nbar
    keep = np.minimum(1.0, cap_frac * feats / seen)
    frac = np.clip(1 - dx / F, 0, None) * np.clip(1 - dy / F, 0, None)
    shared = seen * frac * keep[q] * keep[d]
    return float(np.mean(shared / np.minimum(feats[q], feats[d])))


def track_workload(name: str, seed: int, centres: np.ndarray, feats, pairs: np.ndarray,
                   target_overlap: float, cap_frac: float = 0.9, K: int = 8,
                   measure_pairs: int = 2000, progress=None, noise: float = 8.0,
                   repeat_frac: float = 0.0, repeat_sigma: float = 4.0) -> Workload:
    """Footprint/track model; progress(msg), if given, is called as the
    (possibly long) generation advances.  Chunked draws equal one draw.
    repeat_frac > 0 models repeated texture: that fraction of the tracks
    take a noisy copy (repeat_sigma) of another track's base descriptor, so
    look-alike points sit at unrelated places."""
    rng = np.random.default_rng(seed)
    centres = np.asarray(centres, dtype=np.float64)
    feats = np.asarray(feats, dtype=np.int64)
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    lo, hi = 1e-3, 1e3
    for _ in range(80):
        mid = np.sqrt(lo * hi)
        if _expected_overlap(mid, centres, feats, pairs, cap_frac) < target_overlap:
            lo = mid
        else:
            hi = mid
    F = float(hi)
    nbar = feats.mean()
    rho = cap_frac * nbar / (F * F)
    x0, y0 = centres.min(0) - F / 2
    x1, y1 = centres.max(0) + F / 2
    T = int(round(rho * (x1 - x0) * (y1 - y0)))
    pos = np.empty((T, 2))
    pos[:, 0] = rng.uniform(x0, x1, T)
    pos[:, 1] = rng.uniform(y0, y1, T)
    order = np.argsort(pos[:, 0], kind="stable")
    pos = pos[order]
    chunk = 1 << 20
    parts = []
    for c0 in range(0, T, chunk):
        parts.append(sift_like(rng, min(chunk, T - c0)))
        if progress:
            progress("tracks %d / %d" % (min(T, c0 + chunk), T))
    base = np.concatenate(parts) if parts else sift_like(rng, 0)
    del parts
    if repeat_frac > 0 and T > 1:
        nrep = int(repeat_frac * T)
        dst = rng.choice(T, size=nrep, replace=False)
        src = rng.integers(0, T, size=nrep)
        base[dst] = noisy_copy(rng, base[src], repeat_sigma)
    images, tracks = [], []
    for i, (cx, cy) in enumerate(centres):
        if progress and i and i % 250 == 0:
            progress("images %d / %d" % (i, len(centres)))
        a = np.searchsorted(pos[:, 0], cx - F / 2, side="left")
        b = np.searchsorted(pos[:, 0], cx + F / 2, side="right")
        cand = np.arange(a, b)
        cand = cand[np.abs(pos[a:b, 1] - cy) <= F / 2]
        n_i = int(feats[i])
        cap = int(cap_frac * n_i)
        if len(cand) > cap:
            cand = np.sort(rng.choice(cand, size=cap, replace=False))
        obs = noisy_copy(rng, base[cand], noise)
        fresh = sift_like(rng, n_i - len(cand))
        x = np.concatenate([obs, fresh], axis=0)
        tid = np.concatenate([cand.astype(np.int64), -np.ones(n_i - len(cand), np.int64)])
        perm = rng.permutation(n_i)
        images.append(np.ascontiguousarray(x[perm]))
        tracks.append(tid[perm])
    # realised overlap on a sample of pairs
    samp = pairs if len(pairs) <= measure_pairs else pairs[
        np.sort(rng.choice(len(pairs), measure_pairs, replace=False))]
    ov = []
    for q, d in samp:
        tq = tracks[q][tracks[q] >= 0]
        td = tracks[d][tracks[d] >= 0]
        ov.append(len(np.intersect1d(tq, td, assume_unique=True)) /
                  max(1, min(feats[q], feats[d])))
    ov = np.array(ov) if ov else np.zeros(1)
    W = projection_weights(SEED_W, CODE_BITS + 6 * 8)
    mu = centring_vector(images)
    meta = dict(footprint=F, tracks=T, target_overlap=target_overlap,
                overlap_mean=float(ov.mean()), overlap_min=float(ov.min()),
                overlap_max=float(ov.max()), overlap_sampled_pairs=int(len(samp)))
    return Workload(name=name, images=images, pairs=pairs, W=W, mu=mu, K=K,
                    tracks=tracks, centres=centres, track_pos=pos, meta=meta)


def keypoints(wl: Workload, size_px: float = 4000.0, sigma_px: float = 1.0, subpix: int = 16,
              seed: int = 77) -> List[np.ndarray]:
    """Integer keypoint coordinates (units of 1/subpix pixel), one (n, 2)
    int32 array per image of a footprint/track workload.

    Image i sees its square footprint (side F, centre c_i) as size_px pixels,
    turned by a heading drawn uniformly in [0, 2 pi): a tracked row sits at
    R(heading) (p_track - c_i) size_px / F + size_px / 2 plus N(0, sigma_px^2)
    per axis; a fresh row is uniform over [0, size_px)^2.  The draws use
    their own generator, so the descriptors are unchanged."""
    if wl.tracks is None or wl.track_pos is None:
        raise ValueError("keypoints need a footprint/track workload")
    rng = np.random.default_rng(seed)
    F = float(wl.meta["footprint"])
    out = []
    for i, tid in enumerate(wl.tracks):
        th = rng.uniform(0.0, 2.0 * np.pi)
        rot = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        xy = rng.uniform(0.0, size_px, size=(len(tid), 2))
        t = tid >= 0
        rel = (wl.track_pos[tid[t]] - wl.centres[i]) * (size_px / F)
        xy[t] = rel @ rot.T + size_px / 2 + rng.normal(0.0, sigma_px, size=(int(t.sum()), 2))
        out.append(np.rint(xy * subpix).astype(np.int32))
    return out


def ransac_words(n_pairs: int, iterations: int, seed: int = 99) -> np.ndarray:
    """Random 32-bit words for RANSAC hypotheses: (n_pairs, iterations, 2)
    uint32, two per hypothesis (they pick its two matches)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 32, size=(n_pairs, iterations, 2), dtype=np.uint64).astype(np.uint32)


# ---------------------------------------------------------------- the five workloads

def config1(n: int = 2000, planted: int = 1000, seed: int = 1001) -> Workload:
    """Single pair A -> B: B = noisy copies of a seeded subset of A + fresh, shuffled."""
    rng = np.random.default_rng(seed)
    A = sift_like(rng, n)
    idx = rng.choice(n, size=planted, replace=False)
    B0 = np.concatenate([noisy_copy(rng, A[idx]), sift_like(rng, n - planted)], axis=0)
    perm = rng.permutation(n)
    B = np.ascontiguousarray(B0[perm])
    rows = np.nonzero(perm < planted)[0]
    gt = np.stack([idx[perm[rows]], rows], axis=1).astype(np.int32)
    images = [A, B]
    W = projection_weights(SEED_W, CODE_BITS + 6 * 8)
    return Workload(name="pair-2x%d" % n, images=images,
                    pairs=np.array([[0, 1]], dtype=np.int32), W=W,
                    mu=centring_vector(images), K=2, gt=gt)


def config2(n_images: int = 50, n_feats: int = 8000, k: int = 8, K: int = 8,
            seed: int = 1002, noise: float = 8.0, repeat_frac: float = 0.0) -> Workload:
    """n_images x n_feats, centres uniform in a square, k-NN directed pairs, 40% overlap."""
    rng = np.random.default_rng(seed)
    side = np.sqrt(n_images)
    centres = rng.uniform(0, side, size=(n_images, 2))
    pairs = knn_pairs(centres, k)
    return track_workload("knn-%dx%d" % (n_images, n_feats), seed + 7, centres,
                          np.full(n_images, n_feats), pairs, 0.40, K=K, noise=noise,
                          repeat_frac=repeat_frac)


def config3(strips: int = 25, per_strip: int = 20, lo: int = 2000, hi: int = 20000,
            seed: int = 1003) -> Workload:
    """Flight-strip grid, log-uniform feature counts, 12-neighbourhood, 30% overlap."""
    rng = np.random.default_rng(seed)
    n = strips * per_strip
    feats = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), n))).astype(np.int64)
    centres = np.array([(c, r) for r in range(strips) for c in range(per_strip)], dtype=np.float64)
    pairs = offset_grid_pairs(strips, per_strip, STRIP_12)
    return track_workload("strips-%dx%d-lu%d-%d" % (strips, per_strip, lo, hi), seed + 7,
                          centres, feats, pairs, 0.30)


def config4(n_images: int = 200, n_feats: int = 40000, k: int = 10, seed: int = 1004) -> Workload:
    rng = np.random.default_rng(seed)
    side = np.sqrt(n_images)
    centres = rng.uniform(0, side, size=(n_images, 2))
    pairs = knn_pairs(centres, k)
    return track_workload("knn-%dx%d" % (n_images, n_feats), seed + 7, centres,
                          np.full(n_images, n_feats), pairs, 0.30)


def config5(rows: int = 50, cols: int = 100, n_feats: int = 10000, seed: int = 1005,
            progress=None) -> Workload:
    rng = np.random.default_rng(seed)
    pairs = np.concatenate([band_grid_pairs(rows, cols, 1, 3), cross_links(rng, rows, cols)])
    centres = np.array([(c, r) for r in range(rows) for c in range(cols)], dtype=np.float64)
    return track_workload("grid-%dx%d-%d" % (rows, cols, n_feats), seed + 7, centres,
                          np.full(rows * cols, n_feats), pairs, 0.30, progress=progress)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}

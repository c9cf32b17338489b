"""Device RANSAC (Sec. 2.3.3) through the C-ABI: verified matches and best
inlier counts equal the host verification (chm_ransac_filter, itself equal
to oracle/ransac.py in the CPU tests) on every pair, and the oracle's own
RANSAC on sampled pairs."""
import numpy as np
import pytest

from oracle import ransac as OR
from paper_2505_22089_amd import chm, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_helpers import device  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def random_case(seed, n_images=6, sizes=(0, 1, 2, 40, 300, 1500), coord=1 << 18):
    """Images with random keypoints; pairs whose matches mix -1, random db rows
    and rows that follow a planted similarity (so that hypotheses find real
    inlier sets), plus degenerate pairs (duplicate keypoints: D = 0)."""
    rng = np.random.default_rng(seed)
    n_feats = [int(rng.choice(sizes)) for _ in range(n_images)]
    kps = [rng.integers(-coord + 1, coord, size=(n, 2)).astype(np.int32) for n in n_feats]
    if n_feats[0] >= 4:
        kps[0][:] = kps[0][0]  # every keypoint of image 0 equal: all its hypotheses degenerate
    pairs = np.array([(q, d) for q in range(n_images) for d in range(n_images) if rng.random() < 0.6],
                     dtype=np.int32).reshape(-1, 2)
    offs = np.zeros(len(pairs) + 1, np.int64)
    offs[1:] = np.cumsum([n_feats[q] for q in pairs[:, 0]])
    match = np.full(int(offs[-1]), -1, np.int32)
    for p, (q, d) in enumerate(pairs):
        nq, nd = n_feats[q], n_feats[d]
        if nd == 0 or nq == 0:
            continue
        m = rng.integers(0, nd, size=nq).astype(np.int32)
        m[rng.random(nq) < 0.3] = -1
        # planted: db keypoint of a match moved onto a similarity of the query keypoint
        a, b = int(rng.integers(-3, 4)), int(rng.integers(-3, 4))
        tx, ty = int(rng.integers(-1000, 1000)), int(rng.integers(-1000, 1000))
        sel = np.nonzero((m >= 0) & (rng.random(nq) < 0.5))[0]
        for r in sel:
            x, y = int(kps[q][r, 0]) >> 3, int(kps[q][r, 1]) >> 3
            nx = a * x - b * y + tx + int(rng.integers(-20, 21))
            ny = b * x + a * y + ty + int(rng.integers(-20, 21))
            if abs(nx) < coord and abs(ny) < coord:
                kps[d][m[r]] = (nx, ny)
        match[offs[p]:offs[p + 1]] = m
    return kps, pairs, offs, match


@pytest.mark.parametrize("seed,iters,thr,min_in", [(0, 64, 64, 8), (1, 1, 100, 0), (2, 100, 0, 2),
                                                   (3, 300, 2000, 20), (4, 0, 64, 8), (5, 65, 64, 1)])
def test_device_ransac_equals_host(seed, iters, thr, min_in):
    kps, pairs, offs, match = random_case(seed)
    words = synth.ransac_words(len(pairs), iters, seed=seed)
    ref, ref_best = chm.ransac_filter(kps, pairs, offs, match, words, thr, min_in)
    d_match = _dev(match)
    d_out = torch.full_like(d_match, -7)
    d_best = torch.full((len(pairs),), -7, dtype=torch.int32, device=device())
    d_words = _dev(words.view(np.int32)) if iters else torch.zeros((len(pairs), 0, 2), dtype=torch.int32,
                                                                   device=device())
    work = chm.ransac_filter_device([_dev(k) for k in kps], pairs, offs, d_match, d_out, d_words, thr, min_in,
                                    best_counts=d_best)
    torch.cuda.synchronize()
    assert chm.sao_input_errors(work) == 0
    assert np.array_equal(d_out.cpu().numpy(), ref)
    assert np.array_equal(d_best.cpu().numpy(), ref_best)
    if iters and thr:
        assert (ref >= 0).any()
    # in place: the output may be the match array itself
    chm.ransac_filter_device([_dev(k) for k in kps], pairs, offs, d_match, d_match, d_words, thr, min_in)
    torch.cuda.synchronize()
    assert np.array_equal(d_match.cpu().numpy(), ref)


def test_device_ransac_matches_oracle_on_sampled_pairs():
    kps, pairs, offs, match = random_case(7, sizes=(60, 200, 400))
    iters, thr, min_in = 40, 300, 4
    words = synth.ransac_words(len(pairs), iters, seed=3)
    d_out = torch.full((len(match),), -7, dtype=torch.int32, device=device())
    chm.ransac_filter_device([_dev(k) for k in kps], pairs, offs, _dev(match), d_out, _dev(words.view(np.int32)),
                             thr, min_in)
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    for p in range(0, len(pairs), max(1, len(pairs) // 5)):
        q, d = pairs[p]
        v, _ = OR.ransac_pair(kps[q], kps[d], match[offs[p]:offs[p + 1]], words[p], thr, min_in)
        assert np.array_equal(out[offs[p]:offs[p + 1]], v), p


def _breaks_contract(kq, kd, m):
    lim = 1 << 19
    for r in np.nonzero(m >= 0)[0]:
        if m[r] >= len(kd):
            return True
        if (np.abs(kq[r].astype(np.int64)) >= lim).any() or (np.abs(kd[m[r]].astype(np.int64)) >= lim).any():
            return True
    return False


def test_device_ransac_counts_broken_pairs_and_keeps_the_rest():
    """A coordinate out of range or a db row outside the db image makes that
    pair verify nothing (the host call fails instead); the others are
    unchanged."""
    kps, pairs, offs, match = random_case(11, sizes=(100, 300))
    iters, thr, min_in = 32, 500, 4
    words = synth.ransac_words(len(pairs), iters, seed=5)
    kps_bad = [k.copy() for k in kps]
    bad_q = int(pairs[0, 0])
    rows = np.nonzero(match[offs[0]:offs[1]] >= 0)[0]
    kps_bad[bad_q][rows[0], 0] = 1 << 19  # out of range
    match_bad = match.copy()
    rows1 = np.nonzero(match[offs[1]:offs[2]] >= 0)[0]
    match_bad[offs[1] + rows1[0]] = 10 ** 6  # beyond the db image
    broken = {p for p in range(len(pairs))
              if _breaks_contract(kps_bad[pairs[p, 0]], kps_bad[pairs[p, 1]], match_bad[offs[p]:offs[p + 1]])}
    assert {0, 1} <= broken and len(broken) < len(pairs)
    d_out = torch.full((len(match),), -7, dtype=torch.int32, device=device())
    work = chm.ransac_filter_device([_dev(k) for k in kps_bad], pairs, offs, _dev(match_bad), d_out,
                                    _dev(words.view(np.int32)), thr, min_in)
    torch.cuda.synchronize()
    assert chm.sao_input_errors(work) == len(broken)
    out = d_out.cpu().numpy()
    keep = [p for p in range(len(pairs)) if p not in broken]
    koffs = np.concatenate([[0], np.cumsum([offs[p + 1] - offs[p] for p in keep])]).astype(np.int64)
    ref, _ = chm.ransac_filter(kps_bad, pairs[keep], koffs,
                               np.concatenate([match_bad[offs[p]:offs[p + 1]] for p in keep]), words[keep], thr,
                               min_in)
    got = np.concatenate([out[offs[p]:offs[p + 1]] for p in keep])
    assert np.array_equal(got, ref)
    for p in broken:
        assert (out[offs[p]:offs[p + 1]] == -1).all()


def test_schedule_with_sao_and_device_ransac_per_block_row():
    """An MBR schedule under a binding cap with the device SAO and the device
    RANSAC after every step: the verified matches equal host RANSAC of the
    SAO output on every pair."""
    from tests.gpu_helpers import device as dev
    wl = synth.config5(rows=5, cols=16, n_feats=1200)
    kps = synth.keypoints(wl)
    n = len(wl.images)
    cfg = chm.config(L=wl.L, m=wl.m, K=wl.K, ratio=wl.ratio)
    sizes = [chm.image_bytes(cfg, x.shape[0]) + 256 for x in wl.images]
    cap = 24 * sizes[0]
    sched = chm.schedule_mbr(n, wl.pairs, sizes, cap, 8, keep_handle=True)
    assert len(sched.steps) > 2
    arena = torch.empty(chm.store_overhead_bytes(cfg) + cap + (16 << 20), dtype=torch.uint8, device=dev())
    st = chm.Store(cfg, wl.W, wl.mu, arena)
    offs = np.zeros(len(wl.pairs) + 1, np.int64)
    offs[1:] = np.cumsum([wl.images[q].shape[0] for q in wl.pairs[:, 0]])
    total = int(offs[-1])
    out = torch.full((total,), -7, dtype=torch.int32, device=dev())
    filt = torch.full_like(out, -7)
    ver = torch.full_like(out, -7)
    iters, thr, min_in = 32, 64, 8
    words = synth.ransac_words(len(wl.pairs), iters)
    work, rwork = chm.run_schedule_verify_device(st, sched, wl.pairs, wl.images, offs, out,
                                                 [_dev(k) for k in kps], filt, ver, _dev(words.view(np.int32)),
                                                 iterations=iters,
                                                 thr=thr, min_inliers=min_in)
    torch.cuda.synchronize()
    assert chm.sao_input_errors(work) == 0 and chm.sao_input_errors(rwork) == 0
    chm.schedule_free(sched)
    st.close()
    f = filt.cpu().numpy()
    v = ver.cpu().numpy()
    ref_v, _ = chm.ransac_filter(kps, wl.pairs, offs, f, words, thr, min_in)
    assert np.array_equal(v, ref_v)
    assert (v >= 0).any()

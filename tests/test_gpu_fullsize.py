"""Full-size GPU parity through the C-ABI, in the batched launch configuration
the benchmark times.

* knn-50x8000 (the benchmark workload): every output of all 400 pairs;
* strips (500 images, 2k-20k features) and knn-200x40000: every pair matched
  on the GPU and compared with the oracle's stored per-pair digests
  (tests/golden/make_digests.py; both the LDS-staged and the global-memory
  match paths occur);
* a 1,200-image grid of 10,000-feature images, every pair against stored
  digests;
* a grid view graph run end to end through an MBR schedule whose residency
  cap binds (images loaded and evicted between block rows), every output
  against the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_22089_amd import chm, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from tests.gpu_helpers import device, gpu_arrays, load_all, new_store, run_match  # noqa: E402
from tests.digests import load_golden, match_counts, pair_digests  # noqa: E402


def oracle_slices(wl, pairs):
    """Oracle matches of the listed pairs (images hashed on demand)."""
    ids = sorted(set(np.asarray(pairs).ravel().tolist()))
    H = O.hash_workload(wl, ids)
    out, offs, _, _ = O.match_pairs(H, pairs, wl.L, wl.m, wl.K, wl.ratio)
    return [out[offs[k]:offs[k + 1]] for k in range(len(pairs))]


def gpu_slices(out, offs, idx):
    return [out[offs[p]:offs[p + 1]] for p in idx]


def test_knn_50x8000_all_pairs():
    wl = synth.config2()
    st = new_store(wl)
    load_all(st, wl.images)
    for i in (0, len(wl.images) - 1):
        g = gpu_arrays(st, i)
        ref = O.hash_image(wl.images[i], wl.W, wl.mu, wl.L, wl.m)
        assert np.array_equal(g["codes"], ref.codes) and np.array_equal(g["members"], ref.members)
    out, _, offs = run_match(st, wl.pairs)
    H = O.hash_workload(wl)
    ref, roffs, _, _ = O.match_pairs(H, wl.pairs, wl.L, wl.m, wl.K, wl.ratio)
    assert np.array_equal(offs, roffs)
    assert np.array_equal(out, ref)
    # the query-major kernel (LDS-staged codes, then HBM-only codes, small
    # work-groups), bucket-major groups of one pair and the plain path agree
    st.set_tuning(match_kernel=chm.KERNEL_QUERY_MAJOR)
    assert np.array_equal(run_match(st, wl.pairs)[0], ref)
    st.set_tuning(queries_per_item=1024, wg_threads=1024, lds_codes=0, grid_per_cu=2)
    assert np.array_equal(run_match(st, wl.pairs)[0], ref)
    st.set_tuning(match_kernel=chm.KERNEL_BUCKET_MAJOR, bm_min_db_feats=0)
    assert np.array_equal(run_match(st, wl.pairs)[0], ref)
    st.set_tuning(group_queries=1)
    assert np.array_equal(run_match(st, wl.pairs)[0], ref)
    st.set_tuning(wg_threads=256, lds_codes=0)
    assert np.array_equal(run_match(st, wl.pairs, mode=chm.MATCH_PLAIN)[0], ref)
    st.close()


def check_all_pairs_against_digests(wl, name, out, offs):
    """Every pair's GPU matches against the oracle's stored per-pair digest
    (tests/golden/make_digests.py).  On a mismatch the oracle recomputes the
    first few differing pairs, so the failure says whether the GPU or a stale
    golden file is wrong."""
    dig, cnt, pairs, meta = load_golden(name)
    assert np.array_equal(pairs, wl.pairs), "golden pair list of %s does not match the generator" % name
    assert (int(meta["L"]), int(meta["m"]), int(meta["K"])) == (wl.L, wl.m, wl.K)
    got = pair_digests(out, offs)
    bad = np.nonzero(got != dig)[0]
    if len(bad):
        idx = bad[:3].tolist()
        ref = oracle_slices(wl, wl.pairs[idx])
        diffs = ["pair %d %s: %d outputs differ from the oracle, GPU matches %d, stored count %d"
                 % (p, wl.pairs[p].tolist(), int((g != r).sum()), int((g >= 0).sum()), int(cnt[p]))
                 for p, g, r in zip(idx, gpu_slices(out, offs, idx), ref)]
        raise AssertionError("%d of %d pairs differ from the stored oracle digests; %s"
                             % (len(bad), len(dig), "; ".join(diffs)))
    assert np.array_equal(match_counts(out, offs), cnt)


def test_strips_all_pairs():
    """All 5,554 pairs of the strips workload (500 images, 2k-20k features)."""
    wl = synth.config3()
    st = new_store(wl)
    load_all(st, wl.images)
    nd = np.array([x.shape[0] for x in wl.images])
    assert nd.min() < 10175 < nd.max()  # LDS-staged and global-memory db images both occur
    out, _, offs = run_match(st, wl.pairs)
    check_all_pairs_against_digests(wl, "strips", out, offs)
    st.close()


def test_knn_200x40000_all_pairs():
    """All 2,000 pairs of 200 images x 40,000 features, BF16 projection; then
    the FP32 projection gives the same codes and bucket ids."""
    wl = synth.config4()
    st = new_store(wl)
    load_all(st, wl.images)
    out, _, offs = run_match(st, wl.pairs)
    check_all_pairs_against_digests(wl, "knn-200x40000", out, offs)

    # FP32 projection gives the same codes
    st.close()
    del st
    torch.cuda.empty_cache()
    st32 = new_store(wl, chm.PROJ_FP32)
    load_all(st32, wl.images[:2])
    for i in (0, 1):
        g = gpu_arrays(st32, i)
        ref_h = O.hash_image(wl.images[i], wl.W, wl.mu, wl.L, wl.m)
        assert np.array_equal(g["codes"], ref_h.codes) and np.array_equal(g["ids"], ref_h.ids)
    st32.close()


def test_grid_1200x10000_all_pairs():
    """A 12 x 100 grid of 10,000-feature images (the grid workload's image
    size and view-graph shape on 1,200 of its 5,000 images), all pairs in one
    batched plan, every pair against the stored oracle digests.  The full
    5,000-image grid is compared pair by pair in the benchmark's grid job."""
    wl = synth.config5(rows=12, cols=100)
    st = new_store(wl)
    load_all(st, wl.images)
    out, _, offs = run_match(st, wl.pairs)
    check_all_pairs_against_digests(wl, "grid-1200x10000", out, offs)
    st.close()


@pytest.mark.parametrize("slack_caps", [0, 0.03, 0.1, 1])
def test_grid_through_binding_mbr_schedule(slack_caps):
    """slack_caps = 0: the arena holds little beyond the cap, so most block
    rows free the previous row's evictions before copying (after its end);
    small slacks: copies run ahead until the arena is short of room for a
    row's images or its plan; 1: room for a whole second cap, so copies run
    ahead on the copy stream."""
    wl = synth.config5(rows=8, cols=30, n_feats=2000)
    n = len(wl.images)
    cfg = chm.config(L=wl.L, m=wl.m, K=wl.K, ratio=wl.ratio)
    sizes = [chm.image_bytes(cfg, x.shape[0]) + 256 for x in wl.images]
    cap = 40 * sizes[0]  # 40 of 240 images resident at a time
    sched = chm.schedule_mbr(n, wl.pairs, sizes, cap, 16, keep_handle=True)
    assert sched.iterations >= 2 and max(len(s["load"]) for s in sched.steps) > 0
    arena = torch.empty(chm.store_overhead_bytes(cfg) + int((1 + slack_caps) * cap) + (4 << 20),
                        dtype=torch.uint8, device=device())
    st = chm.Store(cfg, wl.W, wl.mu, arena)
    offs = np.zeros(len(wl.pairs) + 1, np.int64)
    offs[1:] = np.cumsum([wl.images[q].shape[0] for q in wl.pairs[:, 0]])
    out = torch.full((int(offs[-1]),), -7, dtype=torch.int32, device=device())
    chm.run_schedule(st, sched, wl.pairs, wl.images, offs, out)
    assert st.stats().images_loaded == sum(len(x["load"]) for x in sched.steps)
    torch.cuda.synchronize()
    chm.schedule_free(sched)
    H = O.hash_workload(wl)
    ref, roffs, _, _ = O.match_pairs(H, wl.pairs, wl.L, wl.m, wl.K, wl.ratio)
    assert np.array_equal(offs, roffs)
    assert np.array_equal(out.cpu().numpy(), ref)
    st.close()


def test_db_images_around_the_lds_stage_limits():
    """Db images on both sides of each LDS layout limit, in one persistent
    launch and per pair: the last size whose bucket offsets are staged with
    the codes, sizes whose items shrink so their sort order fits above the
    stage, the largest size whose codes fit at all (its items run unsorted)
    and the next size up (codes from HBM, in the same launch), with small db
    images between them so work-groups re-stage, every output against the
    oracle."""
    # Limits of the layout on a CU with 160 KiB of LDS (L = 6, m = 8): the
    # control words and histogram take the top 1040 bytes; codes take 16 B a
    # point from address 0; offsets (6 x 257 int32, 6176 B) join them when a
    # 4096-query sort order (8192 B) still fits; an item's order takes 2 B a
    # query.  On another LDS size the same images are still valid inputs.
    top = 160 * 1024 - 1040
    offsets_staged = (top - 6176 - 8192) // 16        # 9277
    sorted_1024 = (top - 2 * 1024) // 16              # 10047
    codes = top // 16                                 # 10175
    sizes = [offsets_staged, offsets_staged + 1, 10000, sorted_1024, sorted_1024 + 1, codes, codes + 1,
             2000, 700]
    n = len(sizes)
    centres = np.stack([np.arange(n) * 0.5, np.zeros(n)], 1)
    pairs = np.array([(q, d) for d in range(n) for q in ((d + 1) % n, (d + n - 1) % n)], np.int32)
    wl = synth.track_workload("lds-limits", 77, centres, sizes, pairs, 0.4)
    st = new_store(wl)
    load_all(st, wl.images)
    ref = oracle_slices(wl, wl.pairs)
    st.set_tuning(bm_min_db_feats=0)
    out, _, offs = run_match(st, wl.pairs)  # bucket major for every pair
    for p in range(len(wl.pairs)):
        assert np.array_equal(out[offs[p]:offs[p + 1]], ref[p]), ("bucket major", p, wl.pairs[p])
    st.set_tuning(match_kernel=chm.KERNEL_QUERY_MAJOR)
    for tuning in ((3072, 1024, 1, 1), (2048, 1024, 1, 1), (512, 1024, 1, 1), (1536, 1024, 1, 1)):
        st.set_tuning(*tuning)
        out, _, offs = run_match(st, wl.pairs)
        for p in range(len(wl.pairs)):
            assert np.array_equal(out[offs[p]:offs[p + 1]], ref[p]), (tuning, p, wl.pairs[p])
    st.set_tuning(wg_threads=1024, lds_codes=1)
    out, _, offs = run_match(st, wl.pairs, mode=chm.MATCH_PLAIN)
    for p in range(len(wl.pairs)):
        assert np.array_equal(out[offs[p]:offs[p + 1]], ref[p]), ("plain", p)
    st.close()

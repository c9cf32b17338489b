"""GPU parity of the HIP path with the CPU oracle, through the C-ABI.

Integer work (codes, bucket ids, tables, top-K keys, match indices) must be
bit-identical.  Hashing is checked before any match kernel reads the tables.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_22089_amd import chm, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_helpers import device, gpu_arrays, load_all, new_store, run_match  # noqa: E402


def small_workload(sizes, seed=0, L=6, m=8, K=8, copies=0.5):
    rng = np.random.default_rng(seed)
    base = synth.sift_like(rng, max(sizes) if sizes else 1)
    imgs = []
    for n in sizes:
        k = int(copies * n)
        x = np.concatenate([synth.noisy_copy(rng, base[:k]), synth.sift_like(rng, n - k)])
        imgs.append(x[rng.permutation(n)] if n else x)
    W = synth.projection_weights(42, 128 + L * m)
    wl = synth.Workload(name="small", images=imgs, pairs=np.zeros((0, 2), np.int32), W=W,
                        mu=synth.centring_vector(imgs), L=L, m=m, K=K)
    return wl


def check_hash(store, wl, ids):
    for i in ids:
        g = gpu_arrays(store, i)
        ref = O.hash_image(wl.images[i], wl.W[:128 + store.cfg.num_tables * store.cfg.bucket_bits],
                           wl.mu, store.cfg.num_tables, store.cfg.bucket_bits)
        assert np.array_equal(g["codes"], ref.codes), "codes of image %d" % i
        assert np.array_equal(g["ids"], ref.ids), "bucket ids of image %d" % i
        assert np.array_equal(g["offsets"], ref.offsets), "offsets of image %d" % i
        assert np.array_equal(g["members"], ref.members), "members of image %d" % i
        x = wl.images[i].astype(np.int64)
        assert np.array_equal(g["norms"].astype(np.int64), (x * x).sum(1))


@pytest.mark.parametrize("L,m", [(6, 8), (3, 5)])
def test_hash_parity_table_kernels_at_the_lds_limit(L, m):
    """Bucket tables of a batch whose largest image has 8,192 features (built
    in LDS), then of one with 8,193 (scattered to global memory): both equal
    the oracle's, and so does a later rehash of all three images together."""
    wl = small_workload([8192, 8191, 8193], seed=5 + m)
    st = new_store(wl, L=L, m=m)
    load_all(st, wl.images[:2])
    check_hash(st, wl, [0, 1])
    load_all(st, wl.images, ids=[2])
    check_hash(st, wl, [2])
    st.rehash([0, 1, 2])
    torch.cuda.synchronize()
    check_hash(st, wl, [0, 1, 2])


@pytest.mark.parametrize("precision", [chm.PROJ_BF16, chm.PROJ_FP32])
def test_hash_parity_config1(precision):
    wl = synth.config1()
    st = new_store(wl, precision)
    load_all(st, wl.images)
    check_hash(st, wl, [0, 1])
    assert st.stats().fixups > 0


@pytest.mark.parametrize("sizes", [[0, 1, 2, 31, 32, 33], [63, 64, 65, 1000], [4097, 129]])
def test_hash_parity_ragged(sizes):
    wl = small_workload(sizes, seed=len(sizes))
    st = new_store(wl)
    load_all(st, wl.images)
    check_hash(st, wl, range(len(sizes)))


@pytest.mark.parametrize("L,m", [(1, 0), (3, 5), (8, 8), (6, 1)])
def test_hash_parity_table_shapes(L, m):
    wl = small_workload([700, 300], seed=L * 10 + m, L=L, m=m)
    st = new_store(wl)
    load_all(st, wl.images)
    check_hash(st, wl, [0, 1])


def near_hyperplane(wl, n, rng):
    """Descriptors whose projections on some rows are as close to 0 as integer
    steps allow (|p| far below the fp32 accumulation error bound)."""
    Wf = (wl.W.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    out = []
    for k in range(n):
        x = synth.sift_like(rng, 1)[0].astype(np.int64)
        r = int(rng.integers(0, Wf.shape[0]))
        for _ in range(40):
            p = float(Wf[r] @ (x - wl.mu.astype(np.int64)))
            if abs(p) < 1e-6:
                break
            d = int(np.argmax(np.abs(Wf[r]) * ((x > 0) & (x < 255))))
            step = -int(np.sign(p) * np.sign(Wf[r, d]))
            if abs(Wf[r, d]) > 2 * abs(p):
                # a unit step overshoots; try the smallest useful coefficient instead
                cand = np.nonzero((np.abs(Wf[r]) <= 2 * abs(p)) & (np.abs(Wf[r]) > 0) &
                                  (x > 0) & (x < 255))[0]
                if len(cand) == 0:
                    break
                d = int(cand[np.argmax(np.abs(Wf[r, cand]))])
                step = -int(np.sign(p) * np.sign(Wf[r, d]))
            x[d] = np.clip(x[d] + step, 0, 255)
        out.append(x.astype(np.uint8))
    return np.stack(out)


def test_hash_parity_near_hyperplane_descriptors():
    rng = np.random.default_rng(77)
    wl = small_workload([10], seed=5)
    X = near_hyperplane(wl, 256, rng)
    wl.images = [X, np.stack([wl.mu] * 3)]
    for prec in (chm.PROJ_BF16, chm.PROJ_FP32):
        st = new_store(wl, prec)
        load_all(st, wl.images)
        check_hash(st, wl, [0, 1])
        st.close()


def check_matches(st, wl, pairs, mode, K):
    """Matches and top-K keys of the pairs against the oracle; a batched
    plan is checked with both match kernels (bucket major, then query major)."""
    if mode == chm.MATCH_BATCHED:
        out = None
        kernel = st.tuning_dict()
        for k in (chm.KERNEL_BUCKET_MAJOR, chm.KERNEL_QUERY_MAJOR):
            st.set_tuning(match_kernel=k, bm_min_db_feats=0)
            o = check_matches_once(st, wl, pairs, mode, K)
            assert out is None or np.array_equal(o, out)
            out = o
        st.set_tuning(**kernel)
        return out
    return check_matches_once(st, wl, pairs, mode, K)


def check_matches_once(st, wl, pairs, mode, K):
    out, topk, offs = run_match(st, pairs, mode, want_topk=True)
    H = {}
    for p, (q, d) in enumerate(pairs):
        for i in (q, d):
            if i not in H:
                H[i] = O.hash_image(wl.images[i], wl.W[:128 + st.cfg.num_tables * st.cfg.bucket_bits],
                                    wl.mu, st.cfg.num_tables, st.cfg.bucket_bits)
        ro, rt, _ = O.match_pair(H[q], H[d], st.cfg.num_tables, st.cfg.bucket_bits, K,
                                 wl.ratio, want_topk=True,
                                 accept_single=bool(st.cfg.flags & chm.ACCEPT_SINGLE),
                                 whole_last_bucket=bool(st.cfg.flags & chm.WHOLE_LAST_BUCKET))
        a, b = offs[p], offs[p + 1]
        assert np.array_equal(topk[a:b], rt), "top-K keys of pair %d (%d -> %d)" % (p, q, d)
        assert np.array_equal(out[a:b], ro), "matches of pair %d (%d -> %d)" % (p, q, d)
    return out


@pytest.mark.parametrize("mode", [chm.MATCH_PLAIN, chm.MATCH_BATCHED])
def test_match_parity_config1(mode):
    wl = synth.config1()
    st = new_store(wl)
    load_all(st, wl.images)
    out = check_matches(st, wl, [(0, 1), (1, 0), (0, 0)], mode, 2)
    gt = {int(a): int(b) for a, b in wl.gt}
    assert np.mean([out[a] == b for a, b in gt.items()]) > 0.9


@pytest.mark.parametrize("mode", [chm.MATCH_PLAIN, chm.MATCH_BATCHED])
def test_match_parity_accept_single(mode):
    """The d2 = infinity reading: a query with exactly one candidate takes it.
    Small db images and two tables make one-candidate queries common."""
    wl = small_workload([600, 40, 25, 1], seed=31)
    st = new_store(wl, L=2, accept_single=True)
    load_all(st, wl.images)
    out = check_matches(st, wl, [(0, 1), (0, 2), (0, 3), (1, 0)], mode, wl.K)
    assert (out >= 0).any()
    st.close()


@pytest.mark.parametrize("mode,L,m,K,lds", [(chm.MATCH_PLAIN, 3, 5, 4, 1), (chm.MATCH_BATCHED, 3, 5, 4, 1),
                                            (chm.MATCH_BATCHED, 6, 8, 8, 0), (chm.MATCH_BATCHED, 2, 3, 2, 1)])
def test_match_parity_whole_last_bucket(mode, L, m, K, lds):
    """The other reading of step (3): every candidate as close in Hamming
    distance as the K-th is re-ranked.  Few bucket bits make wide tie
    classes; lds 0 reads the codes from HBM."""
    wl = small_workload([700, 500, 300, 40], seed=41, L=L, m=m, K=K)
    st = new_store(wl, whole_last_bucket=True)
    st.set_tuning(lds_codes=lds)
    load_all(st, wl.images)
    out = check_matches(st, wl, [(0, 1), (1, 0), (2, 3), (0, 0)], mode, K)
    assert (out >= 0).any()
    st.close()


@pytest.mark.parametrize("mode", [chm.MATCH_PLAIN, chm.MATCH_BATCHED])
def test_match_parity_arena_low_dword_above_2gib(mode):
    """Regression: every device address of the store has its low 32 bits in
    [2^31, 2^32), so a pointer rebuilt from two 32-bit halves in SGPRs must not
    sign-extend the low half (it once did, and the match kernel faulted)."""
    wl = synth.config1()
    cfg = chm.config(L=wl.L, m=wl.m, K=wl.K, ratio=wl.ratio)
    need = chm.store_overhead_bytes(cfg) + sum(chm.image_bytes(cfg, x.shape[0]) + 256
                                               for x in wl.images) + (16 << 20)
    assert need < (1 << 30)
    big = torch.empty(need + (1 << 32), dtype=torch.uint8, device=device())
    base = big.data_ptr()
    target = ((base >> 32) << 32) + (3 << 30)  # low dword 0xC0000000
    if target < base:
        target += 1 << 32
    arena = big[target - base:target - base + need]
    assert arena.data_ptr() & 0xFFFFFFFF >= 0xC0000000
    st = chm.Store(cfg, wl.W, wl.mu, arena)
    load_all(st, wl.images)
    check_matches(st, wl, [(0, 1), (1, 0)], mode, wl.K)
    st.close()


@pytest.mark.parametrize("ratio", [(99, 100), (1, 1), (1, 2)])
@pytest.mark.parametrize("mode", [chm.MATCH_PLAIN, chm.MATCH_BATCHED])
def test_match_parity_ratio(mode, ratio):
    """Ratio thresholds near and at 1 stress the exact test
    den^2 * d1 < num^2 * d2 in 64-bit integers (at 1/1 a query passes only
    when its nearest candidate is strictly closer than the second)."""
    wl = small_workload([1200, 900, 300], seed=7 + ratio[0], copies=0.3)
    wl.ratio = ratio
    st = new_store(wl)
    load_all(st, wl.images)
    out = check_matches(st, wl, [(0, 1), (1, 0), (2, 0), (1, 1)], mode, wl.K)
    assert (out >= 0).any()
    st.close()


@pytest.mark.parametrize("K", [1, 2, 3, 8, 16, 32])
def test_match_parity_k(K):
    wl = small_workload([900, 700, 0, 1], seed=K)
    st = new_store(wl, K=K)
    load_all(st, wl.images)
    pairs = [(0, 1), (1, 0), (1, 1), (0, 2), (2, 0), (3, 0), (0, 3)]
    check_matches(st, wl, pairs, chm.MATCH_BATCHED, K)
    check_matches(st, wl, pairs, chm.MATCH_PLAIN, K)


@pytest.mark.parametrize("L,m", [(1, 0), (3, 5), (8, 8)])
def test_match_parity_table_shapes(L, m):
    wl = small_workload([600, 500], seed=3 + L, L=L, m=m)
    st = new_store(wl, K=8)
    load_all(st, wl.images)
    check_matches(st, wl, [(0, 1), (1, 0)], chm.MATCH_BATCHED, 8)


def test_match_parity_lds_and_global_paths():
    # one db image above the LDS stage capacity, others below; ragged query counts
    wl = small_workload([12000, 3001, 65, 8000], seed=9, copies=0.3)
    st = new_store(wl, K=8)
    load_all(st, wl.images)
    pairs = [(1, 0), (2, 0), (0, 1), (3, 1), (1, 3), (2, 3)]
    ref = check_matches(st, wl, pairs, chm.MATCH_BATCHED, 8)
    for tun in (dict(match_kernel=chm.KERNEL_QUERY_MAJOR), dict(lds_codes=0), dict(wg_threads=256),
                dict(queries_per_item=64), dict(queries_per_item=4096, grid_per_cu=1),
                dict(match_kernel=chm.KERNEL_BUCKET_MAJOR, group_queries=1, bm_min_db_feats=0),
                dict(bm_min_db_feats=10176)):
        st.set_tuning(**tun)
        for mode in (chm.MATCH_BATCHED, chm.MATCH_PLAIN):
            out, _, _ = run_match(st, pairs, mode)
            assert np.array_equal(out, ref), "tuning %s mode %d" % (tun, mode)


@pytest.mark.parametrize("K", [2, 8])
def test_bucket_major_rounds(K):
    """Bucket-major plans whose kept lists do not fit the arena at once run
    in several rounds that reuse one state block; groups of several pairs
    share a db image (and empty images and self pairs occur).  Every round's
    output equals the oracle and the query-major kernel."""
    wl = small_workload([3000, 2500, 3100, 0, 2900, 1, 2700], seed=17, copies=0.4)
    pairs = [(q, d) for d in range(7) for q in range(7) if q != d and abs(q - d) <= 3] + [(4, 4)]
    st = new_store(wl, K=K, extra=1200 << 10)
    load_all(st, wl.images)
    ref = check_matches(st, wl, pairs, chm.MATCH_BATCHED, K)
    for gq in (1, 6000, 1 << 20):
        st.set_tuning(match_kernel=chm.KERNEL_BUCKET_MAJOR, group_queries=gq, bm_min_db_feats=0)
        assert np.array_equal(run_match(st, pairs)[0], ref), gq
    st.close()


def test_match_duplicates_and_degenerate():
    rng = np.random.default_rng(1)
    wl = small_workload([50], seed=1)
    same = np.repeat(synth.sift_like(rng, 1), 40, axis=0)
    wl.images = [same, np.concatenate([same[:5], synth.sift_like(rng, 30)]), np.stack([wl.mu] * 4)]
    wl.mu = synth.centring_vector(wl.images)
    st = new_store(wl, K=8)
    load_all(st, wl.images)
    check_matches(st, wl, [(0, 1), (1, 0), (0, 0), (2, 2), (2, 1), (1, 2)], chm.MATCH_BATCHED, 8)


def test_batched_replay_is_deterministic():
    wl = small_workload([2000, 2500, 1500], seed=4)
    st = new_store(wl, K=8)
    load_all(st, wl.images)
    pairs = [(0, 1), (1, 2), (2, 0), (1, 0)]
    a, _, _ = run_match(st, pairs, chm.MATCH_BATCHED, repeats=3)
    b, _, _ = run_match(st, pairs, chm.MATCH_PLAIN)
    assert np.array_equal(a, b)


def test_hash_parity_when_fixup_list_overflows():
    """fixup_rel = 0.5 marks most projections borderline: the per-tile list
    overflows and the batch is rebuilt from exact values; bits still match."""
    wl = small_workload([300, 77], seed=21)
    for prec in (chm.PROJ_BF16, chm.PROJ_FP32):
        st = new_store(wl, prec, fixup_rel=0.5)
        load_all(st, wl.images)
        check_hash(st, wl, [0, 1])
        assert st.stats().fixups >= 377 * 176
        st.close()


def test_match_parity_stored_golden_pair():
    """The HIP path reproduces the stored oracle matches of the small golden
    pair (written by tests/golden/make_golden.py)."""
    import os
    from tests.golden import make_golden as G
    A, B, W, mu = G.match_case()
    path = os.path.join(os.path.dirname(__file__), "golden", "match_pair_300.txt")
    expect = np.array([int(v) for l in open(path) if not l.startswith("#") for v in l.split()])
    wl = synth.Workload(name="golden", images=[A, B], pairs=np.array([[0, 1]], np.int32), W=W, mu=mu)
    for mode in (chm.MATCH_PLAIN, chm.MATCH_BATCHED):
        st = new_store(wl)
        load_all(st, wl.images)
        out, _, _ = run_match(st, [(0, 1)], mode)
        assert np.array_equal(out, expect)
        st.close()


@pytest.mark.parametrize("seed", range(12))
def test_random_configurations(seed):
    """Seeded random configurations (tables, bucket bits, K, ratio, both
    flags, image sizes including empty and one-feature images, self pairs),
    both match kernels and both modes, against the oracle's matches and
    top-K keys."""
    rng = np.random.default_rng(1000 + seed)
    L = int(rng.integers(1, 9))
    m = int(rng.integers(0, 9))
    K = int(rng.choice([1, 2, 3, 5, 8, 13, 16, 32]))
    num = int(rng.integers(1, 100))
    den = int(rng.integers(num, 101))
    sizes = [int(rng.choice([0, 1, 2, 63, 64, 65, 300, 1000, 2500])) for _ in range(4)]
    wl = small_workload(sizes, seed=seed, L=L, m=m, K=K, copies=float(rng.uniform(0.1, 0.6)))
    wl.ratio = (num, den)
    accept = bool(rng.integers(0, 2))
    whole = bool(rng.integers(0, 2))
    st = new_store(wl, accept_single=accept, whole_last_bucket=whole)
    if rng.integers(0, 2):
        st.set_tuning(queries_per_item=int(rng.choice([64, 256, 1024, 3072])),
                      wg_threads=int(rng.choice([256, 1024])), lds_codes=int(rng.integers(0, 2)),
                      group_queries=int(rng.choice([1, 2000, 98304])))
    load_all(st, wl.images)
    pairs = [(int(q), int(d)) for q, d in rng.integers(0, 4, size=(6, 2))]
    for mode in (chm.MATCH_BATCHED, chm.MATCH_PLAIN):
        check_matches(st, wl, pairs, mode, K)
    st.close()

"""The autotuner on a small mixed workload (db images below, around and
above the query-major LDS code stage): it times every candidate tuning,
checks that each returns the same matches, applies the fastest, and a
second call is answered from its cache.  The tuned plan's matches equal the
oracle's on every pair."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_22089_amd import autotune, chm, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from tests.gpu_helpers import load_all, new_store, run_match  # noqa: E402


def test_autotune_mixed_workload(tmp_path):
    sizes = [12000, 3000, 9500, 500, 10500, 6000, 20000]
    n = len(sizes)
    centres = np.stack([np.arange(n) * 0.5, np.zeros(n)], 1)
    pairs = np.array([(q, d) for d in range(n) for q in range(n) if q != d and abs(q - d) <= 2], np.int32)
    wl = synth.track_workload("autotune-mix", 91, centres, sizes, pairs, 0.3)
    st = new_store(wl, extra=256 << 20)
    load_all(st, wl.images)
    cache = str(tmp_path / "autotune.json")
    report = {}
    best = autotune.tune(st, wl.pairs, reps=1, cache=cache, report=report)
    assert not report["cached"] and report["timed"] > 10
    assert report["best_ms"] <= report["default_ms"]
    assert st.tuning_dict() == best
    H = O.hash_workload(wl)
    ref, roffs, _, _ = O.match_pairs(H, wl.pairs, wl.L, wl.m, wl.K, wl.ratio)
    out, _, offs = run_match(st, wl.pairs)
    assert np.array_equal(offs, roffs) and np.array_equal(out, ref)
    # the cache answers a second call with the same tuning
    st.set_tuning(match_kernel=chm.KERNEL_QUERY_MAJOR, queries_per_item=512)
    report2 = {}
    again = autotune.tune(st, wl.pairs, reps=1, cache=cache, report=report2)
    assert report2["cached"] and again == best
    st.close()

"""The CHM_E_HIP error path, forced from the host with the library's test
hook (the n-th checked HIP call fails without being made): the failing
entry point returns CHM_E_HIP with a message, and the store and plan work
normally on the next call (codes, tables and matches equal the oracle)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_22089_amd import chm, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from tests.gpu_helpers import device, gpu_arrays, load_all, new_store  # noqa: E402

CHM_E_HIP = -5


def test_hip_failure_surfaces_and_the_store_recovers():
    wl = synth.config1(n=1200, planted=500)
    st = new_store(wl)
    load_all(st, wl.images)
    chm.debug_fail_hip(1)
    with pytest.raises(chm.ChmError) as ei:
        st.rehash([0, 1])
    assert ei.value.status == CHM_E_HIP and "failed" in str(ei.value)
    st.rehash([0, 1])
    torch.cuda.synchronize()
    H = O.hash_workload(wl)
    for i in (0, 1):
        g = gpu_arrays(st, i)
        assert np.array_equal(g["codes"], H[i].codes) and np.array_equal(g["members"], H[i].members)

    pairs = np.array([[0, 1], [1, 0]], np.int32)
    offs = chm.out_offsets(st, pairs)
    ref, roffs, _, _ = O.match_pairs(H, pairs, wl.L, wl.m, wl.K, wl.ratio)
    for mode in (chm.MATCH_BATCHED, chm.MATCH_PLAIN):
        out = torch.full((int(offs[-1]),), -7, dtype=torch.int32, device=device())
        plan = chm.Plan(st, pairs, offs, out, None, mode)
        chm.debug_fail_hip(1)
        with pytest.raises(chm.ChmError) as ei:
            plan.execute()
        assert ei.value.status == CHM_E_HIP
        plan.execute()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref)
        plan.close()

    chm.debug_fail_hip(1)
    with pytest.raises(chm.ChmError) as ei:
        st.stats()
    assert ei.value.status == CHM_E_HIP
    assert st.stats().images_loaded == 2
    # a pending failure can be cancelled
    chm.debug_fail_hip(3)
    chm.debug_fail_hip(0)
    st.rehash([0])
    st.close()

"""The brute force with the library's own fixed workspace
(chm_bruteforce_noalloc) against the entry point with a caller workspace
(chm_bruteforce), through the C-ABI: two calls in a row, the second on a
smaller input, so the shared workspace keeps the first call's contents."""
import numpy as np
import pytest

from paper_2505_22089_amd import chm, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from tests.gpu_helpers import device  # noqa: E402


def inputs(nq, nd, seed):
    rng = np.random.default_rng(seed)
    A = synth.sift_like(rng, nq)
    B = np.concatenate([synth.noisy_copy(rng, A[: min(nq, nd) // 2]), synth.sift_like(rng, nd - min(nq, nd) // 2)])
    return torch.from_numpy(A).to(device()), torch.from_numpy(B).to(device())


def with_caller_workspace(q, d, ratio):
    out = torch.full((q.shape[0],), -7, dtype=torch.int32, device=device())
    work = torch.empty(chm.bruteforce_work_bytes(q.shape[0], d.shape[0]), dtype=torch.uint8, device=device())
    chm.bruteforce(q, d, out, work, ratio)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def with_library_workspace(q, d, ratio):
    out = torch.full((q.shape[0],), -7, dtype=torch.int32, device=device())
    chm.bruteforce_noalloc(q, d, out, ratio)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_bruteforce_equals_workspace_entry_point():
    big = inputs(5000, 9000, 1)
    small = inputs(700, 1300, 2)
    for (q, d), ratio in ((big, (4, 5)), (small, (99, 100))):
        ref = with_caller_workspace(q, d, ratio)
        got = with_library_workspace(q, d, ratio)
        assert np.array_equal(got, ref)
        assert (got >= 0).any()


def test_noalloc_bruteforce_rejects_sizes_beyond_its_workspace():
    need = chm.bruteforce_work_bytes(3_000_000, 300)
    assert need > 32 << 20
    q = torch.empty((3_000_000, 128), dtype=torch.uint8, device=device())
    d = torch.zeros((300, 128), dtype=torch.uint8, device=device())
    out = torch.empty((3_000_000,), dtype=torch.int32, device=device())
    with pytest.raises(chm.ChmError, match="workspace"):
        chm.bruteforce_noalloc(q, d, out)

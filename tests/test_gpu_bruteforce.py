"""GPU parity of the int8-MFMA exhaustive matcher with the oracle's brute force."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_22089_amd import chm, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from tests.gpu_helpers import device, load_all, new_store, run_match  # noqa: E402


def gpu_bruteforce(Xq, Xd, ratio=(4, 5)):
    q = torch.from_numpy(np.ascontiguousarray(Xq)).to(device()) if len(Xq) else \
        torch.empty((0, 128), dtype=torch.uint8, device=device())
    d = torch.from_numpy(np.ascontiguousarray(Xd)).to(device()) if len(Xd) else \
        torch.empty((0, 128), dtype=torch.uint8, device=device())
    out = torch.full((max(1, len(Xq)),), -7, dtype=torch.int32, device=device())
    work = torch.empty(chm.bruteforce_work_bytes(len(Xq), len(Xd)), dtype=torch.uint8, device=device())
    chm.bruteforce(q, d, out, work, ratio)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:len(Xq)]


@pytest.mark.parametrize("nq,nd", [(0, 5), (1, 0), (1, 1), (1, 2), (100, 127), (129, 128),
                                   (129, 129), (50, 255), (257, 256), (70, 257), (513, 511),
                                   (300, 1000), (33, 4097)])
def test_bruteforce_shapes(nq, nd):
    rng = np.random.default_rng(nq * 7 + nd)
    A = synth.sift_like(rng, nq)
    B = np.concatenate([synth.noisy_copy(rng, A[: min(nq, nd) // 2]),
                        synth.sift_like(rng, nd - min(nq, nd) // 2)]) if nd else A[:0]
    for ratio in [(4, 5), (99, 100)]:
        assert np.array_equal(gpu_bruteforce(A, B, ratio), O.bruteforce(A, B, ratio))


def test_bruteforce_ties_and_extremes():
    rng = np.random.default_rng(3)
    x = synth.sift_like(rng, 4)
    D = np.concatenate([np.repeat(x[:1], 3, axis=0), synth.sift_like(rng, 200),
                        np.full((2, 128), 255, np.uint8), np.zeros((2, 128), np.uint8)])
    Q = np.concatenate([x, np.full((1, 128), 255, np.uint8), np.zeros((1, 128), np.uint8)])
    assert np.array_equal(gpu_bruteforce(Q, D), O.bruteforce(Q, D))


def test_bruteforce_mid_size():
    rng = np.random.default_rng(11)
    A = synth.sift_like(rng, 3000)
    B = np.concatenate([synth.noisy_copy(rng, A[:1500]), synth.sift_like(rng, 2500)])
    B = B[rng.permutation(len(B))]
    assert np.array_equal(gpu_bruteforce(A, B), O.bruteforce(A, B))


def test_bruteforce_full_size_sampled_rows():
    """40,000 x 40,000 (the dense reference size): sampled rows against the oracle."""
    rng = np.random.default_rng(12)
    A = synth.sift_like(rng, 40000)
    B = np.concatenate([synth.noisy_copy(rng, A[:20000]), synth.sift_like(rng, 20000)])
    B = B[rng.permutation(len(B))]
    out = gpu_bruteforce(A, B)
    rows = np.sort(rng.choice(40000, 300, replace=False))
    assert np.array_equal(out[rows], O.bruteforce(A[rows], B))


def test_single_bucket_cascade_equals_bruteforce_on_gpu():
    rng = np.random.default_rng(5)
    A = synth.sift_like(rng, 400)
    B = np.concatenate([synth.noisy_copy(rng, A[:200]), synth.sift_like(rng, 200)])
    W = synth.projection_weights(42, 128)
    # with one table of one bucket and K = 32 >= the db's 30 points, cascade
    # hashing re-ranks every db point: exhaustive 2-NN
    small = synth.Workload(name="t2", images=[A[:30], B[:30]], pairs=np.array([[0, 1]], np.int32), W=W,
                           mu=synth.centring_vector([A, B]), L=1, m=0, K=32)
    st2 = new_store(small)
    load_all(st2, small.images)
    out, _, _ = run_match(st2, [(0, 1)])
    assert np.array_equal(out, gpu_bruteforce(A[:30], B[:30]))
    assert np.array_equal(out, O.bruteforce(A[:30], B[:30]))

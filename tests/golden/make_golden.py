"""Writes the stored expected values under tests/golden/ by calling only
the oracle (the matcher of Sec. 2.3.1 and the SAO constraint of Sec. 2.3.3)
on small seeded inputs from the generator.  Run from the repository root:
python tests/golden/make_golden.py"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from oracle import sao as S  # noqa: E402
from paper_2505_22089_amd import synth  # noqa: E402


def match_case():
    """One directed pair: 300 query descriptors, 300 db descriptors of which
    150 are noisy copies; L = 6, m = 8, K = 8, t_r = 4/5."""
    rng = np.random.default_rng(2024)
    A = synth.sift_like(rng, 300)
    B = np.concatenate([synth.noisy_copy(rng, A[:150]), synth.sift_like(rng, 150)])
    B = B[rng.permutation(300)]
    W = synth.projection_weights(42, 176)
    mu = synth.centring_vector([A, B])
    return A, B, W, mu


def sao_case():
    """60 matches: 45 follow a quarter turn plus a shift, 15 are random."""
    rng = np.random.default_rng(7)
    kq = rng.integers(0, 5000, size=(60, 2)).astype(np.int32)
    kd = np.stack([-kq[:, 1] + 300, kq[:, 0] - 40], axis=1).astype(np.int32)
    match = np.arange(60, dtype=np.int32)
    match[45:] = rng.integers(0, 60, 15)
    return kq, kd, match


def main():
    A, B, W, mu = match_case()
    hq, hd = O.hash_image(A, W, mu, 6, 8), O.hash_image(B, W, mu, 6, 8)
    out, _, _ = O.match_pair(hq, hd, 6, 8, 8, (4, 5))
    with open(os.path.join(HERE, "match_pair_300.txt"), "w") as f:
        f.write("# oracle matches (db row or -1) of tests/golden/make_golden.py:match_case, one per query row\n")
        f.write(" ".join(str(int(v)) for v in out) + "\n")
    kq, kd, match = sao_case()
    ced, filt = S.sao_pair(kq, kd, match, 6, (1, 2))
    with open(os.path.join(HERE, "sao_60.txt"), "w") as f:
        f.write("# oracle SAO of tests/golden/make_golden.py:sao_case (N = 6, CED/N <= 1/2): CED, then kept\n")
        f.write(" ".join(str(int(v)) for v in ced) + "\n")
        f.write(" ".join(str(int(v)) for v in filt) + "\n")


if __name__ == "__main__":
    main()

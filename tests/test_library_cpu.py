"""CPU-side checks of libchm: it loads, exports every symbol include/chm.h
declares, validates arguments on the host, and its C++ MBR/GPS scheduler
produces exactly the schedules of the Python oracle (host logic only; no
device call is made here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import mbr
from paper_2505_22089_amd import chm, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "chm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = chm.lib()
    declared = header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(chm.EXPORTS) == declared
    nm = subprocess.run(["nm", "-D", "--defined-only", chm.LIB_PATH], capture_output=True, text=True)
    exported = set(l.split()[-1] for l in nm.stdout.splitlines() if " T " in l)
    assert set(declared) <= exported


def test_library_targets_gfx950_only():
    blob = open(chm.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}


def test_config_defaults_and_validation():
    c = chm.config()
    assert (c.num_tables, c.bucket_bits, c.top_k, c.ratio_num, c.ratio_den) == (6, 8, 8, 4, 5)
    assert c.abi_version == chm.ABI_VERSION and chm.lib().chm_abi_version() == 2
    assert chm.image_bytes(c, 0) > 0
    b8000 = chm.image_bytes(c, 8000)
    assert b8000 >= 8000 * (128 + 16 + 6 + 4 + 12)   # desc, code, L ids, norm, L u16 members
    for bad in (dict(L=0), dict(L=9), dict(m=9), dict(K=0), dict(K=33), dict(ratio=(5, 4)),
                dict(ratio=(0, 5)), dict(fixup_rel=1e-9), dict(precision=7)):
        with pytest.raises(chm.ChmError) as e:
            chm.image_bytes(chm.config(**bad), 10)
        assert e.value.status == -1
    with pytest.raises(chm.ChmError):
        chm.image_bytes(c, chm.MAX_FEATS + 1)


def check_same_schedule(n, pairs, sizes, cap, blk):
    ref = mbr.schedule_mbr(n, pairs, sizes, cap, blk)
    got = chm.schedule_mbr(n, pairs, sizes, cap, blk)
    assert got.iterations == ref.iterations
    assert got.dims == ref.dims and got.bandwidths == ref.bandwidths
    assert got.fallback_pairs == ref.fallback_pairs
    assert len(got.steps) == len(ref.steps)
    for a, b in zip(got.steps, ref.steps):
        assert a["evict"] == b.evict and a["load"] == b.load and a["pairs"] == b.pairs


@pytest.mark.parametrize("seed", range(8))
def test_scheduler_matches_oracle_random(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(3, 70))
    pairs = np.array([(a, b) for a in range(n) for b in range(n)
                      if rng.random() < 0.08], dtype=np.int32).reshape(-1, 2)
    sizes = rng.integers(1, 9, size=n)
    cap = int(sizes.max() * 2 + rng.integers(0, 40))
    check_same_schedule(n, pairs, sizes.tolist(), cap, int(rng.integers(1, 9)))


def test_scheduler_matches_oracle_on_the_5000_image_grid():
    rng = np.random.default_rng(1005)
    pairs = np.concatenate([synth.band_grid_pairs(50, 100, 1, 3), synth.cross_links(rng, 50, 100)])
    sizes = [1_700_000] * 5000
    check_same_schedule(5000, pairs, sizes, 2 << 30, 400)


def test_scheduler_matches_oracle_tight_cap():
    rng = np.random.default_rng(7)
    pairs = np.array([(a, b) for a in range(60) for b in range(60) if a != b and rng.random() < 0.06],
                     dtype=np.int32)
    check_same_schedule(60, pairs, [1] * 60, 5, 2)


def test_gps_order_matches_oracle():
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = 50
        edges = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(80, 2))]
        nodes = sorted(set(rng.integers(0, n, size=40).tolist()) | {a for e in edges for a in e})
        adj = mbr.symmetric_adjacency(n, edges)
        assert chm.gps_order(n, np.array(edges), nodes) == mbr.gps_order(adj, nodes)


def test_scheduler_errors():
    with pytest.raises(chm.ChmError) as e:
        chm.schedule_mbr(2, np.array([[0, 1]]), [3, 3], 5, 1)
    assert e.value.status == -3
    with pytest.raises(chm.ChmError):
        chm.schedule_mbr(2, np.array([[0, 2]]), [1, 1], 5, 1)
    s = chm.schedule_mbr(3, np.zeros((0, 2), np.int32), [1, 1, 1], 4, 1)
    assert s.steps == [] and s.iterations == 0

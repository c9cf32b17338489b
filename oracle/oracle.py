"""ctypes wrapper over the plain C oracle (``chm_oracle.c``).

Test infrastructure only; see the header of ``chm_oracle.c`` for what each
step computes and which section of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

DIM = 128
CODE_BITS = 128
NO_KEY = 0xFFFFFFFF


class _Image(C.Structure):
    _fields_ = [("desc", C.c_void_p), ("codes", C.c_void_p), ("ids", C.c_void_p),
                ("offsets", C.c_void_p), ("members", C.c_void_p), ("n", C.c_int64)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("CHM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.orc_project.argtypes = [vp, i64, vp, i32, vp, vp]
        L.orc_hash.argtypes = [vp, i64, vp, vp, i32, i32, vp, vp]
        L.orc_tables.argtypes = [vp, i64, i32, i32, vp, vp]
        L.orc_match_pair.argtypes = [C.POINTER(_Image), C.POINTER(_Image), i32, i32, i32, i32, i32, i32, i32, vp,
                                     vp]
        L.orc_match_pair.restype = i64
        L.orc_match_pairs.argtypes = [C.POINTER(_Image), vp, i64, vp, i32, i32, i32, i32, i32, i32, i32, vp, vp]
        L.orc_match_pairs.restype = i64
        L.orc_bruteforce.argtypes = [vp, i64, vp, i64, i32, i32, vp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.restype = C.c_int
        _LIB = L
    return _LIB


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def project(X: np.ndarray, W: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """Exact fp64 projections p_r(x) = sum_d W[r,d](x_d - mu_d), shape (n, R)."""
    X = np.ascontiguousarray(X, dtype=np.uint8)
    W = np.ascontiguousarray(W, dtype=np.uint16)
    mu = np.ascontiguousarray(mu, dtype=np.uint8)
    n, R = X.shape[0], W.shape[0]
    P = np.zeros((n, R), dtype=np.float64)
    lib().orc_project(_p(X), n, _p(W), R, _p(mu), _p(P))
    return P


@dataclass
class Hashed:
    desc: np.ndarray      # (n, 128) uint8
    codes: np.ndarray     # (n, 4) uint32
    ids: np.ndarray       # (n, L) uint8
    offsets: np.ndarray   # (L, 2^m + 1) int32
    members: np.ndarray   # (L, n) int32

    @property
    def n(self) -> int:
        return self.desc.shape[0]

    def as_struct(self) -> _Image:
        return _Image(self.desc.ctypes.data, self.codes.ctypes.data, self.ids.ctypes.data,
                      self.offsets.ctypes.data, self.members.ctypes.data, self.n)


def hash_codes(X: np.ndarray, W: np.ndarray, mu: np.ndarray, L: int, m: int):
    """(codes (n,4) uint32, ids (n,L) uint8) of one image."""
    if not (1 <= L <= 8 and 0 <= m <= 8):
        raise ValueError("L must be 1..8 and m 0..8")
    X = np.ascontiguousarray(X, dtype=np.uint8)
    W = np.ascontiguousarray(W, dtype=np.uint16)
    if W.shape != (CODE_BITS + L * m, DIM):
        raise ValueError("W must be (128 + L*m) x 128")
    mu = np.ascontiguousarray(mu, dtype=np.uint8)
    n = X.shape[0]
    codes = np.zeros((n, 4), dtype=np.uint32)
    ids = np.zeros((n, L), dtype=np.uint8)
    lib().orc_hash(_p(X), n, _p(W), _p(mu), L, m, _p(codes), _p(ids))
    return codes, ids


def tables(ids: np.ndarray, m: int):
    """(offsets (L, 2^m+1) int32, members (L, n) int32) bucket lookup tables."""
    ids = np.ascontiguousarray(ids, dtype=np.uint8)
    n, L = ids.shape
    offsets = np.zeros((L, (1 << m) + 1), dtype=np.int32)
    members = np.zeros((L, n), dtype=np.int32)
    lib().orc_tables(_p(ids), n, L, m, _p(offsets), _p(members))
    return offsets, members


def hash_image(X: np.ndarray, W: np.ndarray, mu: np.ndarray, L: int, m: int) -> Hashed:
    codes, ids = hash_codes(X, W, mu, L, m)
    offsets, members = tables(ids, m)
    return Hashed(np.ascontiguousarray(X, dtype=np.uint8), codes, ids, offsets, members)


def match_pair(q: Hashed, d: Hashed, L: int, m: int, K: int, ratio=(4, 5),
               want_topk: bool = False, accept_single: bool = False, whole_last_bucket: bool = False):
    """(matches (nq,) int32, topk keys (nq, K) uint32 or None, candidate count)."""
    out = np.zeros(q.n, dtype=np.int32)
    topk = np.zeros((q.n, K), dtype=np.uint32) if want_topk else None
    sq, sd = q.as_struct(), d.as_struct()
    nc = lib().orc_match_pair(C.byref(sq), C.byref(sd), L, m, K, ratio[0], ratio[1], int(accept_single),
                              int(whole_last_bucket), _p(out),
                              _p(topk) if want_topk else None)
    return out, topk, int(nc)


def match_pairs(images: Sequence[Hashed], pairs: np.ndarray, L: int, m: int, K: int,
                ratio=(4, 5), want_topk: bool = False, accept_single: bool = False,
                whole_last_bucket: bool = False):
    """All directed pairs; returns (out concatenated, out_offsets (P+1), topk, candidates)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    P = pairs.shape[0]
    offs = np.zeros(P + 1, dtype=np.int64)
    if P:
        offs[1:] = np.cumsum([images[q].n for q in pairs[:, 0]])
    out = np.zeros(int(offs[-1]), dtype=np.int32)
    topk = np.zeros((int(offs[-1]), K), dtype=np.uint32) if want_topk else None
    arr = (_Image * max(1, len(images)))(
        *[im.as_struct() if im is not None else _Image(0, 0, 0, 0, 0, 0) for im in images])
    nc = lib().orc_match_pairs(arr, _p(pairs), P, _p(offs), L, m, K, ratio[0], ratio[1], int(accept_single),
                               int(whole_last_bucket),
                               _p(out), _p(topk) if want_topk else None)
    return out, offs, topk, int(nc)


def bruteforce(Xq: np.ndarray, Xd: np.ndarray, ratio=(4, 5)) -> np.ndarray:
    """Exhaustive 2-NN with the ratio test (squared integer distances)."""
    Xq = np.ascontiguousarray(Xq, dtype=np.uint8)
    Xd = np.ascontiguousarray(Xd, dtype=np.uint8)
    out = np.zeros(Xq.shape[0], dtype=np.int32)
    lib().orc_bruteforce(_p(Xq), Xq.shape[0], _p(Xd), Xd.shape[0], ratio[0], ratio[1], _p(out))
    return out


def hash_workload(wl, images: Optional[List[int]] = None) -> List[Optional[Hashed]]:
    """Hash every image of a workload (or only the listed ones)."""
    idx = range(len(wl.images)) if images is None else images
    res: List[Optional[Hashed]] = [None] * len(wl.images)
    for i in idx:
        res[i] = hash_image(wl.images[i], wl.W, wl.mu, wl.L, wl.m)
    return res

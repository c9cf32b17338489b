"""ctypes binding of libchm.so (include/chm.h).

Argument marshalling only: every step of matching runs in the library's HIP
kernels.  Device buffers are torch CUDA tensors (ROCm), streams are torch
streams.  The library must have been built (``build.py``); importing this
module does not load it, the first call does and raises ``ChmError`` if the
library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchm.so")

ABI_VERSION = 2
ACCEPT_SINGLE = 1
WHOLE_LAST_BUCKET = 2
PROJ_BF16, PROJ_FP32 = 0, 1
MATCH_PLAIN, MATCH_BATCHED = 0, 1
MAX_FEATS = 65535

_STATUS = {0: "CHM_OK", -1: "CHM_E_INVALID_ARG", -2: "CHM_E_UNSUPPORTED", -3: "CHM_E_CAPACITY",
           -4: "CHM_E_NOT_RESIDENT", -5: "CHM_E_HIP", -6: "CHM_E_INTERNAL"}


class ChmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("num_tables", C.c_int32), ("bucket_bits", C.c_int32),
                ("top_k", C.c_int32), ("ratio_num", C.c_int32), ("ratio_den", C.c_int32),
                ("proj_precision", C.c_int32), ("flags", C.c_int32), ("fixup_rel", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("h2d_bytes", C.c_uint64), ("d2d_bytes", C.c_uint64), ("resident_bytes", C.c_uint64),
                ("resident_peak", C.c_uint64), ("fixups", C.c_uint64), ("images_loaded", C.c_int64),
                ("images_evicted", C.c_int64), ("resident_images", C.c_int32), ("reserved", C.c_int32),
                ("fixup_flips", C.c_uint64)]


class Tuning(C.Structure):
    _fields_ = [("queries_per_item", C.c_int32), ("wg_threads", C.c_int32),
                ("lds_codes", C.c_int32), ("grid_per_cu", C.c_int32),
                ("match_kernel", C.c_int32), ("bm_min_db_feats", C.c_int32), ("group_queries", C.c_int32),
                ("tail_percent", C.c_int32), ("hbm_item_queries", C.c_int32)]


TUNING_FIELDS = [f for f, _ in Tuning._fields_]
KERNEL_QUERY_MAJOR = 0
KERNEL_BUCKET_MAJOR = 1


# every symbol include/chm.h declares
EXPORTS = [
    "chm_config_default", "chm_last_error", "chm_abi_version", "chm_debug_fail_hip", "chm_image_bytes",
    "chm_store_overhead_bytes", "chm_store_create", "chm_store_destroy", "chm_store_load",
    "chm_store_rehash", "chm_store_evict", "chm_store_image_feats", "chm_store_stats",
    "chm_debug_image", "chm_plan_create", "chm_plan_execute", "chm_plan_destroy",
    "chm_match_pairs", "chm_store_get_tuning", "chm_store_set_tuning",
    "chm_bruteforce_work_bytes", "chm_bruteforce", "chm_bruteforce_noalloc", "chm_schedule_mbr", "chm_schedule_from_steps", "chm_schedule_num_steps",
    "chm_schedule_step", "chm_schedule_info", "chm_schedule_free", "chm_gps_order",
    "chm_run_schedule", "chm_sao_filter", "chm_sao_work_bytes", "chm_sao_filter_device",
    "chm_run_schedule_sao", "chm_run_schedule_verify", "chm_ransac_filter", "chm_ransac_work_bytes",
    "chm_ransac_filter_device", "chm_run_schedule_verify_device",
]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ChmError(-6, "libchm.so is not built (run paper_2505_22089_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        P = C.POINTER
        sig = {
            "chm_config_default": (None, [P(Config)]),
            "chm_last_error": (C.c_char_p, []),
            "chm_abi_version": (i32, []),
            "chm_debug_fail_hip": (None, [i32]),
            "chm_image_bytes": (i32, [P(Config), i32, P(u64)]),
            "chm_store_overhead_bytes": (i32, [P(Config), P(u64)]),
            "chm_store_create": (i32, [P(Config), vp, vp, vp, u64, P(vp)]),
            "chm_store_destroy": (None, [vp]),
            "chm_store_load": (i32, [vp, i32, vp, vp, vp, i32, vp]),
            "chm_store_rehash": (i32, [vp, i32, vp, vp]),
            "chm_store_evict": (i32, [vp, i32, vp]),
            "chm_store_image_feats": (i32, [vp, i32, P(i32)]),
            "chm_store_stats": (i32, [vp, P(Stats)]),
            "chm_debug_image": (i32, [vp, i32, vp, vp, vp, vp, vp, vp]),
            "chm_plan_create": (i32, [vp, vp, i32, vp, vp, vp, i32, vp, P(vp)]),
            "chm_plan_execute": (i32, [vp, vp]),
            "chm_plan_destroy": (None, [vp]),
            "chm_match_pairs": (i32, [vp, vp, i32, vp, vp, i32, vp]),
            "chm_store_get_tuning": (i32, [vp, P(Tuning)]),
            "chm_store_set_tuning": (i32, [vp, P(Tuning)]),
            "chm_bruteforce_work_bytes": (i32, [i32, i32, P(u64)]),
            "chm_bruteforce": (i32, [vp, i32, vp, i32, i32, i32, vp, vp, u64, vp]),
            "chm_bruteforce_noalloc": (i32, [vp, i32, vp, i32, i32, i32, vp, vp]),
            "chm_schedule_mbr": (i32, [i32, vp, i32, vp, u64, i32, P(vp)]),
            "chm_schedule_from_steps": (i32, [i32, i32, vp, vp, u64, i32, vp, vp, vp, vp, vp, vp, P(vp)]),
            "chm_schedule_num_steps": (i32, [vp]),
            "chm_schedule_step": (i32, [vp, i32, P(P(i32)), P(i32), P(P(i32)), P(i32), P(P(i32)), P(i32)]),
            "chm_schedule_info": (i32, [vp, P(i32), P(i32), P(P(i32)), P(P(i32))]),
            "chm_schedule_free": (None, [vp]),
            "chm_gps_order": (i32, [i32, vp, i32, vp, i32, vp]),
            "chm_run_schedule": (i32, [vp, vp, vp, i32, vp, vp, vp, vp, vp]),
            "chm_sao_filter": (i32, [i32, vp, vp, vp, i32, vp, vp, i32, i32, i32, i32, vp, vp]),
            "chm_sao_work_bytes": (i32, [i32, i32, P(u64)]),
            "chm_sao_filter_device": (i32, [i32, vp, vp, vp, i32, vp, vp, i32, i32, i32, vp, vp, vp, u64, vp]),
            "chm_run_schedule_sao": (i32, [vp, vp, vp, i32, vp, vp, i32, vp, vp, vp, i32, i32, i32, vp, vp, u64,
                                           vp]),
            "chm_run_schedule_verify": (i32, [vp, vp, vp, i32, vp, vp, i32, vp, vp, vp, i32, i32, i32, vp, vp, u64,
                                              vp, vp, i32, i32, i32, i32, vp, vp, vp]),
            "chm_ransac_filter": (i32, [i32, vp, vp, vp, i32, vp, vp, vp, i32, i32, i32, i32, vp, vp]),
            "chm_ransac_work_bytes": (i32, [i32, i32, P(u64)]),
            "chm_ransac_filter_device": (i32, [i32, vp, vp, vp, i32, vp, vp, vp, i32, i32, i32, vp, vp, vp, u64,
                                               vp]),
            "chm_run_schedule_verify_device": (i32, [vp, vp, vp, i32, vp, vp, i32, vp, vp, vp, i32, i32, i32, vp,
                                                     vp, u64, vp, i32, i32, i32, vp, vp, u64, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.chm_abi_version() != ABI_VERSION:
            raise ChmError(-6, "libchm ABI %d != binding %d" % (L.chm_abi_version(), ABI_VERSION))
        _lib = L
    return _lib


def _check(st: int) -> None:
    if st != 0:
        raise ChmError(st, lib().chm_last_error().decode(errors="replace"))


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def config(L=6, m=8, K=8, ratio=(4, 5), precision=PROJ_BF16, fixup_rel=1e-4,
           accept_single=False, whole_last_bucket=False) -> Config:
    c = Config()
    lib().chm_config_default(C.byref(c))
    c.num_tables, c.bucket_bits, c.top_k = L, m, K
    c.ratio_num, c.ratio_den = ratio
    c.proj_precision = precision
    c.fixup_rel = fixup_rel
    c.flags = (ACCEPT_SINGLE if accept_single else 0) | (WHOLE_LAST_BUCKET if whole_last_bucket else 0)
    return c


def image_bytes(cfg: Config, n: int) -> int:
    out = C.c_uint64()
    _check(lib().chm_image_bytes(C.byref(cfg), int(n), C.byref(out)))
    return out.value


def store_overhead_bytes(cfg: Config) -> int:
    out = C.c_uint64()
    _check(lib().chm_store_overhead_bytes(C.byref(cfg), C.byref(out)))
    return out.value


class Store:
    """Images resident in a caller-owned device arena (a torch uint8 tensor)."""

    def __init__(self, cfg: Config, W: np.ndarray, mu: np.ndarray, arena):
        self.cfg = cfg
        self.arena = arena
        W = np.ascontiguousarray(W, dtype=np.uint16)
        mu = np.ascontiguousarray(mu, dtype=np.uint8)
        h = C.c_void_p()
        _check(lib().chm_store_create(C.byref(cfg), _np_ptr(W), _np_ptr(mu), _dev_ptr(arena),
                                      arena.numel() * arena.element_size(), C.byref(h)))
        self.handle = h
        self.feats = {}
        self._keep = []

    def close(self):
        if self.handle:
            lib().chm_store_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, ids: Sequence[int], descs, stream=None):
        """descs: device uint8 tensors (n x 128) or host numpy arrays."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        if len(ids) == 0:
            return
        on_dev = [hasattr(d, "is_cuda") and d.is_cuda for d in descs]
        if any(on_dev) and not all(on_dev):
            raise ValueError("descriptors must be all device tensors or all host arrays")
        if all(on_dev):
            ptrs = [(_dev_ptr(d) or 0) for d in descs]
            ns = [int(d.shape[0]) for d in descs]
            keep = None
        else:
            keep = [np.ascontiguousarray(d, dtype=np.uint8) for d in descs]
            ptrs = [k.ctypes.data for k in keep]
            ns = [k.shape[0] for k in keep]
        parr = (C.c_void_p * len(ptrs))(*ptrs)
        narr = np.ascontiguousarray(ns, dtype=np.int32)
        _check(lib().chm_store_load(self.handle, len(ids), _np_ptr(ids), parr, _np_ptr(narr),
                                    1 if all(on_dev) else 0, _stream(stream)))
        if keep is not None:
            # pageable host memory: the copy has been staged by the time the call returns
            import torch
            torch.cuda.synchronize()
        for i, n in zip(ids, ns):
            self.feats[int(i)] = n

    def rehash(self, ids: Sequence[int], stream=None):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        _check(lib().chm_store_rehash(self.handle, len(ids), _np_ptr(ids), _stream(stream)))

    def evict(self, ids: Sequence[int]):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        _check(lib().chm_store_evict(self.handle, len(ids), _np_ptr(ids)))
        for i in ids:
            self.feats.pop(int(i), None)

    def image_feats(self, image_id: int) -> int:
        out = C.c_int32()
        _check(lib().chm_store_image_feats(self.handle, int(image_id), C.byref(out)))
        return out.value

    def stats(self) -> Stats:
        s = Stats()
        _check(lib().chm_store_stats(self.handle, C.byref(s)))
        return s

    def tuning(self) -> Tuning:
        t = Tuning()
        _check(lib().chm_store_get_tuning(self.handle, C.byref(t)))
        return t

    def set_tuning(self, queries_per_item=None, wg_threads=None, lds_codes=None, grid_per_cu=None, **more):
        """Changes the named fields of the store's chm_tuning (the others keep
        their values); keyword names are the fields of Tuning."""
        t = self.tuning()
        vals = dict(queries_per_item=queries_per_item, wg_threads=wg_threads, lds_codes=lds_codes,
                    grid_per_cu=grid_per_cu, **more)
        for k, v in vals.items():
            if k not in TUNING_FIELDS:
                raise TypeError("unknown tuning field %s" % k)
            if v is not None:
                setattr(t, k, int(v))
        _check(lib().chm_store_set_tuning(self.handle, C.byref(t)))

    def tuning_dict(self) -> dict:
        t = self.tuning()
        return {k: int(getattr(t, k)) for k in TUNING_FIELDS}

    def debug_image(self, image_id: int, stream=None):
        """Internal arrays of a resident image as device tensors."""
        import torch
        n = self.image_feats(image_id)
        if n < 0:
            raise ChmError(-4, "image %d is not resident" % image_id)
        L, nb = self.cfg.num_tables, 1 << self.cfg.bucket_bits
        dev = self.arena.device
        codes = torch.empty((n, 4), dtype=torch.int32, device=dev)
        ids = torch.empty((L, n), dtype=torch.uint8, device=dev)
        offs = torch.empty((L, nb + 1), dtype=torch.int32, device=dev)
        mem = torch.empty((L, n), dtype=torch.int16, device=dev)
        norms = torch.empty((n,), dtype=torch.int32, device=dev)
        _check(lib().chm_debug_image(self.handle, int(image_id), _dev_ptr(codes), _dev_ptr(ids),
                                     _dev_ptr(offs), _dev_ptr(mem), _dev_ptr(norms), _stream(stream)))
        return dict(codes=codes, ids=ids, offsets=offs, members=mem, norms=norms)


def out_offsets(store: Store, pairs: np.ndarray) -> np.ndarray:
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    offs = np.zeros(len(pairs) + 1, dtype=np.int64)
    if len(pairs):
        offs[1:] = np.cumsum([store.feats[int(q)] for q in pairs[:, 0]])
    return offs


class Plan:
    """An executable matching plan for a pair list (chm_plan_create)."""

    def __init__(self, store: Store, pairs: np.ndarray, offs: np.ndarray, out, topk=None,
                 mode: int = MATCH_BATCHED, stream=None):
        self.store = store
        self.pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        self.offs = np.ascontiguousarray(offs, dtype=np.int64)
        self.out, self.topk = out, topk
        h = C.c_void_p()
        _check(lib().chm_plan_create(store.handle, _np_ptr(self.pairs), len(self.pairs),
                                     _np_ptr(self.offs), _dev_ptr(out), _dev_ptr(topk), int(mode),
                                     _stream(stream), C.byref(h)))
        self.handle = h

    def execute(self, stream=None):
        _check(lib().chm_plan_execute(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            lib().chm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def match_pairs(store: Store, pairs, out, mode=MATCH_BATCHED, stream=None, offs=None):
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    offs = out_offsets(store, pairs) if offs is None else np.ascontiguousarray(offs, np.int64)
    _check(lib().chm_match_pairs(store.handle, _np_ptr(pairs), len(pairs), _np_ptr(offs),
                                 _dev_ptr(out), int(mode), _stream(stream)))
    return offs


def debug_fail_hip(n: int) -> None:
    """Test hook: the n-th checked HIP call of this thread fails (0 cancels)."""
    lib().chm_debug_fail_hip(int(n))


def bruteforce_work_bytes(nq: int, nd: int) -> int:
    out = C.c_uint64()
    _check(lib().chm_bruteforce_work_bytes(int(nq), int(nd), C.byref(out)))
    return out.value


def bruteforce(q, d, out, work, ratio=(4, 5), stream=None):
    _check(lib().chm_bruteforce(_dev_ptr(q), int(q.shape[0]), _dev_ptr(d), int(d.shape[0]),
                                int(ratio[0]), int(ratio[1]), _dev_ptr(out), _dev_ptr(work),
                                work.numel() * work.element_size(), _stream(stream)))


def bruteforce_noalloc(q, d, out, ratio=(4, 5), stream=None):
    """chm_bruteforce with the library's own fixed device workspace."""
    _check(lib().chm_bruteforce_noalloc(_dev_ptr(q), int(q.shape[0]), _dev_ptr(d), int(d.shape[0]),
                                        int(ratio[0]), int(ratio[1]), _dev_ptr(out), _stream(stream)))


@dataclass
class Schedule:
    steps: List[dict]
    iterations: int
    fallback_pairs: int
    dims: List[int]
    bandwidths: List[int]
    handle: Optional[C.c_void_p] = None


def schedule_mbr(n_images: int, pairs: np.ndarray, image_bytes_: Sequence[int], cap_bytes: int,
                 blk_images: int, keep_handle: bool = False) -> Schedule:
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    sizes = np.ascontiguousarray(image_bytes_, dtype=np.uint64)
    h = C.c_void_p()
    _check(lib().chm_schedule_mbr(int(n_images), _np_ptr(pairs), len(pairs), _np_ptr(sizes),
                                  int(cap_bytes), int(blk_images), C.byref(h)))
    L = lib()
    steps = []
    P32 = C.POINTER(C.c_int32)
    for k in range(L.chm_schedule_num_steps(h)):
        ev, ld, pp = P32(), P32(), P32()
        nev, nld, npp = C.c_int32(), C.c_int32(), C.c_int32()
        _check(L.chm_schedule_step(h, k, C.byref(ev), C.byref(nev), C.byref(ld), C.byref(nld),
                                   C.byref(pp), C.byref(npp)))
        steps.append(dict(evict=[ev[i] for i in range(nev.value)],
                          load=[ld[i] for i in range(nld.value)],
                          pairs=[pp[i] for i in range(npp.value)]))
    it, fb = C.c_int32(), C.c_int32()
    dims, bws = P32(), P32()
    _check(L.chm_schedule_info(h, C.byref(it), C.byref(fb), C.byref(dims), C.byref(bws)))
    sch = Schedule(steps=steps, iterations=it.value, fallback_pairs=fb.value,
                   dims=[dims[i] for i in range(it.value)],
                   bandwidths=[bws[i] for i in range(it.value)])
    if keep_handle:
        sch.handle = h
    else:
        L.chm_schedule_free(h)
    return sch


def schedule_from_steps(n_images: int, pairs: np.ndarray, image_bytes_: Sequence[int], cap_bytes: int,
                        steps: Sequence[dict]) -> Schedule:
    """A library schedule (with its handle, for run_schedule) from explicit
    steps, each a dict of evict / load / pairs lists (chm_schedule_from_steps
    checks the residency they imply)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    sizes = np.ascontiguousarray(image_bytes_, dtype=np.uint64)

    def csr(key):
        offs = np.zeros(len(steps) + 1, np.int32)
        offs[1:] = np.cumsum([len(s[key]) for s in steps])
        ids = np.ascontiguousarray(np.concatenate([np.asarray(s[key], np.int32) for s in steps])
                                   if steps else np.zeros(0, np.int32), dtype=np.int32)
        return offs, ids

    (eo, ei), (lo, li), (po, pi) = csr("evict"), csr("load"), csr("pairs")
    h = C.c_void_p()
    _check(lib().chm_schedule_from_steps(int(n_images), len(pairs), _np_ptr(pairs), _np_ptr(sizes),
                                         int(cap_bytes), len(steps), _np_ptr(eo), _np_ptr(ei), _np_ptr(lo),
                                         _np_ptr(li), _np_ptr(po), _np_ptr(pi), C.byref(h)))
    return Schedule(steps=[dict(evict=list(s["evict"]), load=list(s["load"]), pairs=list(s["pairs"]))
                           for s in steps], iterations=0, fallback_pairs=0, dims=[], bandwidths=[], handle=h)


def schedule_free(s: Schedule) -> None:
    if s.handle:
        lib().chm_schedule_free(s.handle)
        s.handle = None


def gps_order(n: int, edges: np.ndarray, nodes: Sequence[int]) -> List[int]:
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    nodes = np.ascontiguousarray(nodes, dtype=np.int32)
    out = np.zeros(len(nodes), dtype=np.int32)
    _check(lib().chm_gps_order(int(n), _np_ptr(edges), len(edges), _np_ptr(nodes), len(nodes),
                               _np_ptr(out)))
    return out.tolist()


def run_schedule(store: Store, sched: Schedule, pairs: np.ndarray, descs: Sequence[np.ndarray],
                 offs: np.ndarray, out, stream=None) -> None:
    """Runs a schedule kept with keep_handle=True; descs are host arrays per image."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    keep = [np.ascontiguousarray(d, dtype=np.uint8) for d in descs]
    parr = (C.c_void_p * len(keep))(*[k.ctypes.data for k in keep])
    ns = np.ascontiguousarray([k.shape[0] for k in keep], dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    _check(lib().chm_run_schedule(store.handle, sched.handle, _np_ptr(pairs), len(pairs), parr,
                                  _np_ptr(ns), _np_ptr(offs), _dev_ptr(out), _stream(stream)))


def run_schedule_sao(store: Store, sched: Schedule, pairs: np.ndarray, descs: Sequence[np.ndarray],
                     offs: np.ndarray, out, keypoints, filtered, work=None, n_neighbors: int = 6,
                     threshold=(1, 2), stream=None):
    """run_schedule plus the device SAO filter of every step's pairs
    (keypoints: device (n, 2) int32 tensors per image).  Returns the work
    tensor (see sao_input_errors)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    keep = [np.ascontiguousarray(d, dtype=np.uint8) for d in descs]
    parr = (C.c_void_p * len(keep))(*[k.ctypes.data for k in keep])
    ns = np.ascontiguousarray([k.shape[0] for k in keep], dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    kptr = (C.c_void_p * len(keypoints))(*[_dev_ptr(k) for k in keypoints])
    if work is None:
        import torch
        nmax = int(max((ns[q] for q in pairs[:, 0]), default=1))
        work = torch.empty(sao_work_bytes(len(pairs), nmax) + 256, dtype=torch.uint8, device=out.device)
        work = work[(-work.data_ptr()) % 256:]
    _check(lib().chm_run_schedule_sao(store.handle, sched.handle, _np_ptr(pairs), len(pairs), parr,
                                      _np_ptr(ns), len(keep), _np_ptr(offs), _dev_ptr(out),
                                      C.cast(kptr, C.c_void_p), n_neighbors, int(threshold[0]),
                                      int(threshold[1]), _dev_ptr(filtered), _dev_ptr(work),
                                      int(work.numel()), _stream(stream)))
    return work


def run_schedule_verify(store: Store, sched: Schedule, pairs: np.ndarray, descs: Sequence[np.ndarray],
                        offs: np.ndarray, out, keypoints, host_keypoints, filtered, words: np.ndarray,
                        h_filtered: np.ndarray, h_verified: np.ndarray, iterations: int = 64, thr: int = 64,
                        min_inliers: int = 8, n_neighbors: int = 6, threshold=(1, 2), n_threads: int = 0,
                        work=None, stream=None):
    """run_schedule_sao plus RANSAC of every step on host threads beside the
    device: h_filtered receives the SAO output and h_verified the verified
    matches (host int32 arrays laid out like out; h_filtered best pinned).
    Returns the SAO work tensor."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    keep = [np.ascontiguousarray(d, dtype=np.uint8) for d in descs]
    parr = (C.c_void_p * len(keep))(*[k.ctypes.data for k in keep])
    ns = np.ascontiguousarray([k.shape[0] for k in keep], dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    kptr = (C.c_void_p * len(keypoints))(*[_dev_ptr(k) for k in keypoints])
    hk = [np.ascontiguousarray(k, dtype=np.int32) for k in host_keypoints]
    hptr = (C.c_void_p * len(hk))(*[k.ctypes.data for k in hk])
    words = np.ascontiguousarray(words, dtype=np.uint32)
    for a in (h_filtered, h_verified):
        if a.dtype != np.int32 or not a.flags.c_contiguous or a.size < int(offs[-1]):
            raise ValueError("host outputs must be contiguous int32 arrays laid out like out")
    if work is None:
        import torch
        nmax = int(max((ns[q] for q in pairs[:, 0]), default=1))
        work = torch.empty(sao_work_bytes(len(pairs), nmax) + 256, dtype=torch.uint8, device=out.device)
        work = work[(-work.data_ptr()) % 256:]
    _check(lib().chm_run_schedule_verify(store.handle, sched.handle, _np_ptr(pairs), len(pairs), parr,
                                         _np_ptr(ns), len(keep), _np_ptr(offs), _dev_ptr(out),
                                         C.cast(kptr, C.c_void_p), n_neighbors, int(threshold[0]),
                                         int(threshold[1]), _dev_ptr(filtered), _dev_ptr(work),
                                         int(work.numel()), C.cast(hptr, C.c_void_p), _np_ptr(words),
                                         int(iterations), int(thr), int(min_inliers), int(n_threads),
                                         _np_ptr(h_filtered), _np_ptr(h_verified), _stream(stream)))
    return work


def sao_filter(keypoints: Sequence[np.ndarray], pairs: np.ndarray, offs: np.ndarray,
               matches: np.ndarray, n_neighbors: int = 6, threshold=(1, 2), n_threads: int = 0,
               want_ced: bool = False):
    """SAO local constraint (Sec. 2.3.3) on host threads: filtered matches
    (and the CED per query row when want_ced).  keypoints[img] is an (n, 2)
    int32 array; matches is the matcher's output for `pairs` laid out by
    `offs`."""
    kps = [np.ascontiguousarray(k, dtype=np.int32) for k in keypoints]
    nf = np.array([k.shape[0] for k in kps], dtype=np.int32)
    ptrs = (C.c_void_p * max(1, len(kps)))(*[k.ctypes.data for k in kps])
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    matches = np.ascontiguousarray(matches, dtype=np.int32)
    out = np.empty_like(matches)
    ced = np.empty_like(matches) if want_ced else None
    _check(lib().chm_sao_filter(len(pairs), _np_ptr(pairs), C.cast(ptrs, C.c_void_p), _np_ptr(nf),
                                len(kps), _np_ptr(offs), _np_ptr(matches), n_neighbors,
                                int(threshold[0]), int(threshold[1]), n_threads, _np_ptr(out),
                                _np_ptr(ced)))
    return (out, ced) if want_ced else out


def sao_work_bytes(n_pairs: int, max_query_rows: int) -> int:
    v = C.c_uint64()
    _check(lib().chm_sao_work_bytes(int(n_pairs), int(max_query_rows), C.byref(v)))
    return int(v.value)


def sao_filter_device(keypoints, pairs: np.ndarray, offs: np.ndarray, match, out, ced=None, work=None,
                      n_neighbors: int = 6, threshold=(1, 2), stream=None):
    """SAO on the device (n_neighbors <= 8): `keypoints[img]` is a device
    (n, 2) int32 tensor, `match`/`out`/`ced` device int32 tensors laid out
    by `offs`, `work` a device uint8 tensor of sao_work_bytes() bytes
    (allocated here when None).  Returns the work tensor; its first int32 is
    the number of pairs whose input broke the contract (see
    sao_input_errors)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    nf = np.array([0 if k is None else int(k.shape[0]) for k in keypoints], dtype=np.int32)
    ptrs = (C.c_void_p * max(1, len(keypoints)))(*[0 if k is None else _dev_ptr(k) for k in keypoints])
    if work is None:
        import torch
        nmax = int(max((nf[q] for q in pairs[:, 0]), default=1))
        work = torch.empty(sao_work_bytes(len(pairs), nmax) + 256, dtype=torch.uint8, device=match.device)
        work = work[(-work.data_ptr()) % 256:]
    _check(lib().chm_sao_filter_device(len(pairs), _np_ptr(pairs), C.cast(ptrs, C.c_void_p), _np_ptr(nf),
                                       len(keypoints), _np_ptr(offs), _dev_ptr(match), n_neighbors,
                                       int(threshold[0]), int(threshold[1]), _dev_ptr(out), _dev_ptr(ced),
                                       _dev_ptr(work), int(work.numel()), _stream(stream)))
    return work


def sao_input_errors(work) -> int:
    """Pairs of the last device SAO call on `work` whose input broke the
    contract (waits for the call)."""
    return int(work[:4].view(dtype=__import__("torch").int32).item())


def ransac_filter(keypoints: Sequence[np.ndarray], pairs: np.ndarray, offs: np.ndarray, matches: np.ndarray,
                  words: np.ndarray, thr: int, min_inliers: int = 8, n_threads: int = 0):
    """RANSAC verification (Sec. 2.3.3) on host threads: (verified matches,
    best inlier count per pair).  words: (n_pairs, iterations, 2) uint32."""
    kps = [np.ascontiguousarray(k, dtype=np.int32) for k in keypoints]
    nf = np.array([k.shape[0] for k in kps], dtype=np.int32)
    ptrs = (C.c_void_p * max(1, len(kps)))(*[k.ctypes.data for k in kps])
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    matches = np.ascontiguousarray(matches, dtype=np.int32)
    words = np.ascontiguousarray(words, dtype=np.uint32).reshape(len(pairs), -1, 2)
    out = np.empty_like(matches)
    best = np.empty(len(pairs), dtype=np.int32)
    _check(lib().chm_ransac_filter(len(pairs), _np_ptr(pairs), C.cast(ptrs, C.c_void_p), _np_ptr(nf),
                                   len(kps), _np_ptr(offs), _np_ptr(matches), _np_ptr(words),
                                   int(words.shape[1]), int(thr), int(min_inliers), n_threads,
                                   _np_ptr(out), _np_ptr(best)))
    return out, best


def ransac_work_bytes(n_pairs: int, max_query_rows: int) -> int:
    v = C.c_uint64()
    _check(lib().chm_ransac_work_bytes(int(n_pairs), int(max_query_rows), C.byref(v)))
    return int(v.value)


def _aligned_work(nbytes: int, device):
    import torch
    w = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    return w[(-w.data_ptr()) % 256:]


def ransac_filter_device(keypoints, pairs: np.ndarray, offs: np.ndarray, match, out, words, thr: int,
                         min_inliers: int = 8, best_counts=None, work=None, stream=None):
    """RANSAC verification on the device: `keypoints[img]` a device (n, 2)
    int32 tensor, `match`/`out` device int32 tensors laid out by `offs`
    (`out` may be `match`), `words` a device uint32 tensor of shape
    (n_pairs, iterations, 2), `best_counts` an optional device int32 tensor
    per pair.  Returns the work tensor; its first int32 counts the pairs
    whose input broke the contract."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    nf = np.array([0 if k is None else int(k.shape[0]) for k in keypoints], dtype=np.int32)
    ptrs = (C.c_void_p * max(1, len(keypoints)))(*[0 if k is None else _dev_ptr(k) for k in keypoints])
    iterations = int(words.shape[1]) if words.dim() == 3 else 0
    if work is None:
        nmax = int(max((nf[q] for q in pairs[:, 0]), default=1))
        work = _aligned_work(ransac_work_bytes(len(pairs), nmax), match.device)
    _check(lib().chm_ransac_filter_device(len(pairs), _np_ptr(pairs), C.cast(ptrs, C.c_void_p), _np_ptr(nf),
                                          len(keypoints), _np_ptr(offs), _dev_ptr(match), _dev_ptr(words),
                                          iterations, int(thr), int(min_inliers), _dev_ptr(out),
                                          _dev_ptr(best_counts), _dev_ptr(work), int(work.numel()),
                                          _stream(stream)))
    return work


def run_schedule_verify_device(store: "Store", sched: "Schedule", pairs: np.ndarray, descs: Sequence[np.ndarray],
                               offs: np.ndarray, out, keypoints, filtered, verified, words, iterations: int = 64,
                               thr: int = 64, min_inliers: int = 8, n_neighbors: int = 6, threshold=(1, 2),
                               work=None, rwork=None, stream=None):
    """run_schedule_sao plus device RANSAC of every step on the same stream:
    `filtered` receives the SAO output and `verified` the verified matches
    (device int32 tensors laid out like out); `words` a device uint32 tensor
    (n_pairs, iterations, 2).  Returns (SAO work, RANSAC work)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    keep = [np.ascontiguousarray(d, dtype=np.uint8) for d in descs]
    parr = (C.c_void_p * len(keep))(*[k.ctypes.data for k in keep])
    ns = np.ascontiguousarray([k.shape[0] for k in keep], dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    kptr = (C.c_void_p * len(keypoints))(*[_dev_ptr(k) for k in keypoints])
    nmax = int(max((ns[q] for q in pairs[:, 0]), default=1))
    if work is None:
        work = _aligned_work(sao_work_bytes(len(pairs), nmax), out.device)
    if rwork is None:
        rwork = _aligned_work(ransac_work_bytes(len(pairs), nmax), out.device)
    _check(lib().chm_run_schedule_verify_device(store.handle, sched.handle, _np_ptr(pairs), len(pairs), parr,
                                                _np_ptr(ns), len(keep), _np_ptr(offs), _dev_ptr(out),
                                                C.cast(kptr, C.c_void_p), n_neighbors, int(threshold[0]),
                                                int(threshold[1]), _dev_ptr(filtered), _dev_ptr(work),
                                                int(work.numel()), _dev_ptr(words), int(iterations), int(thr),
                                                int(min_inliers), _dev_ptr(verified), _dev_ptr(rwork),
                                                int(rwork.numel()), _stream(stream)))
    return work, rwork

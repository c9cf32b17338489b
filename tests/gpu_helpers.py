"""Helpers shared by the GPU tests: build a store for a workload and compare
its arrays and matches with the oracle."""
import numpy as np
import torch

from paper_2505_22089_amd import chm


def device():
    return torch.device("cuda:0")


def new_store(wl, precision=chm.PROJ_BF16, K=None, L=None, m=None, extra=64 << 20, fixup_rel=1e-4,
              accept_single=False, whole_last_bucket=False):
    cfg = chm.config(L=wl.L if L is None else L, m=wl.m if m is None else m,
                     K=wl.K if K is None else K, ratio=wl.ratio, precision=precision,
                     fixup_rel=fixup_rel, accept_single=accept_single,
                     whole_last_bucket=whole_last_bucket)
    need = chm.store_overhead_bytes(cfg) + sum(chm.image_bytes(cfg, x.shape[0]) + 256
                                               for x in wl.images) + extra
    arena = torch.empty(need, dtype=torch.uint8, device=device())
    W = wl.W[:128 + cfg.num_tables * cfg.bucket_bits]
    return chm.Store(cfg, W, wl.mu, arena)


def load_all(store, images, ids=None):
    ids = list(range(len(images))) if ids is None else list(ids)
    tens = [torch.from_numpy(np.ascontiguousarray(images[i])).to(device()) for i in ids]
    store.load(ids, tens)
    torch.cuda.synchronize()
    return tens


def gpu_arrays(store, image_id):
    d = store.debug_image(image_id)
    torch.cuda.synchronize()
    L = store.cfg.num_tables
    return dict(codes=d["codes"].cpu().numpy().view(np.uint32),
                ids=np.ascontiguousarray(d["ids"].cpu().numpy().T),
                offsets=d["offsets"].cpu().numpy(),
                members=d["members"].cpu().numpy().view(np.uint16).astype(np.int32),
                norms=d["norms"].cpu().numpy().view(np.uint32))


def run_match(store, pairs, mode=chm.MATCH_BATCHED, want_topk=False, repeats=1):
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    offs = chm.out_offsets(store, pairs)
    total = int(offs[-1])
    K = store.cfg.top_k
    out = torch.full((max(total, 1),), -7, dtype=torch.int32, device=device())
    topk = torch.zeros((max(total, 1) * K,), dtype=torch.int32, device=device()) if want_topk else None
    plan = chm.Plan(store, pairs, offs, out, topk, mode)
    for _ in range(repeats):
        plan.execute()
    torch.cuda.synchronize()
    plan.close()
    o = out.cpu().numpy()[:total]
    t = topk.cpu().numpy().view(np.uint32)[:total * K].reshape(total, K) if want_topk else None
    return o, t, offs

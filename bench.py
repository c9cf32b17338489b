"""Benchmark: matched image pairs/s of GPU cascade-hashing matching.

Workload: 50 images x 8,000 SIFT-like uint8 descriptors, 400 directed pairs
from an 8-NN view graph, 40 % planted overlap, L=6 tables x m=8 bits,
n=128-bit codes, K=8, ratio 4/5 (synthetic, seeded).  One step is the whole
hot path over the resident descriptors: projection + fp64 fix-up + bucket
tables for all 50 images, then matching of all 400 pairs in one batched
launch (persistent kernel replayed from a HIP graph).  The plain per-pair
path (one launch per pair, host loop) is timed beside it.

Other workloads (--workload strips | knn-200x40000) run the same step on the
larger synthetic inputs; the default is the one above.  --workload
grid-5000x10000 instead runs the whole MBR-scheduled job (Algorithm 1) from
pinned host memory under GPU residency caps (default 16 GB and 2 GB):
descriptors loaded and freed per block row, hashed and matched on the GPU.

Prints one JSON line.  --gpus N > 1 is not supported: the path runs on one
GPU (pairs would be sharded by contiguous ranges of block rows, one per GPU).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matched image pairs/sec at 8k feats/image (batched vs plain), bit-exact matches"
HBM_PEAK_GBS = 8000.0
# 32-bit integer VALU lane-ops per second: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter scaling under rocprofv3)")
    ap.add_argument("--profile", action="store_true", help="few steps, no CPU leg (for rocprofv3)")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain per-pair path")
    ap.add_argument("--workload", default="knn-50x8000",
                    choices=["knn-50x8000", "strips", "knn-200x40000", "grid-5000x10000"])
    ap.add_argument("--caps", default="16,2", help="grid workload: residency caps in GB")
    ap.add_argument("--size-blk", type=int, default=400, help="grid workload: Size_blk (images)")
    ap.add_argument("--grid-shape", default="50,100,10000", help="grid workload: rows,cols,features")
    ap.add_argument("--grid-sao", action="store_true",
                    help="grid workload: also run the first cap with the device SAO filter per step")
    ap.add_argument("--grid-verify", action="store_true",
                    help="grid workload: also run the first cap with the device SAO per step and RANSAC of "
                         "every step on host threads beside the device (outlier removal included)")
    ap.add_argument("--grid-study", default="",
                    help="grid workload: caps in GB (e.g. 2,0.5) at which to run the schedule study on the "
                         "device: MBR at every --study-blks Size_blk, the load/free-list and graph-partition "
                         "schedules over all pairs, and the per-pair schedule over --naive-pairs pairs")
    ap.add_argument("--study-blks", default="50,100,200,400,800")
    ap.add_argument("--naive-pairs", type=int, default=2000)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--no-reuse", action="store_true",
                    help="also time the plain path re-hashing both images of every pair "
                         "(always on for the benchmark workload)")
    ap.add_argument("--tuning", default="default",
                    help="'default' (the library's), 'auto' (autotuner), or comma-separated "
                         "name=value chm_tuning fields")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus %d requested); sharding over several "
              "GPUs is not built" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        return copy_calibration()
    if args.profile:
        args.steps, args.warmup, args.plain_steps, args.no_cpu = 5, 2, 1, True
    if args.workload == "grid-5000x10000":
        return run_grid(args)
    import torch

    from paper_2505_22089_amd import chm, synth

    dev = torch.device("cuda:0")
    gen = {"knn-50x8000": synth.config2, "strips": synth.config3, "knn-200x40000": synth.config4}
    print("[bench] generating %s" % args.workload, file=sys.stderr, flush=True)
    wl = gen[args.workload]()
    if args.workload != "knn-50x8000" and args.steps == 50:
        args.steps, args.warmup, args.plain_steps = 5, 2, 1
    n_img = len(wl.images)
    P = len(wl.pairs)
    prec = chm.PROJ_FP32 if args.precision == "fp32" else chm.PROJ_BF16
    cfg = chm.config(L=wl.L, m=wl.m, K=wl.K, ratio=wl.ratio, precision=prec)
    need = chm.store_overhead_bytes(cfg) + sum(chm.image_bytes(cfg, x.shape[0]) + 256 for x in wl.images)
    # room beyond the images for the plans: work lists and the bucket-major
    # kept lists (32 B per query of every pair at K = 8)
    arena = torch.empty(need + (640 << 20), dtype=torch.uint8, device=dev)
    store = chm.Store(cfg, wl.W, wl.mu, arena)
    lib_tuning = store.tuning_dict()
    descs = [torch.from_numpy(x).to(dev) for x in wl.images]
    ids = list(range(n_img))
    store.load(ids, descs)
    torch.cuda.synchronize()
    s0 = store.stats()
    store.rehash(ids)
    s1 = store.stats()
    fixups_per_hash = s1.fixups - s0.fixups  # projections recomputed in fp64 by one hash pass
    flips_per_hash = s1.fixup_flips - s0.fixup_flips  # of those, signs the MFMA sum had wrong
    print("[bench] %d images loaded and hashed" % n_img, file=sys.stderr, flush=True)

    stream = torch.cuda.Stream()
    offs = chm.out_offsets(store, wl.pairs)
    total_q = int(offs[-1])
    out_b = torch.empty(total_q, dtype=torch.int32, device=dev)
    out_p = torch.empty(total_q, dtype=torch.int32, device=dev)

    # candidate count of the workload: sum over pairs and tables of
    # hist_q(b) * hist_d(b) (table entries the method returns)
    hist = []
    for i in ids:
        o = store.debug_image(i)["offsets"].cpu().numpy().astype(np.int64)
        hist.append(np.diff(o, axis=1))
    cand = int(sum((hist[q] * hist[d]).sum() for q, d in wl.pairs))
    dense = int(sum(wl.images[q].shape[0] * wl.images[d].shape[0] for q, d in wl.pairs))

    # plain per-pair path: the faster of two launch shapes (a fair baseline)
    plain_best = None
    for tun in (() if args.no_plain else (dict(wg_threads=256, lds_codes=0), dict(wg_threads=1024, lds_codes=1))):
        store.set_tuning(**tun)
        with torch.cuda.stream(stream):
            pp = chm.Plan(store, wl.pairs, offs, out_p, None, chm.MATCH_PLAIN, stream)
            for _ in range(2):
                store.rehash(ids, stream)
                pp.execute(stream)
            stream.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.plain_steps):
                store.rehash(ids, stream)
                pp.execute(stream)
            stream.synchronize()
            dt = (time.perf_counter() - t1) / args.plain_steps
        pp.close()
        if plain_best is None or dt < plain_best[0]:
            plain_best = (dt, tun)
    # plain path without reuse: every pair re-hashes both of its images
    noreuse = None
    if args.no_reuse or (args.workload == "knn-50x8000" and not args.profile and not args.no_plain):
        if plain_best:
            store.set_tuning(**plain_best[1])
        plans = []
        with torch.cuda.stream(stream):
            for p in range(P):
                plans.append(chm.Plan(store, wl.pairs[p:p + 1], offs[p:p + 2], out_p, None,
                                      chm.MATCH_PLAIN, stream))
            stream.synchronize()
            t1 = time.perf_counter()
            for p in range(P):
                store.rehash([int(wl.pairs[p, 0]), int(wl.pairs[p, 1])], stream)
                plans[p].execute(stream)
            stream.synchronize()
            noreuse = P / (time.perf_counter() - t1)
        for pl in plans:
            pl.close()
    # batched path: launch shape chosen by the autotuner (results identical)
    tune_report = None
    if args.tuning == "auto":
        from paper_2505_22089_amd import autotune
        tune_report = {}
        store.set_tuning(**lib_tuning)
        best = autotune.tune(store, wl.pairs, reps=3, cache=None, report=tune_report)
    else:
        store.set_tuning(**lib_tuning)
        if args.tuning != "default":
            # name=value pairs of chm_tuning fields, e.g. match_kernel=0,queries_per_item=2048
            store.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
        best = store.tuning_dict()
    with torch.cuda.stream(stream):
        plan_b = chm.Plan(store, wl.pairs, offs, out_b, None, chm.MATCH_BATCHED, stream)

    def step():
        store.rehash(ids, stream)
        plan_b.execute(stream)

    for _ in range(args.warmup):
        step()
    stream.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for k in range(args.steps):
            ev[k][0].record(stream)
            store.rehash(ids, stream)
            ev[k][1].record(stream)
            plan_b.execute(stream)
            ev[k][2].record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hash_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    match_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    ms_step = wall * 1e3 / args.steps
    value = P / (wall / args.steps)

    plain_value = P / plain_best[0] if plain_best else None
    same = bool(torch.equal(out_b, out_p)) if plain_best else None

    # roofline of the dominant kernel (matching): 32-bit integer lane-ops.
    # Per returned candidate: 4 xor + 4 popcount + key + compare = 10 ops;
    # per query: K exact dot products of 32 packed-u8 dot4 ops.
    K = wl.K
    alg_ops = 10 * cand + 32 * K * total_q
    achieved = alg_ops / (match_ms * 1e-3) / 1e12
    tun = store.tuning_dict()
    nd = np.array([wl.images[d].shape[0] for d in wl.pairs[:, 1]])
    n_bm = int((nd >= tun["bm_min_db_feats"]).sum()) if tun["match_kernel"] == chm.KERNEL_BUCKET_MAJOR else 0
    lds_cap = 10175
    kernels = []
    if n_bm < P:
        kernels.append("k_match<%d,1024,%s,persistent> (query major, %d pairs)"
                       % (8 if K > 4 else K, "LDS-staged codes" if (nd[nd < tun["bm_min_db_feats"]] <= lds_cap).any()
                          else "HBM codes", P - n_bm))
    if n_bm:
        kernels.append("k_match_bm<%d> (bucket major, one launch per table and round, %d pairs)"
                       % (8 if K > 4 else K, n_bm))
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
            "unit": "TOP/s", "frac": round(achieved / ALU_PEAK_TOPS, 4),
            "traffic": recorded_traffic(args.workload),
            "kernel": " + ".join(kernels), "launch_us": round(match_ms * 1e3, 1),
            "ops_per_launch": alg_ops,
            "ops": "10 per candidate (4 xor, 4 popcount, key, compare) + 32 K per query (dot4 re-rank)"}
    # hashing stage against HBM, per descriptor: read 128 B, write the code
    # (16 B), L bucket ids (L B) and the norm (4 B); the table build reads the
    # L ids and writes L u16 members
    n_desc = int(sum(x.shape[0] for x in wl.images))
    hash_bytes = n_desc * (128 + 16 + wl.L + 4 + wl.L + 2 * wl.L)
    hash_gbs = hash_bytes / (hash_ms * 1e-3) / 1e9

    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": describe(wl), "L": wl.L, "m": wl.m, "n": 128, "K": K,
                   "ratio": "%d/%d" % wl.ratio, "projection": "%s MFMA + fp64 fix-up" % args.precision,
                   "mode": "batched", "tuning": best, "plain_tuning": plain_best[1] if plain_best else None},
        "plain_pairs_per_s": round(plain_value, 1) if plain_value else None,
        "plain_noreuse_pairs_per_s": round(noreuse, 1) if noreuse else None,
        "batched_over_plain": round(value / plain_value, 2) if plain_value else None,
        "batched_equals_plain": same,
        "stage_ms": {"hash_all_images": round(hash_ms, 4), "match_all_pairs": round(match_ms, 4)},
        "candidates_per_s": round(cand / (ms_step * 1e-3), 1),
        "dense_equiv_cmp_per_s": round(dense / (ms_step * 1e-3), 1),
        "hash_stage_hbm": {"achieved_GBs": round(hash_gbs, 1), "frac": round(hash_gbs / HBM_PEAK_GBS, 4),
                           "bytes_per_step": hash_bytes,
                           "fp64_fixups_per_descriptor": round(fixups_per_hash / n_desc, 4),
                           "mfma_sign_errors_per_descriptor": flips_per_hash / n_desc},
        "roofline": roof,
    }
    if tune_report is not None:
        res["autotune"] = {"default_tuning_match_ms": round(tune_report["default_ms"], 4),
                           "tuned_match_ms": round(tune_report["best_ms"], 4),
                           "tunings_timed": tune_report["timed"], "default_tuning": lib_tuning}

    if args.workload == "knn-200x40000":
        res["bruteforce"] = bruteforce_leg(wl, descs, stream)
    if not args.profile:
        print("[bench] SAO leg", file=sys.stderr, flush=True)
        res["sao"] = sao_leg(wl, out_b, offs, stream, host_pairs=None if args.workload != "knn-200x40000" else 50)
        res["with_outlier_removal"] = outlier_removal_leg(wl, store, ids, plan_b, out_b, offs, stream, P)
    if not args.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        if args.workload == "knn-50x8000":
            res["cpu_baseline"] = cpu_baseline(wl, out_b.cpu().numpy())
        else:
            res["cpu_baseline"] = cpu_baseline_sampled(wl, out_b.cpu().numpy(), offs)
    print(json.dumps(res), flush=True)
    plan_b.close()
    store.close()


def cpu_baseline(wl, gpu_out, min_seconds=10.0, max_reps=8):
    """The plain C oracle on the host cores, timed on whole steps: hash all
    images and match all pairs, repeated until about ten seconds of CPU work
    have run.  Its output is also compared with the GPU's over every pair."""
    from oracle import oracle as O
    threads = O.max_threads()
    P = len(wl.pairs)
    reps, t_hash, t_match, same = 0, 0.0, 0.0, True
    while reps < max_reps and (reps == 0 or t_hash + t_match < min_seconds):
        t0 = time.perf_counter()
        H = O.hash_workload(wl)
        t1 = time.perf_counter()
        out, soffs, _, _ = O.match_pairs(H, wl.pairs, wl.L, wl.m, wl.K, wl.ratio)
        t2 = time.perf_counter()
        t_hash += t1 - t0
        t_match += t2 - t1
        same = same and bool(np.array_equal(out, gpu_out[:int(soffs[-1])]))
        reps += 1
    t_step = (t_hash + t_match) / reps
    # one thread: the first 8 pairs (their images hashed), scaled to the step
    sub = wl.pairs[:8]
    need = sorted({int(i) for i in sub.ravel()})
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        H1 = O.hash_workload(wl, need)
        t1 = time.perf_counter()
        O.match_pairs(H1, sub, wl.L, wl.m, wl.K, wl.ratio)
        t2 = time.perf_counter()
    finally:
        O.set_threads(threads)
    one = (t1 - t0) / len(need) * len(wl.images) + (t2 - t1) / len(sub) * P
    return {"value": round(P / t_step, 2), "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "the whole step (hash %d images + match all %d pairs) run %d times: %.1f s hashing, "
                      "%.1f s matching" % (len(wl.images), P, reps, t_hash, t_match),
            "gpu_identical_all_pairs": same,
            "one_thread": {"value": round(P / one, 3), "unit": "pairs/s",
                           "sample": "8 pairs and their %d images on 1 thread, scaled to the whole step"
                                     % len(need)}}


def sao_leg(wl, out_b, offs, stream, reps=10, n_neighbors=6, threshold=(1, 2), host_pairs=None):
    """SAO local constraint (Sec. 2.3.3) on the batched matcher's output: the
    device kernel (keypoints resident in HBM, HIP events on the stream) and
    the host implementation on all hardware threads, over all pairs (or the
    first host_pairs), with their outputs compared."""
    import os
    import torch

    from paper_2505_22089_amd import chm, synth
    kps = synth.keypoints(wl)
    d_kps = [torch.from_numpy(k).to(out_b.device) for k in kps]
    nmax = int(max(wl.images[q].shape[0] for q in wl.pairs[:, 0]))
    work = torch.empty(chm.sao_work_bytes(len(wl.pairs), nmax) + 256, dtype=torch.uint8, device=out_b.device)
    work = work[(-work.data_ptr()) % 256:]
    d_out = torch.empty_like(out_b)
    with torch.cuda.stream(stream):
        chm.sao_filter_device(d_kps, wl.pairs, offs, out_b, d_out, None, work, n_neighbors, threshold, stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            chm.sao_filter_device(d_kps, wl.pairs, offs, out_b, d_out, None, work, n_neighbors, threshold,
                                  stream)
        b.record(stream)
    stream.synchronize()
    dev_ms = a.elapsed_time(b) / reps
    bad = chm.sao_input_errors(work)
    g = d_out.cpu().numpy()
    m = out_b.cpu().numpy()
    P = len(wl.pairs) if host_pairs is None else min(host_pairs, len(wl.pairs))
    end = int(offs[P])
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    h = chm.sao_filter(kps, wl.pairs[:P], offs[:P + 1], m[:end], n_neighbors, threshold, n_threads=threads)
    host_s = time.perf_counter() - t0
    # RANSAC verification of the SAO output on host threads (64 hypotheses, 4 px)
    words = synth.ransac_words(P, 64)
    t0 = time.perf_counter()
    v, _ = chm.ransac_filter(kps, wl.pairs[:P], offs[:P + 1], g[:end], words, 64, 8, n_threads=threads)
    ransac_s = time.perf_counter() - t0
    # and on the device, over all pairs (the same words for the host's pairs)
    dwords = torch.from_numpy(synth.ransac_words(len(wl.pairs), 64).view(np.int32)).to(out_b.device)
    d_ver = torch.empty_like(out_b)
    with torch.cuda.stream(stream):
        rwork = chm.ransac_filter_device(d_kps, wl.pairs, offs, d_out, d_ver, dwords, 64, 8, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            chm.ransac_filter_device(d_kps, wl.pairs, offs, d_out, d_ver, dwords, 64, 8, work=rwork, stream=stream)
        b.record(stream)
    stream.synchronize()
    rdev_ms = a.elapsed_time(b) / reps
    dv = d_ver.cpu().numpy()
    return {"n_neighbors": n_neighbors, "threshold": "%d/%d" % threshold,
            "device_ms": round(dev_ms, 4), "device_pairs_per_s": round(len(wl.pairs) / (dev_ms * 1e-3), 1),
            "matches_in": int((m >= 0).sum()), "kept": int((g >= 0).sum()), "input_errors": bad,
            "host_pairs": P, "host_threads": threads, "host_ms": round(host_s * 1e3, 1),
            "host_pairs_per_s": round(P / host_s, 1),
            "device_equals_host": bool(np.array_equal(g[:end], h)),
            "ransac_host_ms": round(ransac_s * 1e3, 1), "ransac_host_pairs_per_s": round(P / ransac_s, 1),
            "ransac_verified": int((v >= 0).sum()),
            "ransac_device_ms": round(rdev_ms, 4), "ransac_device_pairs_per_s": round(len(wl.pairs) / (rdev_ms * 1e-3), 1),
            "ransac_device_equals_host": bool(np.array_equal(dv[:end], v)),
            "ransac_device_input_errors": chm.sao_input_errors(rwork)}


def outlier_removal_leg(wl, store, ids, plan_b, out_b, offs, stream, P, steps=10):
    """The whole step with the paper's outlier removal on the device: rehash
    all images, match all pairs (the batched graph), SAO (6 neighbours,
    CED/N <= 1/2) and RANSAC (64 hypotheses, 4 px, at least 8 inliers) of
    every pair, timed together on the stream (the paper's timings include
    outlier removal)."""
    import torch

    from paper_2505_22089_amd import chm, synth
    dev = out_b.device
    kps = [torch.from_numpy(k).to(dev) for k in synth.keypoints(wl)]
    nmax = int(max(wl.images[q].shape[0] for q in wl.pairs[:, 0]))
    swork = torch.empty(chm.sao_work_bytes(P, nmax) + 256, dtype=torch.uint8, device=dev)
    swork = swork[(-swork.data_ptr()) % 256:]
    rwork = torch.empty(chm.ransac_work_bytes(P, nmax) + 256, dtype=torch.uint8, device=dev)
    rwork = rwork[(-rwork.data_ptr()) % 256:]
    words = torch.from_numpy(synth.ransac_words(P, 64).view(np.int32)).to(dev)
    filt = torch.empty_like(out_b)
    ver = torch.empty_like(out_b)

    def step():
        store.rehash(ids, stream)
        plan_b.execute(stream)
        chm.sao_filter_device(kps, wl.pairs, offs, out_b, filt, None, swork, 6, (1, 2), stream)
        chm.ransac_filter_device(kps, wl.pairs, offs, filt, ver, words, 64, 8, work=rwork, stream=stream)

    with torch.cuda.stream(stream):
        step()
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        stream.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    v = ver.cpu().numpy()
    return {"pairs_per_s": round(P / (ms * 1e-3), 1), "ms_per_step": round(ms, 4), "steps": steps,
            "matches": int((out_b.cpu().numpy() >= 0).sum()), "after_sao": int((filt.cpu().numpy() >= 0).sum()),
            "verified": int((v >= 0).sum()),
            "input_errors": chm.sao_input_errors(swork) + chm.sao_input_errors(rwork),
            "note": "wall clock per step; the SAO and RANSAC calls each upload their pair table once per call "
                    "(one stream synchronisation each)"}


def bruteforce_leg(wl, descs, stream, reps=5):
    """Exhaustive int8-MFMA 2-NN + ratio test on the first pair (40,000 x
    40,000): time per pair and the int8 MFMA roofline (2 * 128 ops per
    descriptor pair, dense int8 peak 5.0 POP/s)."""
    import torch

    from paper_2505_22089_amd import chm
    q, d = int(wl.pairs[0, 0]), int(wl.pairs[0, 1])
    Xq, Xd = descs[q], descs[d]
    out = torch.empty(Xq.shape[0], dtype=torch.int32, device=Xq.device)
    work = torch.empty(chm.bruteforce_work_bytes(Xq.shape[0], Xd.shape[0]), dtype=torch.uint8,
                       device=Xq.device)
    with torch.cuda.stream(stream):
        chm.bruteforce(Xq, Xd, out, work, wl.ratio, stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            chm.bruteforce(Xq, Xd, out, work, wl.ratio, stream)
        b.record(stream)
    stream.synchronize()
    ms = a.elapsed_time(b) / reps
    ops = 2.0 * 128 * Xq.shape[0] * Xd.shape[0]
    tops = ops / (ms * 1e-3) / 1e12
    return {"pair": [q, d], "ms_per_pair": round(ms, 4), "bound": "mfma", "achieved": round(tops, 1),
            "peak": 5000.0, "unit": "TOP/s (int8)", "frac": round(tops / 5000.0, 4)}


def run_grid(args):
    """The whole grid job through MBR schedules under residency caps."""
    import torch

    from paper_2505_22089_amd import chm, synth

    def say(m):
        print("[bench] " + m, file=sys.stderr, flush=True)

    rows, cols, nf = [int(v) for v in args.grid_shape.split(",")]
    say("generating grid %dx%d x %d" % (rows, cols, nf))
    wl = synth.config5(rows=rows, cols=cols, n_feats=nf, progress=say)
    n = len(wl.images)
    P = len(wl.pairs)
    feats = np.array([x.shape[0] for x in wl.images], np.int64)
    cfg = chm.config(L=wl.L, m=wl.m, K=wl.K, ratio=wl.ratio)
    sizes = [chm.image_bytes(cfg, int(f)) + 256 for f in feats]
    # descriptors in one pinned host buffer (DMA-able), one view per image
    total = int(feats.sum()) * 128
    pinned = torch.empty(total, dtype=torch.uint8, pin_memory=True)
    host = pinned.numpy()
    views, o = [], 0
    for x in wl.images:
        v = host[o:o + x.size].reshape(x.shape)
        v[...] = x
        views.append(v)
        o += x.size
    offs = np.zeros(P + 1, np.int64)
    offs[1:] = np.cumsum(feats[wl.pairs[:, 0]])
    dev = torch.device("cuda:0")
    out = torch.empty(int(offs[-1]), dtype=torch.int32, device=dev)
    runs = []
    for cap_gb in [float(c) for c in args.caps.split(",")]:
        cap = int(cap_gb * (1 << 30))
        t0 = time.perf_counter()
        sched = chm.schedule_mbr(n, wl.pairs, sizes, cap, args.size_blk, keep_handle=True)
        t_sched = time.perf_counter() - t0
        arena = torch.empty(chm.store_overhead_bytes(cfg) + cap + (256 << 20), dtype=torch.uint8, device=dev)
        store = chm.Store(cfg, wl.W, wl.mu, arena)
        torch.cuda.synchronize()
        say("cap %.0f GB: %d steps, %d iterations" % (cap_gb, len(sched.steps), sched.iterations))
        t0 = time.perf_counter()
        chm.run_schedule(store, sched, wl.pairs, views, offs, out)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = store.stats()
        runs.append({"cap_GB": cap_gb, "seconds": round(wall, 4), "pairs_per_s": round(P / wall, 1),
                     "h2d_bytes": int(st.h2d_bytes), "images_loaded": int(st.images_loaded),
                     "resident_peak_bytes": int(st.resident_peak), "steps": len(sched.steps),
                     "iterations": sched.iterations, "fallback_pairs": sched.fallback_pairs,
                     "mbr_dims": sched.dims, "schedule_seconds": round(t_sched, 3)})
        say("cap %.0f GB: %.3f s, %.0f pairs/s, %.2f GB H2D" % (cap_gb, wall, P / wall, st.h2d_bytes / 1e9))
        if args.grid_sao and cap_gb == float(args.caps.split(",")[0]):
            # the same schedule again, with the device SAO filter after each step
            store.close()
            store = chm.Store(cfg, wl.W, wl.mu, arena)
            kps = synth.keypoints(wl)
            d_kps = [torch.from_numpy(k).to(dev) for k in kps]
            filt = torch.empty_like(out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            work = chm.run_schedule_sao(store, sched, wl.pairs, views, offs, out, d_kps, filt)
            torch.cuda.synchronize()
            wall_s = time.perf_counter() - t0
            f = filt.cpu().numpy()
            m = out.cpu().numpy()
            runs[-1]["with_device_sao"] = {"seconds": round(wall_s, 4), "pairs_per_s": round(P / wall_s, 1),
                                           "matches": int((m >= 0).sum()), "kept": int((f >= 0).sum()),
                                           "input_errors": chm.sao_input_errors(work)}
            say("cap %.0f GB with SAO: %.3f s, %.0f pairs/s" % (cap_gb, wall_s, P / wall_s))
            del d_kps, work, filt
        if args.grid_verify and cap_gb == float(args.caps.split(",")[0]):
            # again, with RANSAC of every step on host threads beside the device
            store.close()
            store = chm.Store(cfg, wl.W, wl.mu, arena)
            kps = synth.keypoints(wl)
            d_kps = [torch.from_numpy(k).to(dev) for k in kps]
            filt = torch.empty_like(out)
            words = synth.ransac_words(P, 64)
            h_filt = torch.empty(int(offs[-1]), dtype=torch.int32, pin_memory=True).numpy()
            h_ver = np.empty(int(offs[-1]), np.int32)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            work = chm.run_schedule_verify(store, sched, wl.pairs, views, offs, out, d_kps, kps, filt, words,
                                           h_filt, h_ver, iterations=64, thr=64, min_inliers=8)
            torch.cuda.synchronize()
            wall_v = time.perf_counter() - t0
            runs[-1]["with_device_sao_host_ransac"] = {
                "seconds": round(wall_v, 4), "pairs_per_s": round(P / wall_v, 1),
                "matches": int((out.cpu().numpy() >= 0).sum()), "after_sao": int((h_filt >= 0).sum()),
                "verified": int((h_ver >= 0).sum()), "host_threads": os.cpu_count(),
                "ransac": "64 hypotheses, 4 px (64 units), at least 8 inliers",
                "input_errors": chm.sao_input_errors(work)}
            say("cap %.0f GB with SAO + RANSAC: %.3f s, %.0f pairs/s" % (cap_gb, wall_v, P / wall_v))
            # and with the RANSAC on the device too (the same words)
            store.close()
            store = chm.Store(cfg, wl.W, wl.mu, arena)
            d_ver = torch.empty_like(out)
            d_words = torch.from_numpy(words.view(np.int32)).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            work, rwork = chm.run_schedule_verify_device(store, sched, wl.pairs, views, offs, out, d_kps, filt, d_ver,
                                                         d_words, iterations=64, thr=64, min_inliers=8)
            torch.cuda.synchronize()
            wall_d = time.perf_counter() - t0
            dv = d_ver.cpu().numpy()
            runs[-1]["with_device_sao_device_ransac"] = {
                "seconds": round(wall_d, 4), "pairs_per_s": round(P / wall_d, 1), "verified": int((dv >= 0).sum()),
                "equals_host_ransac": bool(np.array_equal(dv, h_ver)),
                "input_errors": chm.sao_input_errors(work) + chm.sao_input_errors(rwork)}
            say("cap %.0f GB with SAO + device RANSAC: %.3f s, %.0f pairs/s" % (cap_gb, wall_d, P / wall_d))
            del d_kps, work, rwork, filt, h_filt, h_ver, d_ver, d_words
        chm.schedule_free(sched)
        store.close()
        del arena
        torch.cuda.empty_cache()
    # parity: every pair against the oracle's stored per-pair digests when
    # they exist for this grid (tests/golden/make_digests.py), and a sample
    # of pairs recomputed by the oracle
    got = out.cpu().numpy()
    name = "grid-%dx%d" % (rows * cols, nf)
    digests = None
    try:
        from tests.digests import load_golden, pair_digests
        dg, _, gp, _ = load_golden(name)
        if np.array_equal(gp, wl.pairs):
            digests = int((pair_digests(got, offs) == dg).sum())
    except (OSError, KeyError):
        pass
    from oracle import oracle as O
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(P, 12, replace=False))
    need = sorted({int(i) for i in wl.pairs[idx].ravel()})
    H = O.hash_workload(wl, need)
    ref, so, _, _ = O.match_pairs(H, wl.pairs[idx], wl.L, wl.m, wl.K, wl.ratio)
    same = all(np.array_equal(ref[so[k]:so[k + 1]], got[offs[p]:offs[p + 1]]) for k, p in enumerate(idx))
    # the schedule study last: its runs reuse the output buffer
    study = grid_study(args, wl, views, offs, sizes, cfg, out, say) if args.grid_study else None
    binding = runs[-1]
    res = {"metric": METRIC, "value": binding["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": round(binding["seconds"] * 1e3, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": describe(wl), "L": wl.L, "m": wl.m, "K": wl.K, "ratio": "%d/%d" % wl.ratio,
                      "size_blk": args.size_blk, "cap_GB": binding["cap_GB"],
                      "path": "MBR schedule: pinned host -> HBM per block row, hash + batched match"},
           "runs": runs, "h2d_floor_bytes": total,
           "naive_h2d_bytes": int(sum(feats[q] + feats[d] for q, d in wl.pairs) * 128),
           "oracle_identical_on_sampled_pairs": bool(same), "sampled_pairs": int(len(idx)),
           "pairs_matching_oracle_digests": digests, "pairs": P}
    if study is not None:
        res["schedule_study"] = study
    print(json.dumps(res), flush=True)


def grid_study(args, wl, views, offs, sizes, cfg, out, say):
    """Data schedules of Sec. 2.2 run through the same device path (pinned
    host memory -> HBM per step, hash, batched match, evict) at each study
    cap: MBR at several Size_blk, the load/free list (pairs in list order,
    least recently used images freed), the graph-partition part-pair
    schedule and, on the first --naive-pairs pairs, the per-pair schedule
    that loads both images of every pair.  Runs over all pairs are compared
    with the oracle digests pair by pair when they are stored."""
    import torch

    from paper_2505_22089_amd import chm
    from paper_2505_22089_amd import schedule_study as SS
    n, P = len(wl.images), len(wl.pairs)
    dev = out.device
    desc = [int(x.shape[0]) * 128 for x in wl.images]
    try:
        from tests.digests import load_golden, pair_digests
        dg, _, gp, _ = load_golden("grid-%dx%d" % (n, int(wl.images[0].shape[0])))
        if not np.array_equal(gp, wl.pairs):
            dg = None
    except (OSError, KeyError):
        dg = None
    rows = []
    for cap_gb in [float(c) for c in args.grid_study.split(",")]:
        cap = int(cap_gb * (1 << 30))
        runs = [("mbr", b) for b in [int(v) for v in args.study_blks.split(",")]]
        runs += [("load/free list", None), ("graph partition", None), ("per pair", None)]
        for kind, blk in runs:
            sub = wl.pairs if kind != "per pair" else wl.pairs[:args.naive_pairs]
            so = offs[:len(sub) + 1]
            t0 = time.perf_counter()
            if kind == "mbr":
                sched = chm.schedule_mbr(n, sub, sizes, cap, blk, keep_handle=True)
            elif kind == "load/free list":
                sched = chm.schedule_from_steps(n, sub, sizes, cap, SS.lru_steps(sub, sizes, cap))
            elif kind == "graph partition":
                sched = chm.schedule_from_steps(n, sub, sizes, cap, SS.partition_steps(n, sub, sizes, cap))
            else:
                sched = chm.schedule_from_steps(n, sub, sizes, cap, SS.naive_steps(sub))
            t_sched = time.perf_counter() - t0
            arena = torch.empty(chm.store_overhead_bytes(cfg) + cap + (256 << 20), dtype=torch.uint8, device=dev)
            store = chm.Store(cfg, wl.W, wl.mu, arena)
            out.fill_(-7)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chm.run_schedule(store, sched, sub, views, so, out)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = store.stats()
            row = {"cap_GB": cap_gb, "schedule": kind, "size_blk": blk, "pairs": int(len(sub)),
                   "seconds": round(wall, 4), "pairs_per_s": round(len(sub) / wall, 1),
                   "h2d_bytes": int(st.h2d_bytes), "h2d_over_floor": round(st.h2d_bytes / sum(desc), 3),
                   "steps": len(sched.steps), "schedule_seconds": round(t_sched, 3),
                   "resident_peak_bytes": int(st.resident_peak)}
            if kind == "mbr":
                row["mbr_dims"] = sched.dims
                row["iterations"] = sched.iterations
            if dg is not None:
                got = out.cpu().numpy()
                row["pairs_matching_oracle_digests"] = int((pair_digests(got[:int(so[-1])], so) ==
                                                            dg[:len(sub)]).sum())
            rows.append(row)
            say("study cap %.2f GB %s%s: %.3f s, %.0f pairs/s, H2D %.2f GB"
                % (cap_gb, kind, "" if blk is None else " blk %d" % blk, wall, len(sub) / wall, st.h2d_bytes / 1e9))
            chm.schedule_free(sched)
            store.close()
            del arena
            torch.cuda.empty_cache()
    return rows


def describe(wl):
    n = np.array([x.shape[0] for x in wl.images])
    m = wl.meta or {}
    return ("%s (%d images x %s SIFT-like u8 descriptors, %d directed pairs, %.0f%% mean overlap)"
            % (wl.name, len(n), ("%d" % n[0]) if n.min() == n.max() else "%d-%d" % (n.min(), n.max()),
               len(wl.pairs), 100 * m.get("overlap_mean", m.get("target_overlap", 0.0))))


def cpu_baseline_sampled(wl, gpu_out, offs, min_seconds=10.0):
    """The oracle on a random sample of pairs (their images hashed first),
    grown until about ten seconds of CPU work have run; hashing is scaled to
    all descriptors and matching to all pairs.  The sampled outputs are
    compared with the GPU's."""
    from oracle import oracle as O
    rng = np.random.default_rng(7)
    order = rng.permutation(len(wl.pairs))
    H = [None] * len(wl.images)
    t_hash = t_match = 0.0
    n_hashed = n_pairs = 0
    same = True
    for c in range(0, len(order), 8):
        idx = np.sort(order[c:c + 8])
        sub = wl.pairs[idx]
        need = sorted({int(i) for i in sub.ravel()} - {i for i in range(len(H)) if H[i] is not None})
        t0 = time.perf_counter()
        for i in need:
            H[i] = O.hash_image(wl.images[i], wl.W, wl.mu, wl.L, wl.m)
        t1 = time.perf_counter()
        out, so, _, _ = O.match_pairs(H, sub, wl.L, wl.m, wl.K, wl.ratio)
        t2 = time.perf_counter()
        t_hash += t1 - t0
        t_match += t2 - t1
        n_hashed += sum(wl.images[i].shape[0] for i in need)
        n_pairs += len(idx)
        for k, p in enumerate(idx):
            same = same and bool(np.array_equal(out[so[k]:so[k + 1]], gpu_out[offs[p]:offs[p + 1]]))
        if t_hash + t_match >= min_seconds:
            break
    n_desc = sum(x.shape[0] for x in wl.images)
    t_full = t_hash * n_desc / max(1, n_hashed) + t_match * len(wl.pairs) / max(1, n_pairs)
    return {"value": round(len(wl.pairs) / t_full, 3), "unit": "pairs/s", "cores": O.max_threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": "%d random pairs (%d images hashed, %.1f s; matching %.1f s), hashing scaled to "
                      "%d descriptors and matching to %d pairs" % (n_pairs, sum(h is not None for h in H),
                                                                   t_hash, t_match, n_desc, len(wl.pairs)),
            "gpu_identical_on_sample": same}


def cpu_model():
    """Host CPU model and the hardware threads the OS shows."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": name, "nproc": os.cpu_count()}


def copy_calibration():
    """A plain device copy of known size (256 MiB, three times), run under
    rocprofv3 --pmc to scale the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 256 << 20
    a = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


MATCH_SOURCES = ("bucket.hip", "chm_host.cpp", "chm_host.h", "chm_internal.h", "match.hip", "match_bm.hip",
                 "match_common.h")


def sources_digest():
    """sha256 over the sources that shape the match kernel and its data (its
    code, launch, work list and the bucket tables it reads): any change
    invalidates the recorded counters."""
    import hashlib
    d = os.path.join(ROOT, "paper_2505_22089_amd", "csrc")
    h = hashlib.sha256()
    for f in MATCH_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def recorded_traffic(workload):
    """HBM bytes per match launch of a workload from the committed counter
    summary, or None when the native sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "match_traffic_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("sources sha256") != sources_digest() or "hbm bytes per launch" not in rec:
        return None
    return float(rec["hbm bytes per launch"])


if __name__ == "__main__":
    main()

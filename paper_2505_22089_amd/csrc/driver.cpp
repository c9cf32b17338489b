// End-to-end run of an MBR schedule (Algorithm 1, CascadeHashingMatching):
// per block row, free what the row no longer needs, load the new images
// (descriptors host -> HBM, then codes and tables on the device) and match
// the row's pairs in one batched launch; optionally the row's matches then
// go through the SAO local constraint on the device (Sec. 2.3.3), on the
// same stream, so outlier removal keeps pace with the block rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "chm.h"
#include "chm_host.h"
#include "chm_internal.h"

using namespace chm;

namespace {

struct SaoStep {
  const int32_t* const* d_kp;
  int32_t nn, num, den;
  int32_t* d_filtered;
  void* d_work;
  uint64_t work_bytes;
};

// RANSAC of every step on the device, after its SAO on the same stream.
struct RansacStep {
  const uint32_t* d_words;
  int32_t iterations, thr, min_inliers;
  int32_t* d_verified;
  void* d_work;
  uint64_t work_bytes;
};

// RANSAC of every step on host threads, beside the device: the step's SAO
// output is copied to h_filtered (pinned host memory, laid out like d_out)
// on a stream of the worker's own once the step's device work ends, then
// RANSAC writes the step's verified matches to h_verified.
struct VerifyStep {
  const int32_t* const* h_kp;
  const uint32_t* h_words;
  int32_t iterations, thr, min_inliers, n_threads;
  int32_t* h_filtered;
  int32_t* h_verified;
};

// The worker thread: takes (step, event marking the end of its device
// work) in step order, copies the step's filtered rows (runs of adjacent
// output ranges, one copy each) and verifies its pairs.  The first error is
// kept; finish() waits for every queued step.
struct VerifyWorker {
  const VerifyStep* v;
  const int32_t* h_pairs;
  const int32_t* h_n_feats;
  const int64_t* h_offs;
  const int32_t* d_filtered;
  hipStream_t ds = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::pair<std::vector<int32_t>, hipEvent_t>> q;
  bool closing = false;
  std::string err;

  void run() {
    for (;;) {
      std::pair<std::vector<int32_t>, hipEvent_t> job;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return closing || !q.empty(); });
        if (q.empty()) return;
        job = std::move(q.front());
        q.pop_front();
      }
      std::vector<int32_t>& pp = job.first;
      std::string e;
      if (hipStreamWaitEvent(ds, job.second, 0) != hipSuccess) e = "verify: stream wait failed";
      std::vector<int32_t> by(pp);
      std::sort(by.begin(), by.end(), [&](int32_t a, int32_t b) { return h_offs[a] < h_offs[b]; });
      for (size_t i = 0; e.empty() && i < by.size();) {
        const int64_t s0 = h_offs[by[i]];
        int64_t s1 = s0 + h_n_feats[h_pairs[2 * by[i]]];
        size_t j = i + 1;
        while (j < by.size() && h_offs[by[j]] == s1) s1 += h_n_feats[h_pairs[2 * by[j++]]];
        if (s1 > s0 && hipMemcpyAsync(v->h_filtered + s0, d_filtered + s0, (size_t)(s1 - s0) * 4,
                                      hipMemcpyDeviceToHost, ds) != hipSuccess)
          e = "verify: copy failed";
        i = j;
      }
      if (e.empty() && hipStreamSynchronize(ds) != hipSuccess) e = "verify: step's device work failed";
      (void)hipEventDestroy(job.second);
      if (e.empty() && !pp.empty())
        e = ransac_pairs((int32_t)pp.size(), pp.data(), h_pairs, v->h_kp, h_n_feats, h_offs, v->h_filtered,
                         v->h_words, v->iterations, v->thr, v->min_inliers, v->n_threads, v->h_verified);
      if (!e.empty()) {
        std::lock_guard<std::mutex> lk(mu);
        if (err.empty()) err = e;
      }
    }
  }
  void push(std::vector<int32_t> pp, hipEvent_t ev) {
    {
      std::lock_guard<std::mutex> lk(mu);
      q.emplace_back(std::move(pp), ev);
    }
    cv.notify_one();
  }
  void finish() {
    if (!th.joinable()) return;
    {
      std::lock_guard<std::mutex> lk(mu);
      closing = true;
    }
    cv.notify_one();
    th.join();
  }
  ~VerifyWorker() {
    finish();
    for (auto& j : q) (void)hipEventDestroy(j.second);
    if (ds) (void)hipStreamDestroy(ds);
  }
};

// What queued work may still read: the plans of the last two steps and the
// slots evicted at them, with the events that mark each step's end on the
// compute stream; and the copy stream with its per-step events.  On the way
// out (normal or not) both streams are drained before anything is freed.
using Held = std::vector<std::pair<uint64_t, uint64_t>>;
struct InFlight {
  chm_store* S;
  hipStream_t s, xs = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr}, cev[2] = {nullptr, nullptr};
  chm_plan* pl[2] = {nullptr, nullptr};
  Held held[2];
  InFlight(chm_store* st, hipStream_t cs) : S(st), s(cs) {}
  ~InFlight() {
    (void)hipStreamSynchronize(s);
    if (xs) (void)hipStreamSynchronize(xs);
    for (int i = 0; i < 2; ++i) {
      plan_free(pl[i]);
      release_held(S, &held[i]);
    }
    for (hipEvent_t e : {ev[0], ev[1], cev[0], cev[1]})
      if (e) (void)hipEventDestroy(e);
    if (xs) (void)hipStreamDestroy(xs);
  }
};

chm_status run_schedule(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs, int32_t P,
                        const void* const* h_descs, const int32_t* h_n_feats, const int64_t* h_offs,
                        int32_t* d_out, void* stream, const SaoStep* sao, const VerifyStep* verify = nullptr,
                        const RansacStep* ransac = nullptr) {
  if (!S || !sc) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (P < 0 || (P && (!h_pairs || !h_offs)) || !h_descs || !h_n_feats)
    return fail(CHM_E_INVALID_ARG, "bad arguments");
  const int nsteps = chm_schedule_num_steps(sc);
  // The schedule's pairs in step order: step k matches entries
  // first[k] .. first[k+1]-1 of (sp, starts).
  std::vector<int32_t> sp, first(nsteps + 1, 0), rows(nsteps, 1), orig;
  std::vector<int64_t> starts;
  for (int k = 0; k < nsteps; ++k) {
    const int32_t *ev, *ld, *pp;
    int32_t nev, nld, npp;
    chm_status st = chm_schedule_step(sc, k, &ev, &nev, &ld, &nld, &pp, &npp);
    if (st) return st;
    for (int i = 0; i < npp; ++i) {
      const int p = pp[i];
      if (p < 0 || p >= P) return fail(CHM_E_INVALID_ARG, "schedule names pair %d of %d", p, P);
      sp.push_back(h_pairs[2 * p]);
      sp.push_back(h_pairs[2 * p + 1]);
      starts.push_back(h_offs[p]);
      orig.push_back(p);
      rows[k] = std::max(rows[k], h_n_feats[h_pairs[2 * p]]);
    }
    first[k + 1] = (int32_t)starts.size();
  }
  const int32_t total = first[nsteps];
  hipStream_t s = (hipStream_t)stream;
  if (sao && total > 0) {
    const int32_t n_max = *std::max_element(rows.begin(), rows.end());
    if (sao->work_bytes < sao_work_bytes(total, n_max)) return fail(CHM_E_CAPACITY, "SAO work buffer too small");
    const hipError_t e = sao_upload(total, sp.data(), sao->d_kp, h_n_feats, starts.data(), sao->d_work, s);
    if (e != hipSuccess) return fail(CHM_E_HIP, "SAO pair table upload failed: %s", hipGetErrorString(e));
  }
  if (ransac && total > 0) {
    const int32_t n_max = *std::max_element(rows.begin(), rows.end());
    if (ransac->work_bytes < ransac_work_bytes(total, n_max))
      return fail(CHM_E_CAPACITY, "RANSAC work buffer too small");
    const hipError_t e =
        ransac_upload(total, sp.data(), sao->d_kp, h_n_feats, starts.data(), orig.data(), ransac->d_work, s);
    if (e != hipSuccess) return fail(CHM_E_HIP, "RANSAC pair table upload failed: %s", hipGetErrorString(e));
  }
  // Two streams: descriptor copies on xs, everything else on the caller's
  // stream s.  The host queues step k+1 while the device runs step k:
  // - step k+1's images are copied on xs into arena memory that no queued
  //   kernel reads: memory that was free when the call began (xs first waits
  //   for s, so work queued before the call is done), or released once the
  //   host has seen the step that last read it end;
  // - the slots evicted at step k+1 were last read by step k, so they are
  //   held until step k's end event; when the arena has no other room for
  //   step k+1's images, the host waits for that event and frees them first;
  // - s waits for step k+1's copies before it hashes the new images.
  // declared before the streams and plans it reads, so it is joined first
  VerifyWorker vw;
  if (verify) {
    vw.v = verify;
    vw.h_pairs = h_pairs;
    vw.h_n_feats = h_n_feats;
    vw.h_offs = h_offs;
    vw.d_filtered = sao->d_filtered;
    if (hipStreamCreateWithFlags(&vw.ds, hipStreamNonBlocking) != hipSuccess)
      return fail(CHM_E_HIP, "stream creation failed");
    vw.th = std::thread([&vw] { vw.run(); });
  }
  InFlight fl(S, s);
  if (hipStreamCreateWithFlags(&fl.xs, hipStreamNonBlocking) != hipSuccess)
    return fail(CHM_E_HIP, "stream creation failed");
  for (hipEvent_t* e : {&fl.ev[0], &fl.ev[1], &fl.cev[0], &fl.cev[1]})
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
      return fail(CHM_E_HIP, "event creation failed");
  if (hipEventRecord(fl.cev[1], s) != hipSuccess || hipStreamWaitEvent(fl.xs, fl.cev[1], 0) != hipSuccess)
    return fail(CHM_E_HIP, "stream ordering failed");
  for (int k = 0; k < nsteps; ++k) {
    const int cur = k & 1;
    // When the arena has no room left for step k, wait for step k-1's end
    // and free its plan and the slots evicted at step k: the state in which
    // a driver without look-ahead would allocate.  CHM_E_CAPACITY when
    // nothing is left to free.
    auto make_room = [&]() -> chm_status {
      if (fl.held[cur].empty() && !fl.pl[cur ^ 1]) return CHM_E_CAPACITY;
      if (k > 0) {
        const hipError_t e = hipEventSynchronize(fl.ev[cur ^ 1]);
        if (e != hipSuccess) return fail(CHM_E_HIP, "schedule step %d failed: %s", k - 1, hipGetErrorString(e));
      }
      plan_free(fl.pl[cur ^ 1]);
      fl.pl[cur ^ 1] = nullptr;
      release_held(S, &fl.held[cur]);
      clear_error();
      return CHM_OK;
    };
    const int32_t *ev, *ld, *pp;
    int32_t nev, nld, npp;
    chm_status st = chm_schedule_step(sc, k, &ev, &nev, &ld, &nld, &pp, &npp);
    if (st) return st;
    std::vector<int32_t> evict;
    for (int i = 0; i < nev; ++i)
      if (S->images.count(ev[i])) evict.push_back(ev[i]);
    st = evict_hold(S, (int32_t)evict.size(), evict.data(), &fl.held[cur]);
    if (st) return st;
    std::vector<int32_t> ids, nf;
    std::vector<const void*> ds;
    for (int i = 0; i < nld; ++i) {
      if (S->images.count(ld[i])) continue;
      ids.push_back(ld[i]);
      ds.push_back(h_descs[ld[i]]);
      nf.push_back(h_n_feats[ld[i]]);
    }
    const int32_t nl = (int32_t)ids.size();
    if (nl > 0) {
      st = load_check(S, nl, ids.data(), ds.data(), nf.data());
      if (st) return st;
      std::vector<ImageSlot> slots;
      st = load_alloc(S, nl, ids.data(), nf.data(), &slots);
      if (st == CHM_E_CAPACITY) {
        const std::string why = chm_last_error();
        const chm_status r = make_room();
        if (r == CHM_E_CAPACITY) return fail(CHM_E_CAPACITY, "%s", why.c_str());
        if (r) return r;
        st = load_alloc(S, nl, ids.data(), nf.data(), &slots);
      }
      if (st) return st;
      std::vector<const ImageSlot*> ptrs;
      st = load_commit(S, nl, ids.data(), ds.data(), slots, false, fl.xs, &ptrs);
      if (st) return st;
      if (hipEventRecord(fl.cev[cur], fl.xs) != hipSuccess || hipStreamWaitEvent(s, fl.cev[cur], 0) != hipSuccess)
        return fail(CHM_E_HIP, "stream ordering failed");
      st = hash_images(S, ptrs, s);
      if (st) return st;
    }
    const int32_t f = first[k], n = first[k + 1] - first[k];
    st = plan_build(S, sp.data() + 2 * (size_t)f, n, starts.data() + f, d_out, nullptr, CHM_MATCH_BATCHED,
                    stream, &fl.pl[cur], false);
    if (st == CHM_E_CAPACITY) {
      const std::string why = chm_last_error();
      const chm_status r = make_room();
      if (r == CHM_E_CAPACITY) return fail(CHM_E_CAPACITY, "%s", why.c_str());
      if (r) return r;
      st = plan_build(S, sp.data() + 2 * (size_t)f, n, starts.data() + f, d_out, nullptr, CHM_MATCH_BATCHED,
                      stream, &fl.pl[cur], false);
    }
    if (st) return st;
    st = chm_plan_execute(fl.pl[cur], stream);
    if (st) return st;
    if (sao && n > 0) {
      const hipError_t e = sao_run(f, n, total, rows[k], d_out, sao->nn, sao->num, sao->den, sao->d_filtered,
                                   nullptr, sao->d_work, s);
      if (e != hipSuccess) return fail(CHM_E_HIP, "SAO launch failed: %s", hipGetErrorString(e));
    }
    if (ransac && n > 0) {
      const hipError_t e = ransac_run(f, n, total, rows[k], sao->d_filtered, ransac->d_words, ransac->iterations,
                                      ransac->thr, ransac->min_inliers, ransac->d_verified, nullptr,
                                      ransac->d_work, s);
      if (e != hipSuccess) return fail(CHM_E_HIP, "RANSAC launch failed: %s", hipGetErrorString(e));
    }
    if (verify && n > 0) {
      hipEvent_t ve = nullptr;
      if (hipEventCreateWithFlags(&ve, hipEventDisableTiming) != hipSuccess || hipEventRecord(ve, s) != hipSuccess) {
        if (ve) (void)hipEventDestroy(ve);
        return fail(CHM_E_HIP, "event record failed");
      }
      vw.push(std::vector<int32_t>(pp, pp + npp), ve);
    }
    if (hipEventRecord(fl.ev[cur], s) != hipSuccess) return fail(CHM_E_HIP, "event record failed");
    // Step k-1 has ended: its plan and the slots evicted at step k (last
    // read by step k-1) are free.
    if (k > 0) {
      const hipError_t e = hipEventSynchronize(fl.ev[cur ^ 1]);
      if (e != hipSuccess) return fail(CHM_E_HIP, "schedule step %d failed: %s", k - 1, hipGetErrorString(e));
      plan_free(fl.pl[cur ^ 1]);
      fl.pl[cur ^ 1] = nullptr;
      release_held(S, &fl.held[cur ^ 1]);
    }
    release_held(S, &fl.held[cur]);
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHM_E_HIP, "schedule run failed: %s", hipGetErrorString(e));
  if (verify) {
    vw.finish();
    if (!vw.err.empty()) return fail(CHM_E_INVALID_ARG, "%s", vw.err.c_str());
  }
  return CHM_OK;
}

}  // namespace

extern "C" chm_status chm_run_schedule(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs,
                                       int32_t P, const void* const* h_descs, const int32_t* h_n_feats,
                                       const int64_t* h_offs, int32_t* d_out, void* stream) {
  clear_error();
  return run_schedule(S, sc, h_pairs, P, h_descs, h_n_feats, h_offs, d_out, stream, nullptr);
}

static chm_status run_schedule_sao(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs, int32_t P,
                                   const void* const* h_descs, const int32_t* h_n_feats, int32_t n_images,
                                   const int64_t* h_offs, int32_t* d_out, const int32_t* const* d_kp,
                                   int32_t n_neighbors, int32_t score_num, int32_t score_den, int32_t* d_filtered,
                                   void* d_work, uint64_t work_bytes, void* stream, const VerifyStep* verify,
                                   const RansacStep* ransac = nullptr) {
  if (!d_kp || !h_n_feats || !d_filtered || !d_work || d_filtered == d_out)
    return fail(CHM_E_INVALID_ARG, "bad SAO buffers");
  if (n_neighbors < 1 || n_neighbors > kSaoMaxNeighbors)
    return fail(CHM_E_INVALID_ARG, "n_neighbors must be 1..%d on the device", kSaoMaxNeighbors);
  if (score_num < 0 || score_den <= 0) return fail(CHM_E_INVALID_ARG, "bad score threshold");
  if (reinterpret_cast<uintptr_t>(d_work) % 256) return fail(CHM_E_INVALID_ARG, "d_work must be 256-byte aligned");
  int32_t n_max = 0;
  for (int32_t p = 0; p < P; ++p) {
    const int32_t q = h_pairs ? h_pairs[2 * p] : -1, d = h_pairs ? h_pairs[2 * p + 1] : -1;
    if (q < 0 || q >= n_images || d < 0 || d >= n_images)
      return fail(CHM_E_INVALID_ARG, "pair %d names an image outside 0..%d", p, n_images - 1);
    if ((h_n_feats[q] > 0 && !d_kp[q]) || (h_n_feats[d] > 0 && !d_kp[d]))
      return fail(CHM_E_INVALID_ARG, "pair %d: NULL keypoints", p);
    if (verify && ((h_n_feats[q] > 0 && !verify->h_kp[q]) || (h_n_feats[d] > 0 && !verify->h_kp[d])))
      return fail(CHM_E_INVALID_ARG, "pair %d: NULL host keypoints", p);
    n_max = std::max(n_max, h_n_feats[q]);
  }
  if (work_bytes < sao_work_bytes(P, n_max)) return fail(CHM_E_CAPACITY, "SAO work buffer too small");
  const hipError_t e = launch_fill_u32(static_cast<uint32_t*>(d_work), 0u, 1, (hipStream_t)stream);
  if (e != hipSuccess) return fail(CHM_E_HIP, "%s", hipGetErrorString(e));
  if (ransac) {
    if (!ransac->d_verified || !ransac->d_work || (ransac->iterations > 0 && !ransac->d_words))
      return fail(CHM_E_INVALID_ARG, "bad RANSAC buffers");
    if (ransac->iterations < 0 || ransac->thr < 0 || ransac->thr >= (1 << 20))
      return fail(CHM_E_INVALID_ARG, "bad RANSAC parameters");
    if (reinterpret_cast<uintptr_t>(ransac->d_work) % 256)
      return fail(CHM_E_INVALID_ARG, "d_rwork must be 256-byte aligned");
    if (ransac->work_bytes < ransac_work_bytes(P, n_max)) return fail(CHM_E_CAPACITY, "RANSAC work buffer too small");
    const hipError_t e = launch_fill_u32(static_cast<uint32_t*>(ransac->d_work), 0u, 1, (hipStream_t)stream);
    if (e != hipSuccess) return fail(CHM_E_HIP, "%s", hipGetErrorString(e));
  }
  const SaoStep sao{d_kp, n_neighbors, score_num, score_den, d_filtered, d_work, work_bytes};
  return run_schedule(S, sc, h_pairs, P, h_descs, h_n_feats, h_offs, d_out, stream, &sao, verify, ransac);
}

extern "C" chm_status chm_run_schedule_sao(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs,
                                           int32_t P, const void* const* h_descs, const int32_t* h_n_feats,
                                           int32_t n_images, const int64_t* h_offs, int32_t* d_out,
                                           const int32_t* const* d_kp, int32_t n_neighbors, int32_t score_num,
                                           int32_t score_den, int32_t* d_filtered, void* d_work,
                                           uint64_t work_bytes, void* stream) {
  clear_error();
  return run_schedule_sao(S, sc, h_pairs, P, h_descs, h_n_feats, n_images, h_offs, d_out, d_kp, n_neighbors,
                          score_num, score_den, d_filtered, d_work, work_bytes, stream, nullptr);
}

extern "C" chm_status chm_run_schedule_verify(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs,
                                              int32_t P, const void* const* h_descs, const int32_t* h_n_feats,
                                              int32_t n_images, const int64_t* h_offs, int32_t* d_out,
                                              const int32_t* const* d_kp, int32_t n_neighbors, int32_t score_num,
                                              int32_t score_den, int32_t* d_filtered, void* d_work,
                                              uint64_t work_bytes, const int32_t* const* h_kp,
                                              const uint32_t* h_words, int32_t iterations, int32_t thr,
                                              int32_t min_inliers, int32_t n_threads, int32_t* h_filtered,
                                              int32_t* h_verified, void* stream) {
  clear_error();
  if (!h_kp || !h_filtered || !h_verified || (iterations > 0 && !h_words) || h_filtered == h_verified)
    return fail(CHM_E_INVALID_ARG, "bad RANSAC buffers");
  if (iterations < 0) return fail(CHM_E_INVALID_ARG, "negative iterations");
  if (thr < 0 || thr >= (1 << 20)) return fail(CHM_E_INVALID_ARG, "thr must be 0..2^20-1");
  const VerifyStep v{h_kp, h_words, iterations, thr, min_inliers, n_threads, h_filtered, h_verified};
  return run_schedule_sao(S, sc, h_pairs, P, h_descs, h_n_feats, n_images, h_offs, d_out, d_kp, n_neighbors,
                          score_num, score_den, d_filtered, d_work, work_bytes, stream, &v);
}

extern "C" chm_status chm_run_schedule_verify_device(
    chm_store* S, const chm_schedule* sc, const int32_t* h_pairs, int32_t P, const void* const* h_descs,
    const int32_t* h_n_feats, int32_t n_images, const int64_t* h_offs, int32_t* d_out, const int32_t* const* d_kp,
    int32_t n_neighbors, int32_t score_num, int32_t score_den, int32_t* d_filtered, void* d_work,
    uint64_t work_bytes, const uint32_t* d_words, int32_t iterations, int32_t thr, int32_t min_inliers,
    int32_t* d_verified, void* d_rwork, uint64_t rwork_bytes, void* stream) {
  clear_error();
  const RansacStep r{d_words, iterations, thr, min_inliers, d_verified, d_rwork, rwork_bytes};
  return run_schedule_sao(S, sc, h_pairs, P, h_descs, h_n_feats, n_images, h_offs, d_out, d_kp, n_neighbors,
                          score_num, score_den, d_filtered, d_work, work_bytes, stream, nullptr, &r);
}

extern "C" chm_status chm_bruteforce_work_bytes(int32_t nq, int32_t nd, uint64_t* out) {
  clear_error();
  if (!out || nq < 0 || nd < 0 || nq >= (1 << 24) || nd >= (1 << 24))
    return fail(CHM_E_INVALID_ARG, "bad arguments");
  const uint64_t b = bruteforce_work_bytes(nq, nd);
  *out = b < 256 ? 256 : b;
  return CHM_OK;
}

extern "C" chm_status chm_bruteforce(const uint8_t* d_q, int32_t nq, const uint8_t* d_d, int32_t nd,
                                     int32_t ra, int32_t rb, int32_t* d_out, void* d_work,
                                     uint64_t work_bytes, void* stream) {
  clear_error();
  uint64_t need = 0;
  chm_status st = chm_bruteforce_work_bytes(nq, nd, &need);
  if (st) return st;
  if (ra <= 0 || rb <= 0 || ra > rb || rb > 46340)
    return fail(CHM_E_INVALID_ARG, "ratio must satisfy 0 < num <= den <= 46340");
  if (nq > 0 && (!d_q || !d_out || !d_work)) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (nd > 0 && !d_d) return fail(CHM_E_INVALID_ARG, "NULL db descriptors");
  if (work_bytes < need) return fail(CHM_E_CAPACITY, "workspace needs %llu bytes", (unsigned long long)need);
  if (((uintptr_t)d_q | (uintptr_t)d_d | (uintptr_t)d_work) % 16)
    return fail(CHM_E_INVALID_ARG, "buffers must be 16-byte aligned");
  hipError_t e = launch_bruteforce(d_q, nq, d_d, nd, ra, rb, d_out, d_work, bruteforce_splits(nq, nd),
                                   (hipStream_t)stream);
  if (e != hipSuccess) return fail(CHM_E_HIP, "brute force launch failed: %s", hipGetErrorString(e));
  return CHM_OK;
}

extern "C" chm_status chm_bruteforce_noalloc(const uint8_t* d_q, int32_t nq, const uint8_t* d_d, int32_t nd,
                                             int32_t ra, int32_t rb, int32_t* d_out, void* stream) {
  clear_error();
  uint64_t need = 0;
  chm_status st = chm_bruteforce_work_bytes(nq, nd, &need);
  if (st) return st;
  if (need > kBfScratchBytes)
    return fail(CHM_E_CAPACITY,
                "brute force of %d x %d descriptors needs %llu bytes of workspace, beyond the %llu-byte "
                "library workspace (use chm_bruteforce with a caller workspace)",
                nq, nd, (unsigned long long)need, (unsigned long long)kBfScratchBytes);
  if (ra <= 0 || rb <= 0 || ra > rb || rb > 46340)
    return fail(CHM_E_INVALID_ARG, "ratio must satisfy 0 < num <= den <= 46340");
  if (nq > 0 && (!d_q || !d_out)) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (nd > 0 && !d_d) return fail(CHM_E_INVALID_ARG, "NULL db descriptors");
  if (((uintptr_t)d_q | (uintptr_t)d_d) % 16) return fail(CHM_E_INVALID_ARG, "buffers must be 16-byte aligned");
  void* work = nullptr;
  hipError_t e = bruteforce_scratch(&work);
  if (e != hipSuccess) return fail(CHM_E_HIP, "library workspace lookup failed: %s", hipGetErrorString(e));
  e = launch_bruteforce(d_q, nq, d_d, nd, ra, rb, d_out, work, bruteforce_splits(nq, nd), (hipStream_t)stream);
  if (e != hipSuccess) return fail(CHM_E_HIP, "brute force launch failed: %s", hipGetErrorString(e));
  return CHM_OK;
}

// End-to-end run of an MBR schedule (Algorithm 1, CascadeHashingMatching):
// per block row, free what the row no longer needs, load the new images
// (descriptors host -> HBM, then codes and tables on the device) and match
// the row's pairs in one batched launch; optionally the row's matches then
// go through the SAO local constraint on the device (Sec. 2.3.3), on the
// same stream, so outlier removal keeps pace with the block rows.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// Plans still read by queued work, and the events that mark their ends.  On
// the way out (normal or not) the stream is drained before anything is freed.
struct InFlight {
  hipStream_t s;
  hipEvent_t ev[2] = {nullptr, nullptr};
  chm_plan* pl[2] = {nullptr, nullptr};
  explicit InFlight(hipStream_t st) : s(st) {}
  ~InFlight() {
    if (pl[0] || pl[1]) (void)hipStreamSynchronize(s);
    plan_free(pl[0]);
    plan_free(pl[1]);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

chm_status run_schedule(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs, int32_t P,
                        const void* const* h_descs, const int32_t* h_n_feats, const int64_t* h_offs,
                        int32_t* d_out, void* stream, const SaoStep* sao) {
  if (!S || !sc) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (P < 0 || (P && (!h_pairs || !h_offs)) || !h_descs || !h_n_feats)
    return fail(CHM_E_INVALID_ARG, "bad arguments");
  const int nsteps = chm_schedule_num_steps(sc);
  // The schedule's pairs in step order: step k matches entries
  // first[k] .. first[k+1]-1 of (sp, starts).
  std::vector<int32_t> sp, first(nsteps + 1, 0), rows(nsteps, 1);
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
  // The host runs one step ahead of the device: while step k runs, it queues
  // step k+1 (evictions are host bookkeeping; the stream orders a reused
  // slot's new copy after the kernels that read its old image), then waits
  // for step k's end before it frees step k's plan.
  InFlight fl(s);
  for (int i = 0; i < 2; ++i)
    if (hipEventCreateWithFlags(&fl.ev[i], hipEventDisableTiming) != hipSuccess)
      return fail(CHM_E_HIP, "event creation failed");
  for (int k = 0; k < nsteps; ++k) {
    const int32_t *ev, *ld, *pp;
    int32_t nev, nld, npp;
    chm_status st = chm_schedule_step(sc, k, &ev, &nev, &ld, &nld, &pp, &npp);
    if (st) return st;
    std::vector<int32_t> evict;
    for (int i = 0; i < nev; ++i)
      if (S->images.count(ev[i])) evict.push_back(ev[i]);
    st = chm_store_evict(S, (int32_t)evict.size(), evict.data());
    if (st) return st;
    std::vector<int32_t> ids, nf;
    std::vector<const void*> ds;
    for (int i = 0; i < nld; ++i) {
      if (S->images.count(ld[i])) continue;
      ids.push_back(ld[i]);
      ds.push_back(h_descs[ld[i]]);
      nf.push_back(h_n_feats[ld[i]]);
    }
    st = chm_store_load(S, (int32_t)ids.size(), ids.data(), ds.data(), nf.data(), 0, stream);
    if (st) return st;
    const int cur = k & 1;
    const int32_t f = first[k], n = first[k + 1] - first[k];
    st = plan_build(S, sp.data() + 2 * (size_t)f, n, starts.data() + f, d_out, nullptr, CHM_MATCH_BATCHED,
                    stream, &fl.pl[cur], false);
    if (st) return st;
    st = chm_plan_execute(fl.pl[cur], stream);
    if (st) return st;
    if (sao && n > 0) {
      const hipError_t e = sao_run(f, n, total, rows[k], d_out, sao->nn, sao->num, sao->den, sao->d_filtered,
                                   nullptr, sao->d_work, s);
      if (e != hipSuccess) return fail(CHM_E_HIP, "SAO launch failed: %s", hipGetErrorString(e));
    }
    if (hipEventRecord(fl.ev[cur], s) != hipSuccess) return fail(CHM_E_HIP, "event record failed");
    if (fl.pl[cur ^ 1]) {
      const hipError_t e = hipEventSynchronize(fl.ev[cur ^ 1]);
      if (e != hipSuccess) return fail(CHM_E_HIP, "schedule step %d failed: %s", k - 1, hipGetErrorString(e));
      plan_free(fl.pl[cur ^ 1]);
      fl.pl[cur ^ 1] = nullptr;
    }
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHM_E_HIP, "schedule run failed: %s", hipGetErrorString(e));
  return CHM_OK;
}

}  // namespace

extern "C" chm_status chm_run_schedule(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs,
                                       int32_t P, const void* const* h_descs, const int32_t* h_n_feats,
                                       const int64_t* h_offs, int32_t* d_out, void* stream) {
  clear_error();
  return run_schedule(S, sc, h_pairs, P, h_descs, h_n_feats, h_offs, d_out, stream, nullptr);
}

extern "C" chm_status chm_run_schedule_sao(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs,
                                           int32_t P, const void* const* h_descs, const int32_t* h_n_feats,
                                           int32_t n_images, const int64_t* h_offs, int32_t* d_out,
                                           const int32_t* const* d_kp, int32_t n_neighbors, int32_t score_num,
                                           int32_t score_den, int32_t* d_filtered, void* d_work,
                                           uint64_t work_bytes, void* stream) {
  clear_error();
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
    n_max = std::max(n_max, h_n_feats[q]);
  }
  if (work_bytes < sao_work_bytes(P, n_max)) return fail(CHM_E_CAPACITY, "SAO work buffer too small");
  const hipError_t e = launch_fill_u32(static_cast<uint32_t*>(d_work), 0u, 1, (hipStream_t)stream);
  if (e != hipSuccess) return fail(CHM_E_HIP, "%s", hipGetErrorString(e));
  const SaoStep sao{d_kp, n_neighbors, score_num, score_den, d_filtered, d_work, work_bytes};
  return run_schedule(S, sc, h_pairs, P, h_descs, h_n_feats, h_offs, d_out, stream, &sao);
}

extern "C" chm_status chm_bruteforce_work_bytes(int32_t nq, int32_t nd, uint64_t* out) {
  clear_error();
  if (!out || nq < 0 || nd < 0 || nq >= (1 << 24) || nd >= (1 << 24))
    return fail(CHM_E_INVALID_ARG, "bad arguments");
  const uint64_t b = (uint64_t)bruteforce_splits(nq, nd) * (uint64_t)nq * 16u;
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

// End-to-end run of an MBR schedule (Algorithm 1, CascadeHashingMatching):
// per block row, free what the row no longer needs, load the new images
// (descriptors host -> HBM, then codes and tables on the device) and match
// the row's pairs in one batched launch.
#include <hip/hip_runtime.h>

#include <vector>

#include "chm.h"
#include "chm_host.h"

using namespace chm;

extern "C" chm_status chm_run_schedule(chm_store* S, const chm_schedule* sc, const int32_t* h_pairs,
                                       int32_t P, const void* const* h_descs, const int32_t* h_n_feats,
                                       const int64_t* h_offs, int32_t* d_out, void* stream) {
  clear_error();
  if (!S || !sc) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (P < 0 || (P && (!h_pairs || !h_offs)) || !h_descs || !h_n_feats)
    return fail(CHM_E_INVALID_ARG, "bad arguments");
  const int nsteps = chm_schedule_num_steps(sc);
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
    std::vector<int32_t> sp;
    std::vector<int64_t> starts;
    for (int i = 0; i < npp; ++i) {
      const int p = pp[i];
      if (p < 0 || p >= P) return fail(CHM_E_INVALID_ARG, "schedule names pair %d of %d", p, P);
      sp.push_back(h_pairs[2 * p]);
      sp.push_back(h_pairs[2 * p + 1]);
      starts.push_back(h_offs[p]);
    }
    chm_plan* pl = nullptr;
    st = plan_build(S, sp.data(), npp, starts.data(), d_out, nullptr, CHM_MATCH_BATCHED, stream, &pl);
    if (st) return st;
    st = chm_plan_execute(pl, stream);
    chm_plan_destroy(pl);
    if (st) return st;
  }
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(CHM_E_HIP, "schedule run failed: %s", hipGetErrorString(e));
  return CHM_OK;
}

extern "C" chm_status chm_bruteforce_work_bytes(int32_t nq, int32_t nd, uint64_t* out) {
  clear_error();
  if (!out || nq < 0 || nd < 0) return fail(CHM_E_INVALID_ARG, "bad arguments");
  *out = 256;
  return CHM_OK;
}

extern "C" chm_status chm_bruteforce(const uint8_t*, int32_t, const uint8_t*, int32_t, int32_t,
                                     int32_t, int32_t*, void*, uint64_t, void*) {
  return fail(CHM_E_UNSUPPORTED, "brute force not built yet");
}

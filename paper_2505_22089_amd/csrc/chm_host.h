// Host-side internals of libchm (store, arena, plans).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "chm.h"
#include "chm_internal.h"

namespace chm {

chm_status fail(chm_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
// True when the test hook (chm_debug_fail_hip) says this checked HIP call
// is to fail without being made.
bool hip_fault_due();

// First-fit sub-allocator over [0, size) of the caller's arena, 256-byte granules.
struct Arena {
  std::map<uint64_t, uint64_t> free_;  // offset -> bytes
  bool alloc(uint64_t bytes, uint64_t* off);
  void release(uint64_t off, uint64_t bytes);
};



struct ImageSlot {
  uint64_t off = 0;
  uint64_t bytes = 0;
  int32_t n = 0;
  uint64_t gen = 0;
};

}  // namespace chm

struct chm_store {
  chm_config cfg;
  int R = 0;
  int nb = 0;
  uint8_t* base = nullptr;
  uint64_t size = 0;
  chm::Arena arena;
  uint16_t* dW = nullptr;
  float* dTau = nullptr;
  double* dCmu = nullptr;
  uint8_t* dMu = nullptr;
  unsigned long long* dFix = nullptr;
  uint32_t* dFixList = nullptr;
  std::unordered_map<int32_t, chm::ImageSlot> images;
  uint64_t gen_counter = 0;
  chm_stats stats;
  chm_tuning tuning;
  int n_cu = 0;
  int n_xcd = 1;  // XCDs of the device (work-groups are dealt to them round-robin)
  int lds_top = 0;  // byte address of the match kernel's LDS control words
  int device = 0;
  hipStream_t cap_stream = nullptr;
};

struct chm_plan {
  chm_store* st = nullptr;
  int mode = 0;
  int n_pairs = 0;
  int n_items = 0;
  int n_bins = 1;
  bool lds_launch = false;                 // batched: the launch stages codes in LDS
  int32_t bins[chm::kMaxBins + 1] = {};    // item offsets of the bins
  int lds_max = 0;
  int32_t* out = nullptr;
  uint32_t* topk = nullptr;
  std::vector<std::pair<int32_t, uint64_t>> gens;
  uint64_t mem_off = 0, mem_bytes = 0;
  chm::PairDev* dPairs = nullptr;
  chm::WorkItem* dItems = nullptr;
  uint32_t* dQueue = nullptr;  // kMaxBins dequeue counters, one per bin
  int32_t* dBins = nullptr;    // kMaxBins + 1 bin offsets
  std::vector<int> pair_begin, pair_count;
  std::vector<char> pair_lds;
  chm::MatchArgs args;
  chm_tuning tun;
  hipGraphExec_t exec = nullptr;
  hipStream_t last_stream = nullptr;
  bool executed = false;
  // Host sources of the plan's device lists.  A plan whose upload was not
  // waited for keeps them until the upload stream has passed it.
  std::vector<chm::PairDev> h_pairs;
  std::vector<chm::WorkItem> h_items;
  // Bucket-major batched plans: the pairs in group order, the group ranges
  // and every round's bin tables in one int32 array, and a separate arena
  // block for the kept lists (reused by each round).
  bool bm = false;
  struct BmRound {
    int begin_off;   // int32 index of the round's n_bins + 1 bin offsets
    int list_off;    // int32 index of its group list
    int max_groups;  // groups of its fullest bin
  };
  std::vector<BmRound> bm_rounds;
  std::vector<int32_t> h_bm_ints;
  int bm_groups = 0;
  int32_t* dBmInts = nullptr;
  uint32_t* dState = nullptr;
  uint64_t state_off = 0, state_bytes = 0;
  hipStream_t upload_stream = nullptr;
  bool upload_pending = false;
};

namespace chm {
HashImage hash_image_of(const chm_store* S, const ImageSlot& sl);
chm_status hash_images(chm_store* S, const std::vector<const ImageSlot*>& slots, hipStream_t s);
int lds_max_feats(const chm_store* S);
// Builds a plan and queues its upload on `stream`.  With wait_upload the
// call returns once the upload is done (the plan may then run on any
// stream); without it the plan must run on `stream`, and plan_free() may be
// called only once that stream has passed the plan's last launch.
chm_status plan_build(chm_store* S, const int32_t* h_pairs, int32_t P, const int64_t* starts,
                      int32_t* d_out, uint32_t* d_topk, int32_t mode, void* stream, chm_plan** out,
                      bool wait_upload = true);
// Releases a plan without waiting: the caller has seen its work finish.
void plan_free(chm_plan* pl);
// chm_store_load in parts: argument checks; arena slots for all images or
// none (CHM_E_CAPACITY, nothing changed); descriptor copies queued on `s`
// and the images registered as resident (their codes and tables are built
// by hash_images on whichever stream has waited for the copies).
chm_status load_check(const chm_store* S, int32_t count, const int32_t* ids, const void* const* descs,
                      const int32_t* n_feats);
chm_status load_alloc(chm_store* S, int32_t count, const int32_t* ids, const int32_t* n_feats,
                      std::vector<ImageSlot>* slots);
chm_status load_commit(chm_store* S, int32_t count, const int32_t* ids, const void* const* descs,
                       std::vector<ImageSlot>& slots, bool on_device, hipStream_t s,
                       std::vector<const ImageSlot*>* ptrs);
// chm_store_evict that, with `held`, hands the slots (offset, bytes) to the
// caller instead of freeing them: queued kernels may still read them.
chm_status evict_hold(chm_store* S, int32_t count, const int32_t* ids,
                      std::vector<std::pair<uint64_t, uint64_t>>* held);
void release_held(chm_store* S, std::vector<std::pair<uint64_t, uint64_t>>* held);
// RANSAC (chm_ransac_filter's test) of the pairs idx[0..n) of a pair list on
// host threads: pair p's matches and output rows start at h_starts[p] of
// h_match / h_out, its words at h_words + p * iterations * 2.  The caller
// has checked the arguments; returns an error message or "".
std::string ransac_pairs(int32_t n, const int32_t* idx, const int32_t* h_pairs, const int32_t* const* h_kp,
                         const int32_t* h_n_feats, const int64_t* h_starts, const int32_t* h_match,
                         const uint32_t* h_words, int32_t iterations, int32_t thr, int32_t min_inliers,
                         int32_t n_threads, int32_t* h_out);
}  // namespace chm

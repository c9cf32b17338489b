// Internal declarations shared by the HIP kernels and the host side of libchm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chm {

constexpr int kDim = 128;
constexpr int kCodeWords = 4;   // 128-bit long code as 4 x u32
constexpr int kRowsPad = 192;   // projection rows padded: 128 code + up to 64 bucket bits
constexpr int kWStride = 136;   // bf16 elements per projection row in LDS (272 B: spreads banks)
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// Device-side view of one resident image.
struct ImageDev {
  const uint8_t* desc;      // n x 128
  const uint4* codes;       // n: long code, bit r in word r/32 at r%32
  const uint8_t* ids;       // L x n_pad: bucket id of each descriptor, table-major
  const uint32_t* norms;    // n: squared L2 norm
  const int32_t* offsets;   // L x (nb + 1)
  const uint16_t* members;  // L x n_pad, ascending inside each bucket
  int32_t n;
  int32_t n_pad;
};

struct PairDev {
  ImageDev q;
  ImageDev d;
  int64_t out_off;
};

struct WorkItem {
  int32_t pair;
  int32_t q0;
  int32_t q1;
  int32_t lds;  // 1 if the db image's codes fit the LDS stage of the kernel
};

struct MatchArgs {
  const PairDev* pairs;
  const WorkItem* items;
  int32_t n_items;
  int32_t item_base;      // non-persistent launches: first item of the launch
  uint32_t* queue;        // persistent launches: dequeue counter (zeroed per run)
  int32_t* out;
  uint32_t* topk;         // optional, K keys per output element
  int32_t L;
  int32_t nb;             // 2^m
  int32_t K;
  int32_t ratio_num;
  int32_t ratio_den;
  int32_t lds_max_feats;  // capacity of the LDS code stage (0 = none)
};

// Hashing of a batch of images, passed by value.
constexpr int kHashBatch = 64;

struct HashImage {
  const uint8_t* desc;
  uint4* codes;
  uint8_t* ids;             // L x n_pad, table-major
  uint32_t* norms;
  int32_t* offsets;
  uint16_t* members;
  int32_t n;
  int32_t n_pad;
};

struct HashBatch {
  HashImage img[kHashBatch];
  int32_t tile_prefix[kHashBatch + 1];  // 32-descriptor tiles before image i
  int32_t count;
  int32_t L;
  int32_t m;
};

struct ProjConsts {
  const uint16_t* W;        // kRowsPad x 128 bf16 bits (rows >= R are zero)
  const float* tau;         // kRowsPad: fixup_rel * ||W_r|| (rounded up), 0 for padding
  const double* cmu;        // kRowsPad: W_r . mu, exact
  const uint8_t* mu;        // 128
  unsigned long long* fixups;  // running count of fp64 recomputes
  uint32_t* fixlist;        // [0] overflow flag, [1..n_waves] per-wave counts, then
                            // n_waves regions of fix_cap/n_waves entries (im<<24 | r<<16 | d)
  uint32_t fix_cap;         // entries the list holds
  int32_t n_waves;          // projection wavefronts of the launch (set by launch_project)
  int32_t R;                // 128 + L*m
};

// Fix-up list capacity and the per-batch descriptor budget that keeps the
// expected list (about 1.6 entries per descriptor) well inside it.
constexpr uint32_t kFixListCap = 1u << 22;
constexpr int kMaxProjWaves = 8192;
constexpr int kHashBatchDescs = 1 << 20;

// Host-side launchers (defined in the .hip files).
hipError_t launch_project(const HashBatch& hb, const ProjConsts& pc, int fp32, int n_cu,
                          hipStream_t s);
hipError_t launch_buckets(const HashBatch& hb, hipStream_t s);
hipError_t launch_match(const MatchArgs& a, int K, int wg, bool lds, bool persistent, int grid,
                        hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s);
size_t match_lds_bytes(int lds_max_feats, int L, int nb);
hipError_t launch_bruteforce(const uint8_t* q, int nq, const uint8_t* d, int nd, int ra, int rb,
                             int32_t* out, void* work, int splits, hipStream_t s);
int bruteforce_splits(int nq, int nd);

}  // namespace chm

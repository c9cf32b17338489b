// Internal declarations shared by the HIP kernels and the host side of libchm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chm {

constexpr int kDim = 128;
constexpr int kCodeWords = 4;   // 128-bit long code as 4 x u32
constexpr int kRowsPad = 192;   // projection rows padded: 128 code + up to 64 bucket bits
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

#if defined(__HIPCC__)
// Inclusive prefix sum over the 64 lanes of a wavefront by DPP (no LDS
// round trips): running sums inside each 16-lane row, then the totals of
// rows 0 and 2 into rows 1 and 3, then the total of rows 0-1 into rows 2-3.
// Called with every lane active.
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}
#endif

// Device-side view of one resident image.
struct ImageDev {
  const uint8_t* desc;      // n x 128
  const uint4* codes;       // n: long code, bit r in word r/32 at r%32
  const uint8_t* ids;       // L x n_pad: bucket id of each descriptor, table-major
  const uint32_t* norms;    // n: squared L2 norm
  const int32_t* offsets;   // L x (nb + 1): padded bucket ranges, multiples of 8
  const int32_t* counts;    // L x nb: members of each bucket (without its pads)
  const uint32_t* members;  // L x m_stride code byte offsets (16 j), ascending inside each
                            // bucket, then pads
  const uint4* tcodes;      // L x m_stride codes in bucket order, or null (small images)
  int32_t n;
  int32_t n_pad;
  int32_t m_stride;         // members per table: n + 7 * min(nb, n), rounded up to 8
  int32_t reserved;
};

struct PairDev {
  ImageDev q;
  ImageDev d;
  int64_t out_off;
  int64_t st_off;           // bucket-major plans: first state row of the pair in its round
};

struct WorkItem {
  int32_t pair;
  int32_t q0;
  int32_t q1;
  int32_t lds;  // 1 if the db image's codes fit the LDS stage of the kernel
};

// Persistent launches split their items into bins, one per XCD (each XCD
// has its own L2): bin b holds items[bin_begin[b] .. bin_begin[b+1]).
constexpr int kMaxBins = 16;


struct MatchArgs {
  const PairDev* pairs;
  const WorkItem* items;
  int32_t n_items;
  int32_t item_base;      // non-persistent launches: first item of the launch
  uint32_t* queue;        // persistent launches: one dequeue counter per bin (zeroed per run)
  const int32_t* bin_begin;  // persistent launches: n_bins + 1 item offsets
  int32_t n_bins;
  int32_t* out;
  uint32_t* topk;         // optional, K keys per output element
  int32_t L;
  int32_t nb;             // 2^m
  int32_t K;
  int32_t ratio_num;
  int32_t ratio_den;
  int32_t accept_single;  // a single candidate passes the ratio test
  int32_t whole_bucket;   // re-rank every candidate as close as the K-th
  int32_t lds_max_feats;  // capacity of the LDS code stage (0 = none)
  int32_t lds_top;        // LDS-staging launches: byte address of the control words
};

// Bucket-major matching (match_bm.hip): one launch per table and round.
// Pairs are ordered so that each group (pairs[groups[g] .. groups[g+1]))
// shares one db image; bin x of the launch holds the groups
// bin_groups[bin_begin[x] .. bin_begin[x+1]), and work-group x + n_bins * k
// takes bucket k % nb of the bin's (k / nb)-th group.  state holds KT keys
// per (pair, query) at row pairs[p].st_off + query.
struct BmArgs {
  const PairDev* pairs;
  const int32_t* groups;
  const int32_t* bin_groups;
  const int32_t* bin_begin;
  uint32_t* state;
  int32_t* out;
  uint32_t* topk;
  int32_t n_bins;
  int32_t t;              // table of this launch
  int32_t L;
  int32_t nb;             // 2^m
  int32_t K;
  int32_t ratio_num;
  int32_t ratio_den;
  int32_t accept_single;
};

// Device RANSAC (ransac_device.hip), in the same two parts as the device
// SAO: ransac_upload writes the pair table (word_pair[p], or p when null, is
// the index of pair p's random words and best count) and returns once it
// is on the device; ransac_run verifies table entries first..first+count-1
// with at most n_max query rows each.  The work buffer's first int32
// counts pairs whose input broke the contract.
uint64_t ransac_work_bytes(int32_t n_pairs, int32_t max_rows);
hipError_t ransac_upload(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                         const int32_t* h_n_feats, const int64_t* h_starts, const int32_t* word_pair,
                         void* d_work, hipStream_t s);
hipError_t ransac_run(int32_t first, int32_t count, int32_t table_pairs, int32_t n_max, const int32_t* d_match,
                      const uint32_t* d_words, int32_t iterations, int32_t thr, int32_t min_inliers,
                      int32_t* d_out, int32_t* d_best_counts, void* d_work, hipStream_t s);

// Device SAO (sao_device.hip).  h_starts[p] is where pair p's query rows
// begin in d_match / d_out / d_ced (only starts are read); the caller has
// checked the arguments.  clear_errors zeroes the work buffer's error word.
constexpr int kSaoMaxNeighbors = 8;
uint64_t sao_work_bytes(int32_t n_pairs, int32_t max_rows);
hipError_t launch_sao(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                      const int32_t* h_n_feats, const int64_t* h_starts, const int32_t* d_match, int32_t nn,
                      int32_t num, int32_t den, int32_t* d_out, int32_t* d_ced, void* d_work, bool clear_errors,
                      hipStream_t s);
// The same in two parts: sao_upload writes the pair table (pairs 0..n-1 of
// the work buffer's table) and returns once it is on the device; sao_run
// filters table entries first..first+count-1 with at most n_max query rows
// each, the table holding table_pairs entries (the scratch follows it).
hipError_t sao_upload(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                      const int32_t* h_n_feats, const int64_t* h_starts, void* d_work, hipStream_t s);
hipError_t sao_run(int32_t first, int32_t count, int32_t table_pairs, int32_t n_max, const int32_t* d_match,
                   int32_t nn, int32_t num, int32_t den, int32_t* d_out, int32_t* d_ced, void* d_work,
                   hipStream_t s);

// LDS of the match kernel.  The LDS-staging kernel takes all of a CU's LDS:
// the db image's codes from address 0 (a code's LDS address is its member
// value 16 j), then its bucket offsets when they fit beside a full-size sort
// (else the walk reads them from L2), and at the top, from lds_top, two
// control words (16 B) and the sort histogram (256 u32).  An item's sort
// order (u16 per query) sits right below lds_top; an item of at most
// kSortMax queries is processed in order of walk length when its order fits
// above the stage, else in query order.  The HBM-only kernel's LDS is the
// order array and the top.
#ifndef CHM_SORT_MAX
#define CHM_SORT_MAX 4096
#endif
constexpr int kSortMax = CHM_SORT_MAX;
constexpr size_t kLdsTop = 16 + 256 * 4;
constexpr size_t kMatchLdsTail = 2 * kSortMax + kLdsTop;
constexpr size_t kLdsTotal = 160 * 1024;

// Largest db image whose codes the LDS stage can hold.
__host__ __device__ constexpr int lds_code_cap() { return (int)((kLdsTotal - kLdsTop) / 16); }
// Queries of an item that can be sorted above a stage of n codes whose
// offsets stay in L2 (lds_top bytes below the top words).
__host__ __device__ constexpr int lds_sort_room(int lds_top, int n) { return (lds_top - 16 * n) / 2; }

// Sections of one image slot in the arena (byte offsets from the slot
// start, each 256-byte aligned): descriptors n x 128, long codes n x 16,
// bucket ids L x n_pad, squared norms n x 4, offsets L x (2^m + 1) int32,
// real member counts L x 2^m int32, members L x m_stride u32, and for images too large for the LDS code stage
// the codes again in bucket order, L x m_stride x 16 (tcodes[t][pos] is the
// code of members[t][pos]).  Used by the host to size and address slots and
// by the hashing kernels to address a slot from its base alone.
struct ImageLayout {
  uint64_t desc, codes, ids, norms, offsets, counts, members, tcodes, total;
  int n_pad;
  int m_stride;
  bool has_tcodes;
};

__host__ __device__ inline uint64_t layout_round(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

__host__ __device__ inline ImageLayout image_layout(int L, int m, int n) {
  ImageLayout l;
  const uint64_t nb = 1ull << m;
  l.n_pad = (int)layout_round((uint64_t)n, 8);
  // each bucket padded to a multiple of 8 members: at most 7 pads per
  // non-empty bucket
  l.m_stride = (int)layout_round((uint64_t)n + 7 * ((uint64_t)n < nb ? (uint64_t)n : nb), 8);
  uint64_t o = 0;
  l.desc = o;    o += layout_round((uint64_t)n * kDim, 256);
  l.codes = o;   o += layout_round((uint64_t)n * 16, 256);
  l.ids = o;     o += layout_round((uint64_t)L * l.n_pad, 256);
  l.norms = o;   o += layout_round((uint64_t)n * 4, 256);
  l.offsets = o; o += layout_round((uint64_t)L * (nb + 1) * 4, 256);
  l.counts = o;  o += layout_round((uint64_t)L * nb * 4, 256);
  l.members = o; o += layout_round((uint64_t)L * l.m_stride * 4, 256);
  l.has_tcodes = n > lds_code_cap();
  l.tcodes = o;  o += l.has_tcodes ? layout_round((uint64_t)L * l.m_stride * 16, 256) : 0;
  l.total = o;
  return l;
}

// Hashing of a batch of images.  The batch is a kernel argument, so it only
// carries each image's slot (its offset from the arena base in 256-byte
// units) and size, 8 bytes an image; kernels expand an entry with
// hash_image().
constexpr int kHashBatch = 128;

struct HashSlot {
  uint32_t off256;          // slot offset / 256 from HashBatch::arena
  int32_t n;
};

struct HashImage {
  const uint8_t* desc;
  uint4* codes;
  uint8_t* ids;             // L x n_pad, table-major
  uint32_t* norms;
  int32_t* offsets;
  int32_t* counts;          // L x nb members per bucket, without pads
  uint32_t* members;        // 16 * db index (the byte offset of its code)
  uint4* tcodes;            // codes in bucket order, or null
  int32_t n;
  int32_t n_pad;
  int32_t m_stride;
};

struct HashBatch {
  uint8_t* arena;
  HashSlot img[kHashBatch];
  int32_t tile_prefix[kHashBatch + 1];  // 32-descriptor tiles before image i
  int32_t count;
  int32_t L;
  int32_t m;
};

__host__ __device__ inline HashImage hash_image_at(uint8_t* base, int n, int L, int m) {
  const ImageLayout l = image_layout(L, m, n);
  HashImage h;
  h.desc = base + l.desc;
  h.codes = reinterpret_cast<uint4*>(base + l.codes);
  h.ids = base + l.ids;
  h.norms = reinterpret_cast<uint32_t*>(base + l.norms);
  h.offsets = reinterpret_cast<int32_t*>(base + l.offsets);
  h.counts = reinterpret_cast<int32_t*>(base + l.counts);
  h.members = reinterpret_cast<uint32_t*>(base + l.members);
  h.tcodes = l.has_tcodes ? reinterpret_cast<uint4*>(base + l.tcodes) : nullptr;
  h.n = n;
  h.n_pad = l.n_pad;
  h.m_stride = l.m_stride;
  return h;
}

__host__ __device__ inline HashImage hash_image(const HashBatch& hb, int im) {
  return hash_image_at(hb.arena + 256ull * hb.img[im].off256, hb.img[im].n, hb.L, hb.m);
}

struct ProjConsts {
  const uint16_t* W;        // kRowsPad x 128 bf16 bits (rows >= R are zero)
  const float* tau;         // 3 x kRowsPad: fixup_rel ||W_r||, fixup_rel |c_r| (both rounded
                            // up), c_r rounded to fp32; 0 for padding rows
  const double* cmu;        // kRowsPad: W_r . mu, exact
  const uint8_t* mu;        // 128
  unsigned long long* fixups;  // running counts: [0] fp64 recomputes, [1] bits they changed
  uint32_t* fixlist;        // n_waves regions of fix_cap/n_waves entries (im<<24 | r<<16 | d),
                            // one per projection wavefront
  uint32_t fix_cap;         // entries the list holds
  int32_t n_waves;          // projection wavefronts of the launch (set by launch_project)
  int32_t R;                // 128 + L*m
};

static_assert(sizeof(HashBatch) + sizeof(ProjConsts) <= 2048, "hashing kernel arguments too large");

// Fix-up list capacity; a batch holds at most kHashBatchDescs descriptors,
// fewer when fixup_rel makes the expected list (about 2800 fixup_rel
// entries per descriptor) more than half the capacity.
constexpr uint32_t kFixListCap = 1u << 22;
constexpr int kMaxProjWaves = 8192;
constexpr int kHashBatchDescs = 1 << 22;

// Host-side launchers (defined in the .hip files).
hipError_t launch_project(const HashBatch& hb, const ProjConsts& pc, int fp32, int n_cu,
                          hipStream_t s);
// Bucket tables of the batch, then the bucket-ordered code copies of its
// images that have one (n_xcd: XCDs the work-groups are dealt to).
hipError_t launch_buckets(const HashBatch& hb, int n_xcd, hipStream_t s);
hipError_t launch_match(const MatchArgs& a, int K, int wg, bool lds, bool persistent, int grid,
                        hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s);
// Table a.t of a bucket-major round over `grid` work-groups (n_bins x the
// largest bin's groups x nb).
hipError_t launch_match_bm(const BmArgs& a, int K, int grid, hipStream_t s);

hipError_t launch_bruteforce(const uint8_t* q, int nq, const uint8_t* d, int nd, int ra, int rb,
                             int32_t* out, void* work, int splits, hipStream_t s);
int bruteforce_splits(int nq, int nd);
uint64_t bruteforce_work_bytes(int nq, int nd);
// The library's own brute-force workspace (chm_bruteforce_noalloc): a static
// device array of kBfScratchBytes per GPU; bruteforce_scratch() returns the
// current device's copy (resolved once per device, kept until the process
// ends).  Devices 0..kBfScratchDevices-1.
constexpr uint64_t kBfScratchBytes = 32ull << 20;
constexpr int kBfScratchDevices = 64;
hipError_t bruteforce_scratch(void** out);

}  // namespace chm

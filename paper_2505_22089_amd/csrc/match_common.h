// Device helpers shared by the two match kernels (match.hip: one lane per
// query walking its own buckets; match_bm.hip: bucket-major, the lanes of a
// wavefront sharing one db bucket).
#pragma once

#include "chm_internal.h"

namespace chm {

// Lanes that share one candidate descriptor in the re-rank (4 or 8).
#ifndef CHM_RERANK_LANES
#define CHM_RERANK_LANES 4
#endif
constexpr int kRerankLanes = CHM_RERANK_LANES;

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4u gcv4u;
typedef __attribute__((address_space(1))) const uint32_t gcu32;
typedef __attribute__((address_space(1))) const uint8_t gcu8;
typedef __attribute__((address_space(1))) const int32_t gci32;
typedef __attribute__((address_space(3))) const int32_t lds_ci32;

// popcount(x) + acc in one instruction
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

// 2 * m + (bit of this lane in `lanes`): appends one pass bit per instruction
__device__ __forceinline__ uint32_t shift_in(uint32_t m, uint64_t lanes) {
  uint32_t r;
  asm("v_addc_co_u32 %0, vcc, %1, %1, %2" : "=v"(r) : "v"(m), "s"(lanes) : "vcc");
  return r;
}

__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// 16-byte load through a global (not flat) pointer.
__device__ __forceinline__ uint4 ldg4(const void* p) {
  const v4u v = *(gcv4u*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Inserts key into the ascending list top unless it repeats a kept key (a
// key equal to the last one changes nothing, so only the first KT - 1 are
// tested): the smallest XOR of key with them is zero exactly for a repeat.
// The test stays in VALU registers; equality compares would build a lane
// mask through the scalar unit, one dependent round trip per kept key.
template <int KT>
__device__ __forceinline__ void insert_unique(uint32_t (&top)[KT], uint32_t key) {
  uint32_t m = key ^ top[0];
  int k = 1;
#pragma unroll
  for (; k + 1 < KT - 1; k += 2) m = min3u(m, key ^ top[k], key ^ top[k + 1]);
  if (k < KT - 1) m = min(m, key ^ top[k]);
  key = m == 0u ? kNoKey : key;
#pragma unroll
  for (int k = KT - 1; k >= 1; --k) top[k] = med3u(top[k - 1], key, top[k]);
  top[0] = min(top[0], key);
}

// Ascending sort of 8 keys: Batcher's odd-even merge network, 19
// compare-exchanges in 6 layers.
__device__ __forceinline__ void sort8(uint32_t (&v)[8]) {
  auto ce = [&](int i, int j) {
    const uint32_t lo = min(v[i], v[j]), hi = max(v[i], v[j]);
    v[i] = lo;
    v[j] = hi;
  };
  ce(0, 2); ce(1, 3); ce(4, 6); ce(5, 7);
  ce(0, 4); ce(1, 5); ce(2, 6); ce(3, 7);
  ce(0, 1); ce(2, 3); ce(4, 5); ce(6, 7);
  ce(2, 4); ce(3, 5);
  ce(1, 4); ce(3, 6);
  ce(1, 2); ce(3, 4); ce(5, 6);
}

// The 8 smallest of the ascending lists a and b, ascending, into a:
// min(a[k], b[7 - k]) is a bitonic sequence holding them, which three
// half-cleaner layers sort.
__device__ __forceinline__ void merge8_lowest(uint32_t (&a)[8], const uint32_t (&b)[8]) {
  uint32_t m[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) m[k] = min(a[k], b[7 - k]);
  auto ce = [&](int i, int j) {
    const uint32_t lo = min(m[i], m[j]), hi = max(m[i], m[j]);
    m[i] = lo;
    m[j] = hi;
  };
  ce(0, 4); ce(1, 5); ce(2, 6); ce(3, 7);
  ce(0, 2); ce(1, 3); ce(4, 6); ce(5, 7);
  ce(0, 1); ce(2, 3); ce(4, 5); ce(6, 7);
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = m[k];
}

typedef __attribute__((address_space(3))) const v4u lds_v4u;

// Long code of the db point whose code lies at byte offset off (16 j): in
// LDS the staged codes start at LDS address 0 (the kernel has no static LDS,
// which launch_one checks), so off is the LDS address itself.
template <bool LDSC>
__device__ __forceinline__ uint4 code_at(const char* gCodes, uint32_t off) {
  if (LDSC) {
    const v4u v = *reinterpret_cast<lds_v4u*>((size_t)off);
    return make_uint4(v.x, v.y, v.z, v.w);
  }
  return ldg4(gCodes + off);
}

// A pointer that is the same in every lane, kept in SGPRs.  readfirstlane
// returns int: each half goes through uint32_t before widening, so the low
// half is not sign-extended into the high one.
__device__ __forceinline__ const char* uniform_ptr(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
  return reinterpret_cast<const char*>(((uint64_t)hi << 32) | (uint64_t)lo);
}

// Per lane: cond (bit of this lane in the wave mask `lanes`) ? t : f.
__device__ __forceinline__ uint32_t sel_lanes(uint64_t lanes, uint32_t t, uint32_t f) {
  uint32_t r;
  asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(f), "v"(t), "s"(lanes));
  return r;
}

// Sum over the G lanes of each aligned group of G (G = 4 or 8): quad
// swaps, then for G = 8 the mirror inside the half-row, which pairs each
// quad with the other one.
template <int G>
__device__ __forceinline__ uint32_t sum_lanes(uint32_t v) {
  static_assert(G == 4 || G == 8, "groups of 4 or 8 lanes");
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  if (G == 8) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  return v;
}

__device__ __forceinline__ uint32_t lane_read(uint32_t v, int src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}


// Loads through a constant-address-space pointer: with a wavefront-uniform
// address they compile to scalar loads into SGPRs (the data is read-only for
// the whole kernel).
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}
__device__ __forceinline__ uint4 ld_uniform4(const void* p) {
  const v4u v = *(const __attribute__((address_space(4))) v4u*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}

}  // namespace chm

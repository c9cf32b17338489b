// Cascade-hashing matching of directed image pairs (Sec. 2.3.1 steps (1)-(4)).
//
// One lane owns one query descriptor x_i of the query image:
//  (1) for each table t it walks the db image's bucket beta_t(x_i); the
//      bucket's members (ascending db indices, u16) are read as aligned
//      16-byte blocks of eight, one block ahead of use;
//  (2) for each candidate j it forms h = popcount(c(x_i) xor c(y_j)) over the
//      128-bit long codes and the key (h << 24) | j, whose order is the
//      paper's ranking by Hamming distance with ties broken by db index;
//  (3) it keeps the KT smallest distinct keys in registers: a sorted list
//      updated with median-of-three steps; a key equal to a kept one is a
//      candidate an earlier table already returned and is dropped, which
//      makes the candidate list a set (a key equal to the last kept one
//      leaves the list unchanged, so it needs no test).  Keys of a block of
//      eight candidates are computed first; only those below the current
//      KT-th key are inserted, each lane looping over its own passes;
//  (4) for the first K kept candidates it computes the exact squared distance
//      ||x||^2 + ||y||^2 - 2 x.y with packed-u8 dot products and int32
//      accumulation, and applies the ratio test on squared distances
//      (den^2 * d1 < num^2 * d2).
//
// Work items are (pair, query range).  Batched plans run one persistent grid
// that dequeues items with an atomic counter; inside a work-group, wavefronts
// take 64-query chunks of the item dynamically.  Plain plans launch one grid
// per pair.  With LDSC the db image's codes and bucket offsets are staged in
// LDS once per item (skipped when consecutive items share the db image).
#include "chm_internal.h"

namespace chm {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4u gcv4u;
typedef __attribute__((address_space(1))) const uint32_t gcu32;
typedef __attribute__((address_space(1))) const uint8_t gcu8;
typedef __attribute__((address_space(1))) const int32_t gci32;

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

template <int KT>
__device__ __forceinline__ void insert_unique(uint32_t (&top)[KT], uint32_t key) {
  bool dup = false;
#pragma unroll
  for (int k = 0; k < KT - 1; ++k) dup |= (key == top[k]);
  key = dup ? kNoKey : key;
#pragma unroll
  for (int k = KT - 1; k >= 1; --k) top[k] = med3u(top[k - 1], key, top[k]);
  top[0] = min(top[0], key);
}

template <bool LDSC>
__device__ __forceinline__ uint4 code_of(const uint4* sCodes, const uint4* gCodes, uint32_t j) {
  if (LDSC) return sCodes[j];
  return ldg4(gCodes + j);
}

template <int KT, bool LDSC>
__device__ __forceinline__ void match_query(const MatchArgs& a, const PairDev& P, int q,
                                            const uint4* sCodes, const int32_t* offs) {
  const uint4 qc = ldg4(P.q.codes + q);
  uint32_t qb0 = 0, qb1 = 0;  // bucket ids of the query, one byte per table
  for (int t = 0; t < a.L; ++t) {
    const uint32_t b = *(gcu8*)(P.q.ids + (size_t)t * P.q.n_pad + q);
    if (t < 4) qb0 |= b << (8 * t);
    else qb1 |= b << (8 * (t - 4));
  }
  uint32_t top[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) top[k] = kNoKey;
  uint32_t thr = kNoKey;  // top[KT - 1] as of the last block

  const uint16_t* members = P.d.members;
  const int n_pad = P.d.n_pad;
  const int stride = a.nb + 1;
  // Walk the L buckets as one sequence of aligned 8-member blocks.
  int t = -1, s = 0, e = 0, p = 0;
  auto next_table = [&]() {
    for (++t; t < a.L; ++t) {
      const uint32_t b = ((t < 4 ? qb0 >> (8 * t) : qb1 >> (8 * (t - 4)))) & 0xFFu;
      s = offs[t * stride + b];
      e = offs[t * stride + b + 1];
      if (s < e) {
        p = s & ~7;
        return;
      }
    }
  };
  next_table();
  uint4 blk = make_uint4(0, 0, 0, 0);
  if (t < a.L) blk = ldg4(members + (size_t)t * n_pad + p);
  while (t < a.L) {
    const uint4 cur = blk;
    const int base = p - s;       // slot k holds position p + k; valid iff 0 <= base + k < len
    const int len = e - s;
    p += 8;
    if (p >= e) next_table();
    if (t < a.L) blk = ldg4(members + (size_t)t * n_pad + p);
    const uint32_t w[4] = {cur.x, cur.y, cur.z, cur.w};
    // Keys of the block; a slot passes when it could enter the kept list
    // (key below the current KT-th key).  Only passing slots are inserted,
    // lane by lane, so the insertion cost follows each lane's own passes.
    uint32_t key[8];
    uint32_t pmask = 0;  // slot k at bit 7 - k
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t j = (k & 1) ? (w[k >> 1] >> 16) : (w[k >> 1] & 0xFFFFu);
      const uint4 c = code_of<LDSC>(sCodes, P.d.codes, j);
      const uint32_t h =
          bcnt_acc(qc.w ^ c.w, bcnt_acc(qc.z ^ c.z, bcnt_acc(qc.y ^ c.y, bcnt_acc(qc.x ^ c.x, 0u))));
      key[k] = (h << 24) | j;
      pmask = shift_in(pmask, __ballot(key[k] < thr));
    }
    // slots outside [s, e): k < -base or k >= len - base
    {
      const int lo = max(0, -base), hi = min(8, len - base);
      const uint32_t valid = (0xFFu >> lo) & ~(0xFFu >> hi);
      pmask &= valid;
    }
    while (pmask) {
      const uint32_t i = 7u - (31u - __builtin_clz(pmask));
      pmask &= ~(0x80u >> i);
      const uint32_t s01 = (i & 1) ? key[1] : key[0], s23 = (i & 1) ? key[3] : key[2];
      const uint32_t s45 = (i & 1) ? key[5] : key[4], s67 = (i & 1) ? key[7] : key[6];
      const uint32_t s03 = (i & 2) ? s23 : s01, s47 = (i & 2) ? s67 : s45;
      insert_unique<KT>(top, (i & 4) ? s47 : s03);
    }
    thr = top[KT - 1];
  }

  const int64_t o = P.out_off + q;
  if (a.topk) {
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (k < a.K) a.topk[o * a.K + k] = top[k];
  }

  // Euclidean re-rank of the first K candidates and ratio test.
  const uint4* xq = reinterpret_cast<const uint4*>(P.q.desc + (size_t)q * kDim);
  uint4 x[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) x[v] = ldg4(xq + v);
  const uint32_t nq = *(gcu32*)(P.q.norms + q);
  uint32_t d1 = 0xFFFFFFFFu, d2 = 0xFFFFFFFFu;
  int j1 = -1, cnt = 0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    if (k < a.K && top[k] != kNoKey) {
      const uint32_t j = top[k] & 0xFFFFFFu;
      const uint4* yp = reinterpret_cast<const uint4*>(P.d.desc + (size_t)j * kDim);
      uint32_t dot = 0;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const uint4 y = ldg4(yp + v);
        dot = __builtin_amdgcn_udot4(x[v].x, y.x, dot, false);
        dot = __builtin_amdgcn_udot4(x[v].y, y.y, dot, false);
        dot = __builtin_amdgcn_udot4(x[v].z, y.z, dot, false);
        dot = __builtin_amdgcn_udot4(x[v].w, y.w, dot, false);
      }
      const uint32_t e2 = nq + *(gcu32*)(P.d.norms + j) - 2u * dot;
      if (e2 < d1) {
        d2 = d1;
        d1 = e2;
        j1 = (int)j;
      } else if (e2 < d2) {
        d2 = e2;
      }
      ++cnt;
    }
  }
  const bool pass = cnt >= 2 && (uint64_t)a.ratio_den * (uint64_t)a.ratio_den * d1 <
                                    (uint64_t)a.ratio_num * (uint64_t)a.ratio_num * d2;
  a.out[o] = pass ? j1 : -1;
}

template <int KT, bool LDSC, int WG>
__device__ __forceinline__ void run_item(const MatchArgs& a, const PairDev& P, const WorkItem& w,
                                         const uint4* sCodes, const int32_t* offs, int* s_chunk) {
  // Wavefronts take 64-query chunks of the item in turn.
  const int lane = __lane_id();
  for (;;) {
    int c = 0;
    if (lane == 0) c = atomicAdd(s_chunk, 64);
    c = __builtin_amdgcn_readfirstlane(__shfl(c, 0));  // uniform across the wave
    const int q = w.q0 + c + lane;
    if (w.q0 + c >= w.q1) break;
    if (q < w.q1) match_query<KT, LDSC>(a, P, q, sCodes, offs);
  }
}

template <int KT, int WG, bool LDSC, bool PERSIST>
__global__ __launch_bounds__(WG) void k_match(MatchArgs a) {
  extern __shared__ uint4 smem[];
  __shared__ int s_item;
  __shared__ int s_chunk;
  const int ncodes = a.lds_max_feats;
  uint4* sCodes = smem;
  int32_t* sOffs = reinterpret_cast<int32_t*>(smem + (LDSC ? ncodes : 0));
  const uint4* staged = nullptr;
  int it = PERSIST ? 0 : a.item_base + (int)blockIdx.x;

  for (;;) {
    if (PERSIST) {
      if (threadIdx.x == 0) s_item = (int)atomicAdd(a.queue, 1u);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(s_item);  // uniform: item fields in SGPRs
      if (it >= a.n_items) break;
    }
    if (threadIdx.x == 0) s_chunk = 0;
    const WorkItem w = a.items[it];
    const PairDev& P = a.pairs[w.pair];
    const bool use_lds = LDSC && P.d.n <= ncodes;
    if (use_lds && staged != P.d.codes) {
      for (int j = threadIdx.x; j < P.d.n; j += WG) sCodes[j] = ldg4(P.d.codes + j);
      for (int i = threadIdx.x; i < a.L * (a.nb + 1); i += WG) sOffs[i] = *(gci32*)(P.d.offsets + i);
      staged = P.d.codes;
    }
    __syncthreads();
    if (use_lds)
      run_item<KT, true, WG>(a, P, w, sCodes, sOffs, &s_chunk);
    else
      run_item<KT, false, WG>(a, P, w, nullptr, P.d.offsets, &s_chunk);
    __syncthreads();
    if (!PERSIST) break;
  }
}

size_t match_lds_bytes(int lds_max_feats, int L, int nb) {
  return (size_t)lds_max_feats * sizeof(uint4) + (size_t)L * (nb + 1) * sizeof(int32_t);
}

template <int KT, int WG, bool LDSC, bool PERSIST>
static hipError_t launch_one(const MatchArgs& a, int grid, hipStream_t s) {
  const size_t lds = LDSC ? match_lds_bytes(a.lds_max_feats, a.L, a.nb) : 0;
  auto fn = k_match<KT, WG, LDSC, PERSIST>;
  if (LDSC) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(grid), dim3(WG), lds, s, a);
  return hipGetLastError();
}

template <int KT>
static hipError_t launch_k(const MatchArgs& a, int wg, bool lds, bool persistent, int grid,
                           hipStream_t s) {
  if (wg == 1024) {
    if (lds) return persistent ? launch_one<KT, 1024, true, true>(a, grid, s)
                               : launch_one<KT, 1024, true, false>(a, grid, s);
    return persistent ? launch_one<KT, 1024, false, true>(a, grid, s)
                      : launch_one<KT, 1024, false, false>(a, grid, s);
  }
  if (lds) return persistent ? launch_one<KT, 256, true, true>(a, grid, s)
                             : launch_one<KT, 256, true, false>(a, grid, s);
  return persistent ? launch_one<KT, 256, false, true>(a, grid, s)
                    : launch_one<KT, 256, false, false>(a, grid, s);
}

hipError_t launch_match(const MatchArgs& a, int K, int wg, bool lds, bool persistent, int grid,
                        hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (K <= 2) return launch_k<2>(a, wg, lds, persistent, grid, s);
  if (K <= 4) return launch_k<4>(a, wg, lds, persistent, grid, s);
  if (K <= 8) return launch_k<8>(a, wg, lds, persistent, grid, s);
  if (K <= 16) return launch_k<16>(a, wg, lds, persistent, grid, s);
  return launch_k<32>(a, wg, lds, persistent, grid, s);
}

}  // namespace chm

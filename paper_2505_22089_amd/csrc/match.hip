// Cascade-hashing matching of directed image pairs (Sec. 2.3.1 steps (1)-(4)).
//
// One lane owns one query descriptor x_i of the query image:
//  (1) for each table t it walks the db image's bucket beta_t(x_i)
//      (members are ascending db indices);
//  (2) for each candidate j it forms h = popcount(c(x_i) xor c(y_j)) over the
//      128-bit long codes and the key (h << 24) | j, whose order is the
//      paper's ranking by Hamming distance with ties broken by db index;
//  (3) it keeps the KT smallest distinct keys in registers (a sorted list
//      updated with a branch-free median-of-three insertion; a key equal to a
//      kept one is a candidate already returned by an earlier table and is
//      skipped, which makes the candidate list a set);
//  (4) for the first K kept candidates it computes the exact squared distance
//      ||x||^2 + ||y||^2 - 2 x.y with 4-byte unsigned dot products and int32
//      accumulation, and applies the ratio test on squared distances
//      (den^2 * d1 < num^2 * d2).
//
// Work items are (pair, query range).  Batched plans run one persistent grid
// that dequeues items with an atomic counter; plain plans launch one grid per
// pair.  With LDSC the db image's codes and bucket offsets are staged in LDS
// once per item (or per run of items on the same db image).
#include "chm_internal.h"

namespace chm {

template <int KT>
__device__ __forceinline__ void insert_unique(uint32_t (&top)[KT], uint32_t key) {
  bool dup = false;
#pragma unroll
  for (int k = 0; k < KT; ++k) dup |= (key == top[k]);
  key = dup ? kNoKey : key;
#pragma unroll
  for (int k = KT - 1; k >= 1; --k) top[k] = min(max(top[k - 1], key), top[k]);
  top[0] = min(top[0], key);
}

__device__ __forceinline__ uint32_t bucket_of(uint2 ids, int t) {
  return ((t < 4 ? ids.x >> (8 * t) : ids.y >> (8 * (t - 4)))) & 0xFFu;
}

template <int KT, bool LDSC>
__device__ __forceinline__ void match_query(const MatchArgs& a, const PairDev& P, int q,
                                            const uint4* sCodes, const int32_t* offs) {
  const uint4 qc = P.q.codes[q];
  const uint2 qid = P.q.ids[q];
  uint32_t top[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) top[k] = kNoKey;

  for (int t = 0; t < a.L; ++t) {
    const uint32_t b = bucket_of(qid, t);
    const int s = offs[t * (a.nb + 1) + b];
    const int e = offs[t * (a.nb + 1) + b + 1];
    const uint16_t* mem = P.d.members + (size_t)t * P.d.n_pad;
    for (int pos = s; pos < e; ++pos) {
      const uint32_t j = mem[pos];
      const uint4 c = LDSC ? sCodes[j] : P.d.codes[j];
      const uint32_t h = __popc(qc.x ^ c.x) + __popc(qc.y ^ c.y) + __popc(qc.z ^ c.z) +
                         __popc(qc.w ^ c.w);
      insert_unique<KT>(top, (h << 24) | j);
    }
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
  for (int v = 0; v < 8; ++v) x[v] = xq[v];
  const uint32_t nq = P.q.norms[q];
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
        const uint4 y = yp[v];
        dot = __builtin_amdgcn_udot4(x[v].x, y.x, dot, false);
        dot = __builtin_amdgcn_udot4(x[v].y, y.y, dot, false);
        dot = __builtin_amdgcn_udot4(x[v].z, y.z, dot, false);
        dot = __builtin_amdgcn_udot4(x[v].w, y.w, dot, false);
      }
      const uint32_t e = nq + P.d.norms[j] - 2u * dot;
      if (e < d1) {
        d2 = d1;
        d1 = e;
        j1 = (int)j;
      } else if (e < d2) {
        d2 = e;
      }
      ++cnt;
    }
  }
  const bool pass = cnt >= 2 && (uint64_t)a.ratio_den * (uint64_t)a.ratio_den * d1 <
                                    (uint64_t)a.ratio_num * (uint64_t)a.ratio_num * d2;
  a.out[o] = pass ? j1 : -1;
}

template <int KT, int WG, bool LDSC, bool PERSIST>
__global__ __launch_bounds__(WG) void k_match(MatchArgs a) {
  extern __shared__ uint4 smem[];
  __shared__ int s_item;
  const int ncodes = a.lds_max_feats;
  uint4* sCodes = smem;
  int32_t* sOffs = reinterpret_cast<int32_t*>(smem + (LDSC ? ncodes : 0));
  const uint4* staged = nullptr;
  int it = PERSIST ? 0 : a.item_base + (int)blockIdx.x;

  for (;;) {
    if (PERSIST) {
      if (threadIdx.x == 0) s_item = (int)atomicAdd(a.queue, 1u);
      __syncthreads();
      it = s_item;
      __syncthreads();
      if (it >= a.n_items) break;
    }
    const WorkItem w = a.items[it];
    const PairDev& P = a.pairs[w.pair];
    const int32_t* offs = P.d.offsets;
    if (LDSC && P.d.n > ncodes) {
      // Does not fit the stage: read the codes from global memory.
      for (int q = w.q0 + (int)threadIdx.x; q < w.q1; q += WG)
        match_query<KT, false>(a, P, q, nullptr, P.d.offsets);
      if (!PERSIST) break;
      continue;
    }
    if (LDSC) {
      if (staged != P.d.codes) {
        __syncthreads();
        for (int j = threadIdx.x; j < P.d.n; j += WG) sCodes[j] = P.d.codes[j];
        for (int i = threadIdx.x; i < a.L * (a.nb + 1); i += WG) sOffs[i] = P.d.offsets[i];
        staged = P.d.codes;
        __syncthreads();
      }
      offs = sOffs;
    }
    for (int q = w.q0 + (int)threadIdx.x; q < w.q1; q += WG)
      match_query<KT, LDSC>(a, P, q, sCodes, offs);
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

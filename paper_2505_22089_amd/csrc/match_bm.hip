// Bucket-major cascade-hashing matching (Sec. 2.3.1 steps (1)-(4)).
//
// Step (1) makes every query in bucket b of table t a candidate of the same
// db points: the members of the db image's bucket b.  This kernel runs one
// table per launch and gives each wavefront one db bucket: its 64 lanes hold
// queries that fall into that bucket (from every pair of a group of pairs
// that share the db image), and they walk the bucket's members together.
// The members and their long codes are the same for every lane, so they are
// read with scalar loads into SGPRs: no per-lane gathers, no LDS.
//
// For every (pair, query) the kept list of step (3) (the KT smallest distinct
// keys (h << 24) | 16 j so far) lives in registers during a launch and in a
// state array between the L launches of a round: table 0 starts it empty,
// tables 1 .. L-2 read and write it back, and the last table re-ranks the
// first K exactly and applies the ratio test (step (4)), with the lanes of
// the wavefront in groups of kRerankLanes sharing each candidate descriptor.
// The keys of a block of 8 members are computed for all lanes (4 xor + 4
// popcount per key); those below a lane's current KT-th key are inserted one
// per lane per round, a key equal to a kept one dropped (it is a candidate an
// earlier table returned, or a pad of the bucket), exactly as the
// query-major kernel does, so both give the same kept list: the KT smallest
// distinct keys over the union of the L buckets.
//
// Work: launch t has one work-group (one wavefront) per (group, bucket);
// groups are dealt to bins, one per XCD, and work-group x + n_bins * k takes
// the k-th (group, bucket) of bin x, so a db image's buckets stay in one
// XCD's L2.
#include "match_common.h"

namespace chm {

typedef __attribute__((address_space(1))) v4u gv4u;

// Kept list of a (pair, query) between launches: KT keys at row * KT.
template <int KT>
__device__ __forceinline__ void state_load(const uint32_t* st, uint64_t row, uint32_t (&top)[KT]) {
  const uint32_t* p = st + row * KT;
  if (KT == 2) {
    typedef uint32_t v2u __attribute__((ext_vector_type(2)));
    const v2u v = *(const __attribute__((address_space(1))) v2u*)p;
    top[0] = v.x;
    top[1 % KT] = v.y;
  } else {
#pragma unroll
    for (int k = 0; k < KT; k += 4) {
      const v4u v = *(gcv4u*)(p + k);
      top[k] = v.x;
      top[(k + 1) % KT] = v.y;
      top[(k + 2) % KT] = v.z;
      top[(k + 3) % KT] = v.w;
    }
  }
}

template <int KT>
__device__ __forceinline__ void state_store(uint32_t* st, uint64_t row, const uint32_t (&top)[KT]) {
  uint32_t* p = st + row * KT;
  if (KT == 2) {
    typedef uint32_t v2u __attribute__((ext_vector_type(2)));
    v2u v;
    v.x = top[0];
    v.y = top[1 % KT];
    *(__attribute__((address_space(1))) v2u*)p = v;
  } else {
#pragma unroll
    for (int k = 0; k < KT; k += 4) {
      v4u v;
      v.x = top[k];
      v.y = top[(k + 1) % KT];
      v.z = top[(k + 2) % KT];
      v.w = top[(k + 3) % KT];
      *(gv4u*)(p + k) = v;
    }
  }
}

__device__ __forceinline__ uint32_t lane_read_u(uint32_t v, int src) { return lane_read(v, src); }

// One wavefront per (group, bucket b) of table a.t.  FIRST: table 0 (the
// kept lists start empty); LAST: table L-1 (re-rank and output).
template <int KT, bool FIRST, bool LAST>
__global__ __launch_bounds__(64) void k_match_bm(BmArgs a) {
  const int lane = __lane_id();
  const int x = (int)(blockIdx.x % (unsigned)a.n_bins);
  const int k = (int)(blockIdx.x / (unsigned)a.n_bins);
  const int gslot = k / a.nb;
  const int b = k - gslot * a.nb;
  const int g0 = ld_uniform(a.bin_begin + x), g1 = ld_uniform(a.bin_begin + x + 1);
  if (gslot >= g1 - g0) return;
  const int g = ld_uniform(a.bin_groups + g0 + gslot);
  const int p0 = ld_uniform(a.groups + g), p1 = ld_uniform(a.groups + g + 1);
  const int t = a.t;
  const int stride = a.nb + 1;

  // the db image (the same for every pair of the group) and its bucket b
  const PairDev* P0 = a.pairs + p0;
  const int32_t* doffs = ld_uniform(&P0->d.offsets);
  const int ds = ld_uniform(doffs + t * stride + b), de = ld_uniform(doffs + t * stride + b + 1);
  if (!FIRST && !LAST && ds == de) return;  // no candidate: the kept lists stay as they are
  const uint32_t* dmem = ld_uniform(&P0->d.members) + (size_t)t * (uint32_t)ld_uniform(&P0->d.m_stride) + ds;
  const uint4* dtc = ld_uniform(&P0->d.tcodes);
  if (dtc) dtc += (size_t)t * (uint32_t)ld_uniform(&P0->d.m_stride) + ds;
  const char* dcodes = reinterpret_cast<const char*>(ld_uniform(&P0->d.codes));
  const int nblk = (de - ds) >> 3;

  // queries of the group in bucket b of table t: pair p contributes the
  // real members of its query image's bucket b
  int total = 0;
  for (int p = p0; p < p1; ++p) total += ld_uniform(ld_uniform(&a.pairs[p].q.counts) + t * a.nb + b);

  for (int c0 = 0; c0 < total; c0 += 64) {
    const int gi = c0 + lane;
    const bool valid = gi < total;
    // the lane's pair and its position in that pair's bucket
    int pp = p0, il = 0, pre = 0;
    for (int p = p0; p < p1; ++p) {
      const int cnt = ld_uniform(ld_uniform(&a.pairs[p].q.counts) + t * a.nb + b);
      if (gi >= pre && gi < pre + cnt) {
        pp = p;
        il = gi - pre;
      }
      pre += cnt;
    }
    const PairDev& P = a.pairs[pp];
    const int qs = P.q.offsets[t * stride + b];
    const uint32_t qi = valid ? (*(gcu32*)(P.q.members + (size_t)t * (uint32_t)P.q.m_stride + qs + il) >> 4) : 0u;
    const uint4 qc = valid ? ldg4(P.q.codes + qi) : make_uint4(0u, 0u, 0u, 0u);
    const uint64_t row = (uint64_t)P.st_off + qi;

    uint32_t top[KT];
    if (FIRST || !valid) {
#pragma unroll
      for (int kk = 0; kk < KT; ++kk) top[kk] = kNoKey;
    } else {
      state_load<KT>(a.state, row, top);
    }
    uint32_t thr = top[KT - 1];

    // Insertion of a block's passing keys (as in the query-major kernel):
    // each round every lane takes its lowest remaining passing slot.
    uint32_t pkey[8];
    uint64_t ppass[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      pkey[kk] = kNoKey;
      ppass[kk] = 0;
    }
    auto drain = [&]() {
      uint64_t any = ppass[0] | ppass[1] | ppass[2] | ppass[3] | ppass[4] | ppass[5] | ppass[6] | ppass[7];
      while (any) {
        uint32_t v = kNoKey;
#pragma unroll
        for (int kk = 7; kk >= 0; --kk) v = sel_lanes(ppass[kk], pkey[kk], v);
        uint64_t seen = 0;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const uint64_t rest = ppass[kk] & seen;
          seen |= ppass[kk];
          ppass[kk] = rest;
        }
        any = ppass[0] | ppass[1] | ppass[2] | ppass[3] | ppass[4] | ppass[5] | ppass[6] | ppass[7];
        insert_unique<KT>(top, v);
      }
      thr = top[KT - 1];
    };
    // The bucket's members as aligned blocks of 8 (pads repeat the first
    // member); member value 16 j is the byte offset of db point j's code.
    const uint32_t lim_on = valid ? 1u : 0u;
    if constexpr (FIRST && KT == 8) {
      // Table 0: every candidate is a member of this one bucket, so no key
      // can repeat a kept one except the pads (copies of member 0, the same
      // slots in every lane); each block's keys, pads masked, are sorted and
      // merged with the list whole, with no insertion rounds.
      const uint32_t m0 = nblk > 0 ? ld_uniform(dmem) : 0u;
      for (int blk = 0; blk < nblk; ++blk) {
        uint32_t mv[8];
        uint4 cv[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) mv[kk] = ld_uniform(dmem + 8 * blk + kk);
        if (dtc) {
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) cv[kk] = ld_uniform4(dtc + 8 * blk + kk);
        } else {
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) cv[kk] = ld_uniform4(dcodes + mv[kk]);
        }
        uint32_t v[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const uint32_t h = bcnt_acc(qc.w ^ cv[kk].w,
                                      bcnt_acc(qc.z ^ cv[kk].z, bcnt_acc(qc.y ^ cv[kk].y, bcnt_acc(qc.x ^ cv[kk].x, 0u))));
          const bool pad = mv[kk] == m0 && (blk > 0 || kk > 0);  // uniform
          v[kk] = pad ? kNoKey : (h << 24) | mv[kk];
        }
        sort8(v);
        merge8_lowest(top, v);
      }
    } else {
    for (int blk = 0; blk < nblk; ++blk) {
      uint32_t mv[8];
      uint4 cv[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) mv[kk] = ld_uniform(dmem + 8 * blk + kk);
      if (dtc) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) cv[kk] = ld_uniform4(dtc + 8 * blk + kk);
      } else {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) cv[kk] = ld_uniform4(dcodes + mv[kk]);
      }
      drain();  // the previous block's insertions while this block's loads are in flight
      const uint32_t lim = lim_on ? thr : 0u;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const uint32_t h = bcnt_acc(qc.w ^ cv[kk].w,
                                    bcnt_acc(qc.z ^ cv[kk].z, bcnt_acc(qc.y ^ cv[kk].y, bcnt_acc(qc.x ^ cv[kk].x, 0u))));
        pkey[kk] = (h << 24) | mv[kk];
        ppass[kk] = __ballot(pkey[kk] < lim);
      }
    }
    drain();
    }

    if (!LAST) {
      if (valid) state_store<KT>(a.state, row, top);
      continue;
    }

    const int64_t o = P.out_off + qi;
    if (a.topk && valid) {  // keys as (h << 24) | j
#pragma unroll
      for (int kk = 0; kk < KT; ++kk)
        if (kk < a.K)
          a.topk[o * a.K + kk] =
              top[kk] == kNoKey ? kNoKey : (top[kk] & 0xFF000000u) | ((top[kk] & 0xFFFFFFu) >> 4);
    }
    // Exact re-rank of the first K kept candidates and the ratio test, with
    // the wavefront's lanes in groups of G: in round gr, group r serves the
    // (pair, query) of lane NG gr + r, each of its lanes reading one slice
    // of the query and of each candidate descriptor.
    constexpr int G = kRerankLanes;
    constexpr int NG = 64 / G;
    constexpr int SL = kDim / G / 16;
    const uint32_t xoff = (uint32_t)(lane % G) * (kDim / G);
    const uint64_t qrow = (uint64_t)(P.q.desc + (size_t)qi * kDim);
    const uint32_t qnorm = valid ? *(gcu32*)(P.q.norms + qi) : 0u;
    const char* ddesc = reinterpret_cast<const char*>(ld_uniform(&P0->d.desc));
    const char* dnorm = reinterpret_cast<const char*>(ld_uniform(&P0->d.norms));
    const int dn = ld_uniform(&P0->d.n);
    int result = -1;
    if (dn > 0) {  // else no query has a candidate (and row 0 does not exist)
#pragma unroll 1
      for (int gr = 0; gr < G; ++gr) {
        const int src = NG * gr + lane / G;
        const bool vs = lane_read_u(valid ? 1u : 0u, src) != 0u;
        const uint64_t rs = ((uint64_t)lane_read_u((uint32_t)(qrow >> 32), src) << 32) |
                            (uint64_t)lane_read_u((uint32_t)qrow, src);
        const uint32_t nqs = lane_read_u(qnorm, src);
        const char* xr = vs ? reinterpret_cast<const char*>(rs) : ddesc;  // a lane without a query reads db row 0
        uint4 xs[SL];
#pragma unroll
        for (int v = 0; v < SL; ++v) xs[v] = ldg4(xr + xoff + 16u * v);
        uint32_t d1 = 0xFFFFFFFFu, d2 = 0xFFFFFFFFu, j1 = 0xFFFFFFFFu, cnt = 0;
        constexpr int KB = KT < 8 / SL ? KT : 8 / SL;
#pragma unroll
        for (int k0 = 0; k0 < KT; k0 += KB) {
          uint4 y[KB][SL];
          uint32_t ny[KB], jj[KB];
          bool ok[KB];
#pragma unroll
          for (int kk = 0; kk < KB; ++kk) {
            const uint32_t key = lane_read_u(top[k0 + kk], src);
            ok[kk] = vs && k0 + kk < a.K && key != kNoKey;
            jj[kk] = (key & 0xFFFFFFu) >> 4;
            const uint32_t j = ok[kk] ? jj[kk] : 0u;
#pragma unroll
            for (int v = 0; v < SL; ++v) y[kk][v] = ldg4(ddesc + (j * (uint32_t)kDim + xoff + 16u * v));
            ny[kk] = *(gcu32*)(dnorm + 4u * j);
          }
#pragma unroll
          for (int kk = 0; kk < KB; ++kk) {
            uint32_t dot = 0;
#pragma unroll
            for (int v = 0; v < SL; ++v) {
              dot = __builtin_amdgcn_udot4(xs[v].x, y[kk][v].x, dot, false);
              dot = __builtin_amdgcn_udot4(xs[v].y, y[kk][v].y, dot, false);
              dot = __builtin_amdgcn_udot4(xs[v].z, y[kk][v].z, dot, false);
              dot = __builtin_amdgcn_udot4(xs[v].w, y[kk][v].w, dot, false);
            }
            dot = sum_lanes<G>(dot);
            const uint32_t e2 = ok[kk] ? nqs + ny[kk] - 2u * dot : 0xFFFFFFFFu;
            j1 = e2 < d1 ? jj[kk] : j1;
            d2 = med3u(d1, e2, d2);
            d1 = min(d1, e2);
            cnt += ok[kk] ? 1u : 0u;
          }
        }
        const bool pass = cnt >= 2 ? (uint64_t)a.ratio_den * (uint64_t)a.ratio_den * d1 <
                                         (uint64_t)a.ratio_num * (uint64_t)a.ratio_num * d2
                                   : cnt == 1 && a.accept_single != 0;
        const uint32_t got = lane_read_u(pass ? j1 : 0xFFFFFFFFu, (lane % NG) * G);
        if (lane / NG == gr) result = (int)got;
      }
    }
    if (valid) a.out[o] = result;
  }
}

template <int KT>
static hipError_t launch_bm_k(const BmArgs& a, int grid, hipStream_t s) {
  const bool first = a.t == 0, last = a.t == a.L - 1;
  if (first && last)
    hipLaunchKernelGGL((k_match_bm<KT, true, true>), dim3(grid), dim3(64), 0, s, a);
  else if (first)
    hipLaunchKernelGGL((k_match_bm<KT, true, false>), dim3(grid), dim3(64), 0, s, a);
  else if (last)
    hipLaunchKernelGGL((k_match_bm<KT, false, true>), dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_match_bm<KT, false, false>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_match_bm(const BmArgs& a, int K, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (K <= 2) return launch_bm_k<2>(a, grid, s);
  if (K <= 4) return launch_bm_k<4>(a, grid, s);
  if (K <= 8) return launch_bm_k<8>(a, grid, s);
  if (K <= 16) return launch_bm_k<16>(a, grid, s);
  return launch_bm_k<32>(a, grid, s);
}

}  // namespace chm

// Cascade-hashing matching of directed image pairs (Sec. 2.3.1 steps (1)-(4)).
//
// One lane owns one query descriptor x_i of the query image:
//  (1) for each table t it walks the db image's bucket beta_t(x_i); the
//      bucket's members (16 j for db index j, ascending, padded to whole
//      blocks) are read as aligned 32-byte blocks of eight, one block ahead
//      of use, and the codes of a block are read before the previous
//      block's insertions run;
//  (2) for each candidate j it forms h = popcount(c(x_i) xor c(y_j)) over the
//      128-bit long codes and the key (h << 24) | 16 j, whose order is the
//      paper's ranking by Hamming distance with ties broken by db index;
//  (3) it keeps the KT smallest distinct keys in registers: a sorted list
//      updated with median-of-three steps; a key equal to a kept one is a
//      candidate an earlier table already returned (or a pad of the bucket,
//      a copy of its first member) and is dropped, which makes the
//      candidate list a set (a key equal to the last kept one leaves the
//      list unchanged, so it needs no test).  Keys of a block of eight
//      candidates are computed first; only those below the current KT-th
//      key are inserted, one per lane per round, selected with wave masks.
//      The walk's first blocks, while every lane is in its first bucket
//      (where only pads can repeat a key), are sorted and merged whole;
//  (4) for the first K kept candidates it computes the exact squared distance
//      ||x||^2 + ||y||^2 - 2 x.y with packed-u8 dot products and int32
//      accumulation, and applies the ratio test on squared distances
//      (den^2 * d1 < num^2 * d2).  The lanes of the wavefront share this
//      step: groups of kRerankLanes lanes read whole candidate descriptors
//      for one query at a time.  Two other readings are flags: a lone
//      candidate accepted, and the whole tie class of the K-th candidate
//      re-ranked (a second, per-lane walk).
//
// Work items are (pair, query range); an item's queries are taken in order
// of walk length, so the lanes of a wavefront walk about as far.  Batched
// plans run one persistent grid that dequeues items with atomic counters,
// one bin of items per XCD (the items of a db image share a bin, so its
// data stays in that XCD's L2); inside a work-group, wavefronts take
// 64-query chunks of the item dynamically.  Plain plans launch one grid per
// pair.  With LDSC the db image's codes and bucket offsets are staged in LDS
// once per item (skipped when consecutive items share the db image); db
// images too large for the stage are read from their bucket-ordered code
// copy, in the same launch.
#include <atomic>

#include "match_common.h"

namespace chm {

// Blocks of a walk merged whole into the kept list (KT = 8) while every
// lane is in its first bucket: the first and up to this many - 1 more.
constexpr int kMergeBlocks = 3;

// Called by all 64 lanes of the wavefront (the re-rank is cooperative);
// a lane with valid false owns no query (q is any valid index) and writes
// nothing.
template <int KT, bool LDSC, typename OffPtr>
__device__ __forceinline__ void match_query(const MatchArgs& a, const PairDev& P, int q, bool valid,
                                            OffPtr offs) {
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

  // Members of table t start at byte 4 * t * m_stride; bucket ranges are
  // padded to whole aligned blocks of 8, so every slot of a block is a
  // member of the bucket or a copy of its first member.  A member is the
  // byte offset 16 j of db point j's code, and keys (h << 24) | 16 j order
  // like (h, j).
  const char* mbase = uniform_ptr(P.d.members);
  const char* gcodes = uniform_ptr(P.d.codes);
  const char* tcodes = P.d.tcodes ? uniform_ptr(P.d.tcodes) : nullptr;
  const uint32_t mstride = 4u * (uint32_t)P.d.m_stride;
  const int stride = a.nb + 1;
  // Walk the L buckets as one sequence of aligned 8-member blocks; toff and
  // ob follow table t (byte offset of its members, index of its offsets).
  int t = -1, p = 0, e = 0, ob = -stride;
  uint32_t toff = 0u - mstride;
  auto next_table = [&]() {
    for (++t; t < a.L; ++t) {
      toff += mstride;
      ob += stride;
      const uint32_t b = ((t < 4 ? qb0 >> (8 * t) : qb1 >> (8 * (t - 4)))) & 0xFFu;
      p = offs[ob + b];
      e = offs[ob + b + 1];
      if (p < e) return;
    }
  };
  // Insertion of a block's passing keys: each round every lane takes its
  // lowest remaining passing slot (lanes with none take kNoKey, a no-op), so
  // the rounds follow the largest per-lane pass count of the wave and the
  // selection runs on the wave masks.
  auto drain = [&](const uint32_t (&key)[8], uint64_t (&pass)[8]) {
    uint64_t any = pass[0] | pass[1] | pass[2] | pass[3] | pass[4] | pass[5] | pass[6] | pass[7];
    while (any) {
      uint32_t x = kNoKey;
#pragma unroll
      for (int k = 7; k >= 0; --k) x = sel_lanes(pass[k], key[k], x);
      uint64_t seen = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint64_t rest = pass[k] & seen;
        seen |= pass[k];
        pass[k] = rest;
      }
      any = pass[0] | pass[1] | pass[2] | pass[3] | pass[4] | pass[5] | pass[6] | pass[7];
      insert_unique<KT>(top, x);
    }
    thr = top[KT - 1];
  };
  // One block: its 8 code reads are issued first, the previous block's
  // insertions run while they are in flight, then the block's keys and, per
  // slot, the wave mask of lanes whose key could enter the kept list (below
  // the current KT-th key) are formed; they wait for the next step.  A lane
  // without a block (valid false) reads a harmless one and passes nothing.
  uint32_t pkey[8];
  uint64_t ppass[8];
  auto step = [&](const uint4& x0, const uint4& x1, uint32_t moff, bool valid) {
    const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    uint4 c[8];
    if (!LDSC && tcodes) {  // the block's codes, contiguous at 4x its members' offset
#pragma unroll
      for (int k = 0; k < 8; ++k) c[k] = ldg4(tcodes + 4u * moff + 16u * k);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) c[k] = code_at<LDSC>(gcodes, w[k]);
    }
    drain(pkey, ppass);
    const uint32_t lim = valid ? thr : 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t h = bcnt_acc(qc.w ^ c[k].w,
                                  bcnt_acc(qc.z ^ c[k].z, bcnt_acc(qc.y ^ c[k].y, bcnt_acc(qc.x ^ c[k].x, 0u))));
      pkey[k] = (h << 24) | w[k];
      ppass[k] = __ballot(pkey[k] < lim);
    }
  };
  // Members of the lane's next block, or of the table's first block (always
  // present when any lane of the wave has a block) for a lane without one.
  auto load = [&](uint4& x0, uint4& x1, uint32_t& off, bool valid) {
    off = valid ? toff + 4u * (uint32_t)p : 0u;
    x0 = ldg4(mbase + off);
    x1 = ldg4(mbase + off + 16u);
  };
  auto advance = [&]() {
    p += 8;
    if (p >= e) next_table();
    return t < a.L;
  };
  // The wave steps through blocks together (lanes with fewer blocks idle
  // through the rest); two member register sets alternate, so the next
  // block's members load while this block is used.
  if (valid) next_table();
  else t = a.L;
  bool cur = t < a.L;
  if (__ballot(cur) != 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      pkey[k] = kNoKey;
      ppass[k] = 0;
    }
    uint4 A0, A1, B0, B1;
    uint32_t offA, offB;
    load(A0, A1, offA, cur);
    // While every lane of the wave is still in its first bucket, a block
    // needs no insertion rounds: the members of one bucket are distinct, so
    // the only keys that can repeat a kept one are pads (copies of the
    // bucket's first member w0), which are masked; the block's keys are
    // sorted and merged with the list whole.  The walk's first block (an
    // empty list) is done so for KT < 8, kMergeBlocks blocks for KT = 8.
    const int t0 = t;
    int tA = t0, tB = t0;
    int merge_left = KT == 8 ? kMergeBlocks : KT < 8 ? 1 : 0;  // (longer lists: registers)
    bool first = true;
    uint32_t w0 = 0;
    auto merge = [&](const uint4& x0, const uint4& x1, bool valid, int tblk) {
      if (merge_left <= 0) return;
      if (__ballot(valid && tblk != t0) != 0) {
        merge_left = 0;
        return;
      }
      --merge_left;
      const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
      if (first) w0 = w[0];
      uint32_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = (!valid || (w[k] == w0 && (k > 0 || !first))) ? kNoKey : pkey[k];
      sort8(v);
      if constexpr (KT == 8) {
        merge8_lowest(top, v);
      } else {
#pragma unroll
        for (int k = 0; k < KT; ++k) top[k] = k < 8 ? v[k & 7] : kNoKey;
      }
      first = false;
      thr = top[KT - 1];
#pragma unroll
      for (int k = 0; k < 8; ++k) ppass[k] = 0;
    };
    for (;;) {
      const bool nb = cur && advance();
      load(B0, B1, offB, nb);
      tB = t;
      step(A0, A1, offA, cur);
      merge(A0, A1, cur, tA);
      cur = nb;
      if (__ballot(cur) == 0) break;
      const bool na = cur && advance();
      load(A0, A1, offA, na);
      tA = t;
      step(B0, B1, offB, cur);
      merge(B0, B1, cur, tB);
      cur = na;
      if (__ballot(cur) == 0) break;
    }
    drain(pkey, ppass);
  }

  const int64_t o = P.out_off + q;
  if (a.topk && valid) {  // keys as (h << 24) | j
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (k < a.K)
        a.topk[o * a.K + k] = top[k] == kNoKey ? kNoKey : (top[k] & 0xFF000000u) | ((top[k] & 0xFFFFFFu) >> 4);
  }

  if (a.whole_bucket) {  // uniform: the variant that re-ranks the K-th's whole tie class
    // Hamming distance of the K-th candidate (or of the last, with fewer)
    uint32_t hk = 0;
    bool any = false;
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (k < a.K && top[k] != kNoKey) {
        hk = top[k] >> 24;
        any = true;
      }
    uint32_t d1 = 0xFFFFFFFFu, d2 = 0xFFFFFFFFu;
    int j1 = -1, cnt = 0;
    if (valid && any) {
      // a second walk over the query's buckets: each candidate once (pads
      // repeat the bucket's first member; a candidate that shares the
      // query's bucket in an earlier table was seen there), every one
      // within hk re-ranked by exact distance
      const uint4* xq = reinterpret_cast<const uint4*>(P.q.desc + (size_t)q * kDim);
      const uint32_t nq = *(gcu32*)(P.q.norms + q);
      for (int tt = 0; tt < a.L; ++tt) {
        const uint32_t bq = ((tt < 4 ? qb0 >> (8 * tt) : qb1 >> (8 * (tt - 4)))) & 0xFFu;
        const int s0 = offs[tt * stride + bq], s1 = offs[tt * stride + bq + 1];
        if (s0 >= s1) continue;
        const uint32_t tpos = (uint32_t)tt * (uint32_t)P.d.m_stride;
        const uint32_t first = *(gcu32*)(mbase + 4u * (tpos + (uint32_t)s0));
        for (int sp = s0; sp < s1; ++sp) {
          const uint32_t w = *(gcu32*)(mbase + 4u * (tpos + (uint32_t)sp));
          if (sp > s0 && w == first) continue;  // a pad
          const uint4 c = (!LDSC && tcodes) ? ldg4(tcodes + 16u * (tpos + (uint32_t)sp)) : code_at<LDSC>(gcodes, w);
          const uint32_t h = bcnt_acc(qc.w ^ c.w, bcnt_acc(qc.z ^ c.z, bcnt_acc(qc.y ^ c.y, bcnt_acc(qc.x ^ c.x, 0u))));
          if (h > hk) continue;
          const uint32_t j = w >> 4;
          bool seen = false;
          for (int t2 = 0; t2 < tt; ++t2) {
            const uint32_t b2 = ((t2 < 4 ? qb0 >> (8 * t2) : qb1 >> (8 * (t2 - 4)))) & 0xFFu;
            seen |= *(gcu8*)(P.d.ids + (size_t)t2 * P.d.n_pad + j) == b2;
          }
          if (seen) continue;
          const uint4* yp = reinterpret_cast<const uint4*>(P.d.desc + (size_t)j * kDim);
          uint32_t dot = 0;
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            const uint4 x = ldg4(xq + v), y = ldg4(yp + v);
            dot = __builtin_amdgcn_udot4(x.x, y.x, dot, false);
            dot = __builtin_amdgcn_udot4(x.y, y.y, dot, false);
            dot = __builtin_amdgcn_udot4(x.z, y.z, dot, false);
            dot = __builtin_amdgcn_udot4(x.w, y.w, dot, false);
          }
          const uint32_t e2 = nq + *(gcu32*)(P.d.norms + j) - 2u * dot;
          if (e2 < d1 || (e2 == d1 && (int)j < j1)) {  // candidate order: by distance, then index
            d2 = d1;
            d1 = e2;
            j1 = (int)j;
          } else {
            d2 = min(d2, e2);
          }
          ++cnt;
        }
      }
    }
    const bool pass = cnt >= 2 ? (uint64_t)a.ratio_den * (uint64_t)a.ratio_den * d1 <
                                     (uint64_t)a.ratio_num * (uint64_t)a.ratio_num * d2
                               : cnt == 1 && a.accept_single != 0;
    if (valid) a.out[o] = pass ? j1 : -1;
    return;
  }

  // Exact re-rank of the first K candidates and ratio test, with the
  // wavefront's lanes in groups of kRerankLanes: in round g, group r serves
  // the query of lane (64 / kRerankLanes) g + r, each of its lanes reading
  // one 128 / kRerankLanes-byte slice of the query and of candidate k, so a
  // load instruction covers whole descriptors.  The group sums its partial
  // dot products across its lanes, keeps the two smallest distances in
  // candidate order, applies the ratio test and hands the verdict to the
  // query's own lane.
  constexpr int G = kRerankLanes;
  constexpr int NG = 64 / G;             // groups (queries served per round)
  constexpr int SL = kDim / G / 16;      // 16-byte loads per lane per descriptor
  const int lane = __lane_id();
  const uint32_t xoff = (uint32_t)(lane % G) * (kDim / G);
  const char* qdesc = uniform_ptr(P.q.desc);
  const char* ddesc = uniform_ptr(P.d.desc);
  const char* qnorm = uniform_ptr(P.q.norms);
  const char* dnorm = uniform_ptr(P.d.norms);
  int result = -1;
  if (P.d.n > 0) {  // else no query has a candidate (and row 0 does not exist)
#pragma unroll 1
    for (int g = 0; g < G; ++g) {
      const int src = NG * g + lane / G;
      const uint32_t qs = lane_read((uint32_t)q, src);
      const bool vs = lane_read(valid ? 1u : 0u, src) != 0u;
      uint4 xs[SL];
#pragma unroll
      for (int v = 0; v < SL; ++v) xs[v] = ldg4(qdesc + (qs * (uint32_t)kDim + xoff + 16u * v));
      const uint32_t nqs = *(gcu32*)(qnorm + 4u * qs);
      uint32_t d1 = 0xFFFFFFFFu, d2 = 0xFFFFFFFFu, j1 = 0xFFFFFFFFu, cnt = 0;
      // candidates in chunks of KB (loads of a chunk, then its arithmetic)
      constexpr int KB = KT < 8 / SL ? KT : 8 / SL;
#pragma unroll
      for (int k0 = 0; k0 < KT; k0 += KB) {
        uint4 y[KB][SL];
        uint32_t ny[KB], jj[KB];
        bool ok[KB];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {  // loads of the candidates first
          const uint32_t key = lane_read(top[k0 + kk], src);
          ok[kk] = vs && k0 + kk < a.K && key != kNoKey;
          jj[kk] = (key & 0xFFFFFFu) >> 4;
          const uint32_t j = ok[kk] ? jj[kk] : 0u;  // a lane without a candidate reads row 0
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
          j1 = e2 < d1 ? jj[kk] : j1;     // first strictly smallest in candidate order
          d2 = med3u(d1, e2, d2);         // second smallest of {d1, d2, e2} (d1 <= d2)
          d1 = min(d1, e2);
          cnt += ok[kk] ? 1u : 0u;
        }
      }
      // d2 is infinite with one candidate: it passes only under accept_single
      const bool pass = cnt >= 2 ? (uint64_t)a.ratio_den * (uint64_t)a.ratio_den * d1 <
                                       (uint64_t)a.ratio_num * (uint64_t)a.ratio_num * d2
                                 : cnt == 1 && a.accept_single != 0;
      const uint32_t got = lane_read(pass ? j1 : 0xFFFFFFFFu, (lane % NG) * G);
      if (lane / NG == g) result = (int)got;
    }
  }
  if (valid) a.out[o] = result;
}

// LDS of the per-item query sort: order (u16 per query) and histogram.
struct SortLds {
  uint16_t* order;
  uint32_t* hist;
};

// Sort key of a query: 255 less its walk length (aligned blocks over the L
// buckets, clamped to 255), so that ascending keys are longest walks first.
template <typename OffPtr>
__device__ __forceinline__ int walk_key(const MatchArgs& a, const PairDev& P, int q, OffPtr offs) {
  const int stride = a.nb + 1;
  int len = 0;
  for (int t = 0; t < a.L; ++t) {
    const int b = *(gcu8*)(P.q.ids + (size_t)t * P.q.n_pad + q);
    len += (offs[t * stride + b + 1] - offs[t * stride + b]) >> 3;
  }
  return 255 - min(len, 255);
}

// Orders the item's queries by their walk length, longest first, so that
// the 64 lanes of a wavefront walk about as many blocks each (a counting
// sort; the key is computed again for the scatter rather than stored).
// Equal lengths come in any order: every query's result is independent of
// who computes it and when.
template <int WG, typename OffPtr>
__device__ __forceinline__ void sort_item(const MatchArgs& a, const PairDev& P, const WorkItem& w,
                                          OffPtr offs, const SortLds& s) {
  const int nq = w.q1 - w.q0;
  for (int i = threadIdx.x; i < 256; i += WG) s.hist[i] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < nq; i += WG) atomicAdd(&s.hist[walk_key(a, P, w.q0 + i, offs)], 1u);
  __syncthreads();
  if (threadIdx.x < 64) {  // exclusive scan, 4 bins per lane
    const int lane = threadIdx.x;
    uint32_t v[4], run = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = s.hist[4 * lane + k];
      run += v[k];
    }
    const uint32_t incl = wave_incl_add(run);
    uint32_t base = incl - run;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s.hist[4 * lane + k] = base;
      base += v[k];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nq; i += WG)
    s.order[atomicAdd(&s.hist[walk_key(a, P, w.q0 + i, offs)], 1u)] = (uint16_t)i;
  __syncthreads();
}

template <int KT, bool LDSC, int WG, typename OffPtr>
__device__ __forceinline__ void run_item(const MatchArgs& a, const PairDev& P, const WorkItem& w,
                                         OffPtr offs, int* s_chunk, const SortLds& s, bool sorted) {
  if (sorted) sort_item<WG>(a, P, w, offs, s);
  // Wavefronts take 64-query chunks of the item in turn.
  const int lane = __lane_id();
  for (;;) {
    int c = 0;
    if (lane == 0) c = atomicAdd(s_chunk, 64);
    c = __builtin_amdgcn_readfirstlane(__shfl(c, 0));  // uniform across the wave
    if (w.q0 + c >= w.q1) break;
    const int i = c + lane;
    const bool valid = w.q0 + i < w.q1;
    const int qi = valid ? (sorted ? (int)s.order[i] : i) : 0;
    match_query<KT, LDSC>(a, P, w.q0 + qi, valid, offs);
  }
}

template <int KT, int WG, bool LDSC, bool PERSIST>
__global__ __launch_bounds__(WG) void k_match(MatchArgs a) {
  // All LDS is dynamic: the staged codes from address 0, so a code's LDS
  // address is its member value (16 j) itself; the control words and the
  // sort histogram at the top; an item's sort order just below them.
  extern __shared__ uint4 smem[];
  char* lds = reinterpret_cast<char*>(smem);
  const int top = LDSC ? a.lds_top : 2 * kSortMax;
  const int ncodes = LDSC ? a.lds_max_feats : 0;
  const int offs_bytes = (a.L * (a.nb + 1) * 4 + 15) & ~15;
  int* sCtl = reinterpret_cast<int*>(lds + top);
  int& s_item = sCtl[0];
  int& s_chunk = sCtl[1];
  SortLds sl;
  sl.hist = reinterpret_cast<uint32_t*>(sCtl + 4);
  const uint4* staged = nullptr;
  int stage_end = 0;        // bytes of LDS the current stage occupies
  bool staged_offs = false;  // whether they include the bucket offsets
  int it = PERSIST ? 0 : a.item_base + (int)blockIdx.x;
  // Persistent: start with the bin of this work-group's XCD (work-groups
  // are dealt to the XCDs round-robin), then help the other bins in turn.
  // Each bin is left after one failed dequeue, so every work-group ends
  // after at most n_items + n_bins dequeues.
  int bin = PERSIST ? (int)(blockIdx.x % (unsigned)a.n_bins) : 0, visited = 0;

  for (;;) {
    if (PERSIST) {
      if (threadIdx.x == 0) {
        int got = -1;
        while (visited < a.n_bins) {
          const int b0 = a.bin_begin[bin], b1 = a.bin_begin[bin + 1];
          if (b0 < b1) {
            const int i = (int)atomicAdd(a.queue + bin, 1u);
            if (i < b1 - b0) {
              got = b0 + i;
              break;
            }
          }
          bin = bin + 1 == a.n_bins ? 0 : bin + 1;
          ++visited;
        }
        s_item = got;
      }
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(s_item);  // uniform: item fields in SGPRs
      if (it < 0) break;
    }
    if (threadIdx.x == 0) s_chunk = 0;
    const WorkItem w = a.items[it];
    const PairDev& P = a.pairs[w.pair];
    const bool use_lds = LDSC && P.d.n <= ncodes;
    if (use_lds && staged != P.d.codes) {
      // the offsets join the stage when a full-size sort still fits above it
      const int code_bytes = 16 * P.d.n;
      staged_offs = code_bytes + offs_bytes + 2 * kSortMax <= top;
      stage_end = code_bytes + (staged_offs ? offs_bytes : 0);
      for (int j = threadIdx.x; j < P.d.n; j += WG) smem[j] = ldg4(P.d.codes + j);
      if (staged_offs) {
        int32_t* so = reinterpret_cast<int32_t*>(lds + code_bytes);
        for (int i = threadIdx.x; i < a.L * (a.nb + 1); i += WG) so[i] = *(gci32*)(P.d.offsets + i);
      }
      staged = P.d.codes;
    }
    const int nq = w.q1 - w.q0;
    const bool sorted = nq <= kSortMax && top - 2 * nq >= (use_lds ? stage_end : 0);
    if (sorted && !use_lds && top - 2 * nq < stage_end) staged = nullptr;  // the order overwrites the stage
    sl.order = reinterpret_cast<uint16_t*>(lds + top - 2 * (sorted ? nq : 0));
    __syncthreads();
    // The offsets pointer carries its address space in its type, so each
    // walk reads them with LDS or global loads, not flat ones.
    gci32* goffs = (gci32*)P.d.offsets;
    if (use_lds && staged_offs)
      run_item<KT, true, WG>(a, P, w, reinterpret_cast<lds_ci32*>((size_t)(16 * P.d.n)), &s_chunk, sl, sorted);
    else if (use_lds)
      run_item<KT, true, WG>(a, P, w, goffs, &s_chunk, sl, sorted);
    else
      run_item<KT, false, WG>(a, P, w, goffs, &s_chunk, sl, sorted);
    __syncthreads();
    if (!PERSIST) break;
  }
}


template <int KT, int WG, bool LDSC, bool PERSIST>
static hipError_t launch_one(const MatchArgs& a, int grid, hipStream_t s) {
  const size_t lds = LDSC ? (size_t)a.lds_top + kLdsTop : kMatchLdsTail;
  auto fn = k_match<KT, WG, LDSC, PERSIST>;
  // The code stage must start at LDS address 0: the kernel may have no
  // static LDS.  That is a property of the one code object (the same on
  // every device), read once per process; concurrent first calls store the
  // same value.
  static std::atomic<int> static_lds{-1};
  int sl = static_lds.load(std::memory_order_relaxed);
  if (sl < 0) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(fn));
    if (e != hipSuccess) return e;
    sl = (int)attr.sharedSizeBytes;
    static_lds.store(sl, std::memory_order_relaxed);
  }
  if (sl != 0) return hipErrorInvalidKernelFile;
  {
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

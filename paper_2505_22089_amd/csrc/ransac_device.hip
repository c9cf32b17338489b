// RANSAC global verification (Sec. 2.3.3) on the device: the computation
// of chm_ransac_filter (2D similarity through two matches, exact integer
// inlier test, the best hypothesis verifies the pair when it has enough
// inliers), one work-group per pair at a time.
//
// A pair's matches are first compacted, in query-row order, into the
// work-group's scratch: (p_x, p_y, q_x, q_y) and (query row, db row) per
// match.  Hypotheses are then taken 64 at a time, one per lane: every
// wavefront walks a quarter of the matches, each match read once per
// wavefront (the same address in every lane) and tested against the
// lane's hypothesis; the four partial counts of a hypothesis are summed in
// LDS.  The best hypothesis (most inliers, the earlier on ties) is a max
// over packed keys (count + 1) << 32 | ~t.  Inputs that break the
// contract (a db row outside the db image, a coordinate out of range) make
// the pair verify nothing and are counted in the work buffer's first word.
//
// Exactness: coordinates are below 2^19 in magnitude, so differences are
// below 2^20, D = |dp|^2 and the components of w = dq conj(dp) below 2^41,
// each residual component D f - (w e) below 3 * 2^61 (exact in int64), and
// its square and the limit D^2 thr^2 below 2^126 (exact in a signed 128-bit
// integer): the same values as the host's.
#include <algorithm>
#include <vector>

#include "chm.h"
#include "chm_host.h"
#include "chm_internal.h"

namespace chm {

namespace {

constexpr int kRansacWG = 256;
constexpr int kRansacGrid = 512;  // work-groups resident at once (two per CU)
constexpr int64_t kCoordLimit = int64_t(1) << 19;

struct RansacPair {
  const int32_t* kq;   // query keypoints (x, y)
  const int32_t* kd;   // db keypoints
  int64_t start;       // first row of the pair in the match / output arrays
  int32_t nq;
  int32_t nd;
  int32_t word_pair;   // the pair's index in the caller's list (its random words, its count)
  int32_t pad;
};
static_assert(sizeof(RansacPair) == 40, "table entry layout");

struct RansacArgs {
  const RansacPair* pairs;
  int32_t n_pairs;
  const int32_t* match;
  const uint32_t* words;
  int32_t iterations;
  int64_t thr;
  int32_t min_inliers;
  int32_t* out;
  int32_t* best_counts;
  uint8_t* scratch;
  uint64_t scratch_stride;  // bytes per work-group
  int32_t n_max;            // capacity in matches of a work-group's scratch
  int32_t* errors;
};

struct Sim {
  int64_t pix, piy, qix, qiy, D, wr, wi;
};

__device__ __forceinline__ Sim make_sim(const int4& a, const int4& b) {
  Sim s;
  s.pix = a.x;
  s.piy = a.y;
  s.qix = a.z;
  s.qiy = a.w;
  const int64_t dpx = (int64_t)b.x - s.pix, dpy = (int64_t)b.y - s.piy;
  const int64_t dqx = (int64_t)b.z - s.qix, dqy = (int64_t)b.w - s.qiy;
  s.D = dpx * dpx + dpy * dpy;
  s.wr = dqx * dpx + dqy * dpy;
  s.wi = dqy * dpx - dqx * dpy;
  return s;
}

__device__ __forceinline__ bool inlier(const Sim& s, const int4& k, __int128 lim) {
  const int64_t ex = (int64_t)k.x - s.pix, ey = (int64_t)k.y - s.piy;
  const int64_t fx = (int64_t)k.z - s.qix, fy = (int64_t)k.w - s.qiy;
  const int64_t rx = s.D * fx - (s.wr * ex - s.wi * ey);
  const int64_t ry = s.D * fy - (s.wr * ey + s.wi * ex);
  return (__int128)rx * rx + (__int128)ry * ry <= lim;
}

// Hypothesis t of a pair with M >= 2 matches: matches i and j.
__device__ __forceinline__ void pick(const uint32_t* w, int t, int M, int* i, int* j) {
  *i = (int)(w[2 * t] % (uint32_t)M);
  int jj = (int)(w[2 * t + 1] % (uint32_t)(M - 1));
  *j = jj >= *i ? jj + 1 : jj;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    v = o > v ? o : v;
  }
  return v;
}

__global__ __launch_bounds__(kRansacWG) void k_ransac(RansacArgs a) {
  __shared__ int32_t sWave[kRansacWG / 64];
  __shared__ int32_t sBad;
  __shared__ uint32_t sCnt[kRansacWG];
  __shared__ uint64_t sBest;
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int wave = tid >> 6;
  int4* PQ = reinterpret_cast<int4*>(a.scratch + (uint64_t)blockIdx.x * a.scratch_stride);
  int2* RM = reinterpret_cast<int2*>(PQ + a.n_max);
  const int64_t thr2 = a.thr * a.thr;
  for (int e = blockIdx.x; e < a.n_pairs; e += gridDim.x) {
    const RansacPair pr = a.pairs[e];
    if (tid == 0) sBad = 0;
    __syncthreads();
    // 1. the matches in query-row order
    int M = 0;
    for (int r0 = 0; r0 < pr.nq; r0 += kRansacWG) {
      const int r = r0 + tid;
      const int m = r < pr.nq ? a.match[pr.start + r] : -1;
      bool ok = m >= 0;
      int4 v = make_int4(0, 0, 0, 0);
      if (ok) {
        if (m >= pr.nd) {
          ok = false;
          atomicOr(&sBad, 1);
        } else {
          v = make_int4(pr.kq[2 * (size_t)r], pr.kq[2 * (size_t)r + 1], pr.kd[2 * (size_t)m],
                        pr.kd[2 * (size_t)m + 1]);
          const int32_t c[4] = {v.x, v.y, v.z, v.w};
          for (int q = 0; q < 4; ++q)
            if (c[q] <= -kCoordLimit || c[q] >= kCoordLimit) atomicOr(&sBad, 1);
        }
      }
      const uint64_t bal = __ballot(ok);
      const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (lane == 0) sWave[wave] = __popcll(bal);
      __syncthreads();
      int off = M;
      for (int w = 0; w < wave; ++w) off += sWave[w];
      int tot = 0;
      for (int w = 0; w < kRansacWG / 64; ++w) tot += sWave[w];
      if (ok) {
        PQ[off + before] = v;
        RM[off + before] = make_int2(r, m);
      }
      M += tot;
      __syncthreads();  // sWave is rewritten by the next chunk
    }
    // 2. every row unverified until shown otherwise (all reads of the
    // matches are done: the output may alias them)
    for (int r = tid; r < pr.nq; r += kRansacWG) a.out[pr.start + r] = -1;
    __syncthreads();  // the scratch and sBad are complete
    const bool bad = sBad != 0;
    if (bad) {
      if (tid == 0) {
        atomicAdd(a.errors, 1);
        if (a.best_counts) a.best_counts[pr.word_pair] = 0;
      }
      continue;  // uniform
    }
    const uint32_t* w = a.words + (size_t)pr.word_pair * (size_t)a.iterations * 2;
    // 3. hypotheses, 64 at a time; wavefront `wave` walks matches wave, wave + 4, ...
    uint64_t best = 0;
    if (M >= 2) {
      for (int t0 = 0; t0 < a.iterations; t0 += 64) {
        const int t = t0 + lane;
        bool ok = t < a.iterations;
        Sim s = {0, 0, 0, 0, 0, 0, 0};
        if (ok) {
          int i, j;
          pick(w, t, M, &i, &j);
          s = make_sim(PQ[i], PQ[j]);
          ok = s.D != 0;
        }
        const __int128 lim = (__int128)s.D * (__int128)s.D * (__int128)thr2;
        uint32_t c = 0;
        for (int k = wave; k < M; k += kRansacWG / 64) {
          const int4 pk = PQ[k];
          c += (ok && inlier(s, pk, lim)) ? 1u : 0u;
        }
        sCnt[tid] = c;
        __syncthreads();
        if (wave == 0) {
          uint32_t sum = 0;
          for (int v = 0; v < kRansacWG / 64; ++v) sum += sCnt[lane + 64 * v];
          const uint64_t key = ok ? ((uint64_t)(sum + 1) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)t) : 0ull;
          best = key > best ? key : best;
        }
        __syncthreads();  // sCnt is rewritten by the next group
      }
      if (wave == 0) {
        best = wave_max_u64(best);
        if (lane == 0) sBest = best;
      }
    } else if (tid == 0) {
      sBest = 0;
    }
    __syncthreads();
    best = sBest;
    const int nbest = best ? (int)(best >> 32) - 1 : -1;
    if (a.best_counts && tid == 0) a.best_counts[pr.word_pair] = max(nbest, 0);
    // 4. the best hypothesis' inliers are the verified matches
    if (nbest >= 0 && nbest >= a.min_inliers) {
      const int tb = (int)(0xFFFFFFFFu - (uint32_t)best);
      int i, j;
      pick(w, tb, M, &i, &j);
      const Sim s = make_sim(PQ[i], PQ[j]);
      const __int128 lim = (__int128)s.D * (__int128)s.D * (__int128)thr2;
      for (int k = tid; k < M; k += kRansacWG)
        if (inlier(s, PQ[k], lim)) {
          const int2 rm = RM[k];
          a.out[pr.start + rm.x] = rm.y;
        }
    }
    __syncthreads();  // the scratch is rewritten by the next pair
  }
}

uint64_t round256(uint64_t x) { return (x + 255) & ~255ull; }

uint64_t scratch_stride(int32_t n_max) { return round256(24ull * (uint64_t)std::max(n_max, 1)); }

}  // namespace

uint64_t ransac_work_bytes(int32_t n_pairs, int32_t max_rows) {
  return 256 + round256(sizeof(RansacPair) * (uint64_t)std::max(n_pairs, 0)) +
         (uint64_t)kRansacGrid * scratch_stride(max_rows);
}

hipError_t ransac_upload(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                         const int32_t* h_n_feats, const int64_t* h_starts, const int32_t* word_pair,
                         void* d_work, hipStream_t s) {
  std::vector<RansacPair> hp((size_t)n_pairs);
  for (int32_t p = 0; p < n_pairs; ++p) {
    const int32_t q = h_pairs[2 * p], d = h_pairs[2 * p + 1];
    hp[(size_t)p] = RansacPair{d_kp[q], d_kp[d], h_starts[p], h_n_feats[q], h_n_feats[d],
                               word_pair ? word_pair[p] : p, 0};
  }
  uint8_t* w = static_cast<uint8_t*>(d_work);
  hipError_t e = hipSuccess;
  if (n_pairs > 0)
    e = hipMemcpyAsync(w + 256, hp.data(), sizeof(RansacPair) * hp.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // hp is freed on return
  return e;
}

hipError_t ransac_run(int32_t first, int32_t count, int32_t table_pairs, int32_t n_max, const int32_t* d_match,
                      const uint32_t* d_words, int32_t iterations, int32_t thr, int32_t min_inliers,
                      int32_t* d_out, int32_t* d_best_counts, void* d_work, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  uint8_t* w = static_cast<uint8_t*>(d_work);
  RansacArgs a;
  a.pairs = reinterpret_cast<const RansacPair*>(w + 256) + first;
  a.n_pairs = count;
  a.match = d_match;
  a.words = d_words;
  a.iterations = iterations;
  a.thr = thr;
  a.min_inliers = min_inliers;
  a.out = d_out;
  a.best_counts = d_best_counts;
  a.scratch = w + 256 + round256(sizeof(RansacPair) * (uint64_t)table_pairs);
  a.scratch_stride = scratch_stride(n_max);
  a.n_max = std::max(n_max, 1);
  a.errors = reinterpret_cast<int32_t*>(w);
  hipLaunchKernelGGL(k_ransac, dim3(std::min(count, kRansacGrid)), dim3(kRansacWG), 0, s, a);
  return hipGetLastError();
}

}  // namespace chm

extern "C" chm_status chm_ransac_work_bytes(int32_t n_pairs, int32_t max_query_rows, uint64_t* out_bytes) {
  chm::clear_error();
  if (!out_bytes || n_pairs < 0 || max_query_rows < 0) return chm::fail(CHM_E_INVALID_ARG, "bad arguments");
  *out_bytes = chm::ransac_work_bytes(n_pairs, max_query_rows);
  return CHM_OK;
}

extern "C" chm_status chm_ransac_filter_device(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                                               const int32_t* h_n_feats, int32_t n_images, const int64_t* h_offs,
                                               const int32_t* d_match, const uint32_t* d_words, int32_t iterations,
                                               int32_t thr, int32_t min_inliers, int32_t* d_out,
                                               int32_t* d_best_counts, void* d_work, uint64_t work_bytes,
                                               void* stream) {
  using namespace chm;
  clear_error();
  if (n_pairs < 0 || n_images < 0 || iterations < 0) return fail(CHM_E_INVALID_ARG, "negative count");
  if (n_pairs == 0) return CHM_OK;
  if (!h_pairs || !d_kp || !h_n_feats || !h_offs || !d_match || !d_out || !d_work || (iterations > 0 && !d_words))
    return fail(CHM_E_INVALID_ARG, "NULL array");
  if (thr < 0 || thr >= (1 << 20)) return fail(CHM_E_INVALID_ARG, "thr must be 0..2^20-1");
  if (reinterpret_cast<uintptr_t>(d_work) % 256) return fail(CHM_E_INVALID_ARG, "d_work must be 256-byte aligned");
  int32_t n_max = 0;
  for (int32_t p = 0; p < n_pairs; ++p) {
    const int32_t q = h_pairs[2 * p], d = h_pairs[2 * p + 1];
    if (q < 0 || q >= n_images || d < 0 || d >= n_images)
      return fail(CHM_E_INVALID_ARG, "pair %d names an image outside 0..%d", p, n_images - 1);
    if (h_n_feats[q] < 0 || h_n_feats[d] < 0) return fail(CHM_E_INVALID_ARG, "negative row count");
    if ((h_n_feats[q] > 0 && !d_kp[q]) || (h_n_feats[d] > 0 && !d_kp[d]))
      return fail(CHM_E_INVALID_ARG, "pair %d: NULL keypoints", p);
    if (h_offs[p] < 0 || h_offs[p + 1] - h_offs[p] != h_n_feats[q])
      return fail(CHM_E_INVALID_ARG, "pair %d: offsets do not span the query image's rows", p);
    n_max = std::max(n_max, h_n_feats[q]);
  }
  const uint64_t need = ransac_work_bytes(n_pairs, n_max);
  if (work_bytes < need)
    return fail(CHM_E_CAPACITY, "work buffer holds %llu bytes, %llu needed", (unsigned long long)work_bytes,
                (unsigned long long)need);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_fill_u32(static_cast<uint32_t*>(d_work), 0u, 1, s);
  if (e == hipSuccess) e = ransac_upload(n_pairs, h_pairs, d_kp, h_n_feats, h_offs, nullptr, d_work, s);
  if (e == hipSuccess)
    e = ransac_run(0, n_pairs, n_pairs, n_max, d_match, d_words, iterations, thr, min_inliers, d_out, d_best_counts,
                   d_work, s);
  if (e != hipSuccess) return fail(CHM_E_HIP, "RANSAC launch failed: %s", hipGetErrorString(e));
  return CHM_OK;
}

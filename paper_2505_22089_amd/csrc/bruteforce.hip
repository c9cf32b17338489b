// Exhaustive matching: every db descriptor is a candidate; the two nearest by
// exact squared distance and the ratio test of Sec. 2.3.1 step (4).
//
// The dense distance step is an int8 MFMA GEMM with int32 accumulation:
// with x' = x - 128 and y' = y - 128 (int8), ||x - y||^2 = ||x'||^2 +
// ||y'||^2 - 2 x'.y', all exact in int32.  For a query the nearest db rows
// are those with the largest score s = 2 x'.y' - ||y'||^2.  Each work-group
// owns 128 queries and one contiguous split of the db; every lane keeps a
// running top-2 of s for the 16 query rows its accumulators hold, over the
// db columns it sees; lanes are merged with butterflies and splits by a
// second kernel, which also applies the ratio test.
//
// The top-2 runs on packed keys T s + (T - 1 - c), c the column inside its
// T-column LDS tile (|s| < 2^23, so T = 256 still fits int32): one
// shift-add forms the key from the accumulator and a per-column bias, a max
// and a median-of-three keep the two largest, and the tile of the best key
// is recorded once per tile.  Ties between equal
// scores cannot change the output (equal best and second distances fail
// the ratio test for any t_r <= 1), so which column wins one is immaterial.
#include <climits>
#include <mutex>

#include "chm_internal.h"

namespace chm {

typedef int32_t i32x4v __attribute__((ext_vector_type(4)));
typedef int32_t i32x16v __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

#ifndef CHM_BF_WAVES
#define CHM_BF_WAVES 8
#endif
constexpr int kBfWaves = CHM_BF_WAVES;  // waves per work-group
// 32-query row blocks per wave: each staged db fragment feeds that many
// independent MFMA chains, which halves LDS reads per multiply-add at 2
#ifndef CHM_BF_ROWBLOCKS
#define CHM_BF_ROWBLOCKS 1
#endif
constexpr int kBfRB = CHM_BF_ROWBLOCKS;
constexpr int kBfQ = 32 * kBfRB * kBfWaves;  // queries per work-group
#ifndef CHM_BF_TILE
#define CHM_BF_TILE 256
#endif
constexpr int kBfD = CHM_BF_TILE;    // db rows per LDS tile
constexpr int kBfShift = kBfD == 256 ? 8 : 7;  // log2 kBfD
static_assert(kBfD == 128 || kBfD == 256, "tile of 128 or 256 db rows");
static_assert(64 * kBfWaves >= 2 * kBfD, "the tile stagers (two per row) are whole waves of the work-group");
// Key of an empty column (a zero row past the db): below every real key
// T s + (T - 1 - c) >= T (-2^22 - 2^21).
constexpr int32_t kBfEmpty = INT_MIN / 2 - (1 << 29);
constexpr int kBfStride = 144;       // bytes per staged row (pad spreads banks)
constexpr int kBfTargetWG = 1024;    // aim for this many work-groups (splits of the db)

__device__ __forceinline__ int32_t med3i(int32_t a, int32_t b, int32_t c) {
  int32_t r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

__device__ __forceinline__ void merge2(int32_t& s1, int32_t& j1, int32_t& s2, int32_t t1, int32_t u1,
                                       int32_t t2) {
  const int32_t lo = min(s1, t1);
  const int32_t nj = (t1 > s1 || (t1 == s1 && u1 < j1)) ? u1 : j1;
  s2 = max(lo, max(s2, t2));
  s1 = max(s1, t1);
  j1 = nj;
}

__global__ __launch_bounds__(64 * kBfWaves, 4) void k_bf_partial(const uint8_t* Q, int nq, const uint8_t* D,
                                                    int nd, int split_cols, int4* work) {
  __shared__ __attribute__((aligned(16))) uint8_t sD[kBfD * kBfStride];
  __shared__ int32_t sN[kBfD];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = __lane_id();
  const int half = lane >> 5;
  const int qbase = blockIdx.x * kBfQ + wave * 32 * kBfRB;  // the wave's first query row
  const int c0 = blockIdx.y * split_cols;
  const int c1 = min(nd, c0 + split_cols);

  i32x4v A[kBfRB][4];
#pragma unroll
  for (int rb = 0; rb < kBfRB; ++rb) {
    const int qr = qbase + 32 * rb + (lane & 31);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      u32x4v v = {0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u};
      if (qr < nq) v = *reinterpret_cast<const u32x4v*>(Q + (size_t)qr * kDim + 32 * ks + 16 * half);
      v ^= 0x80808080u;
      A[rb][ks] = __builtin_bit_cast(i32x4v, v);
    }
  }
  constexpr int E = 16 * kBfRB;  // accumulator elements per lane
  int32_t s1[E], s2[E], t1[E];   // best and second keys, tile of the best
#pragma unroll
  for (int e = 0; e < E; ++e) {
    s1[e] = INT_MIN;
    s2[e] = INT_MIN;
    t1[e] = -1;
  }

  for (int tile = c0; tile < c1; tile += kBfD) {
    __syncthreads();
    // the first 2 kBfD threads stage the tile, half a row each: 64 bytes as
    // four 16-byte pieces (whole waves, so the shuffle below is uniform)
    if (tid < 2 * kBfD) {
      const int row = tid >> 1, part = tid & 1;
      const int g = tile + row;
      int32_t nrm = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        u32x4v v = {0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u};
        if (g < c1) v = *reinterpret_cast<const u32x4v*>(D + (size_t)g * kDim + 64 * part + 16 * k);
        v ^= 0x80808080u;
        *reinterpret_cast<u32x4v*>(sD + row * kBfStride + 64 * part + 16 * k) = v;
#pragma unroll
        for (int w = 0; w < 4; ++w) nrm = __builtin_amdgcn_sdot4((int)v[w], (int)v[w], nrm, false);
      }
      nrm += __shfl_xor(nrm, 1);
      // key bias of the column: -T ||y'||^2 + (T - 1 - c); an empty column
      // (a zero row, dot 0) gets kBfEmpty, below every real key
      if (part == 0) sN[row] = (g < c1) ? -(nrm << kBfShift) + (kBfD - 1 - row) : kBfEmpty;
    }
    __syncthreads();
    int32_t before[E];
#pragma unroll
    for (int e = 0; e < E; ++e) before[e] = s1[e];
#pragma unroll
    for (int blk = 0; blk < kBfD / 32; ++blk) {
      const int crow = blk * 32 + (lane & 31);
      i32x16v acc[kBfRB];
#pragma unroll
      for (int rb = 0; rb < kBfRB; ++rb) acc[rb] = i32x16v{};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const i32x4v B = *reinterpret_cast<const i32x4v*>(sD + crow * kBfStride + 32 * ks + 16 * half);
#pragma unroll
        for (int rb = 0; rb < kBfRB; ++rb)
          acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[rb][ks], B, acc[rb], 0, 0, 0);
      }
      const int32_t bias = sN[crow];
#pragma unroll
      for (int rb = 0; rb < kBfRB; ++rb) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int32_t key = (acc[rb][e] << (kBfShift + 1)) + bias;  // T (2 x'.y' - ||y'||^2) + T - 1 - c
          s2[16 * rb + e] = med3i(s1[16 * rb + e], s2[16 * rb + e], key);
          s1[16 * rb + e] = max(s1[16 * rb + e], key);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) t1[e] = s1[e] != before[e] ? tile : t1[e];
  }
  // merge the 32 lanes that hold the same query rows (lanes of one half);
  // from here on a best key travels with its global column
  int32_t j1[E];
#pragma unroll
  for (int e = 0; e < E; ++e) j1[e] = s1[e] == INT_MIN ? -1 : t1[e] + (kBfD - 1 - (s1[e] & (kBfD - 1)));
#pragma unroll
  for (int e = 0; e < E; ++e) {
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
      const int32_t u = __shfl_xor(s1[e], d), uj = __shfl_xor(j1[e], d), u2 = __shfl_xor(s2[e], d);
      merge2(s1[e], j1[e], s2[e], u, uj, u2);
    }
    const int row = qbase + 32 * (e >> 4) + 8 * ((e & 15) >> 2) + 4 * half + (e & 3);
    if ((lane & 31) == 0 && row < nq) work[(size_t)blockIdx.y * nq + row] = make_int4(s1[e], j1[e], s2[e], 0);
  }
}

__global__ void k_bf_merge(const int4* work, int splits, const uint8_t* Q, int nq, int nd, int ra,
                           int rb, int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  int32_t s1 = INT_MIN, j1 = -1, s2 = INT_MIN;
  for (int sp = 0; sp < splits; ++sp) {
    const int4 v = work[(size_t)sp * nq + i];
    merge2(s1, j1, s2, v.x, v.y, v.z);
  }
  int32_t nrm = 0;
  const u32x4v* x = reinterpret_cast<const u32x4v*>(Q + (size_t)i * kDim);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const u32x4v v = x[k] ^ 0x80808080u;
#pragma unroll
    for (int w = 0; w < 4; ++w) nrm = __builtin_amdgcn_sdot4((int)v[w], (int)v[w], nrm, false);
  }
  if (nd < 2) {
    out[i] = -1;
    return;
  }
  // keys back to scores: s = key >> log2 T (arithmetic)
  const int64_t e1 = (int64_t)nrm - (s1 >> kBfShift), e2 = (int64_t)nrm - (s2 >> kBfShift);
  out[i] = ((int64_t)rb * rb * e1 < (int64_t)ra * ra * e2) ? j1 : -1;
}

// Workspace of chm_bruteforce_noalloc: a file-scope device array, one copy
// per GPU, holding the per-split partial top-2 of every query (16 B per
// query and split).  Host code never uses the array's name as an address:
// bruteforce_scratch() resolves this device's copy once and caches it.
__device__ __align__(256) uint8_t g_bf_scratch[kBfScratchBytes];

namespace {
std::mutex g_bf_scratch_mu;
void* g_bf_scratch_ptr[kBfScratchDevices] = {};
}  // namespace

hipError_t bruteforce_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kBfScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_bf_scratch_mu);
  if (!g_bf_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_bf_scratch));
    if (e != hipSuccess) return e;
    g_bf_scratch_ptr[dev] = p;
  }
  *out = g_bf_scratch_ptr[dev];
  return hipSuccess;
}

int bruteforce_splits(int nq, int nd) {
  const int qt = (nq + kBfQ - 1) / kBfQ;
  const int dt = (nd + kBfD - 1) / kBfD;
  int s = (kBfTargetWG + qt - 1) / (qt > 0 ? qt : 1);
  if (s > dt) s = dt;
  if (s < 1) s = 1;
  return s;
}

hipError_t launch_bruteforce(const uint8_t* q, int nq, const uint8_t* d, int nd, int ra, int rb,
                             int32_t* out, void* work, int splits, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const int dt = (nd + kBfD - 1) / kBfD;
  const int split_cols = ((dt + splits - 1) / splits) * kBfD;
  int4* w = reinterpret_cast<int4*>(work);
  if (nd > 0) {
    hipLaunchKernelGGL(k_bf_partial, dim3((nq + kBfQ - 1) / kBfQ, splits), dim3(64 * kBfWaves), 0, s, q, nq,
                       d, nd, split_cols, w);
  }
  hipLaunchKernelGGL(k_bf_merge, dim3((nq + 255) / 256), dim3(256), 0, s, w, nd > 0 ? splits : 0, q,
                     nq, nd, ra, rb, out);
  return hipGetLastError();
}

}  // namespace chm

// Exhaustive matching: every db descriptor is a candidate; the two nearest by
// exact squared distance and the ratio test of Sec. 2.3.1 step (4).
//
// The dense distance step is an int8 MFMA GEMM with int32 accumulation:
// with x' = x - 128 and y' = y - 128 (int8), ||x - y||^2 = ||x'||^2 +
// ||y'||^2 - 2 x'.y', all exact in int32.  For a query the nearest db rows
// are those with the largest score s = 2 x'.y' - ||y'||^2.  A pre-pass
// writes y' and each db row's key bias to the workspace once.  Each
// work-group owns 256 queries and one contiguous split of the db, which it
// walks in 256-row tiles: the tiles are copied straight from global memory
// into LDS (global_load_lds, two buffers: the next tile streams in while the
// current one is multiplied; 16-byte pieces XOR-swizzled by row so the
// operand reads of 16 rows fall on distinct banks).  Every lane keeps a
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
#include <algorithm>
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
constexpr int kBfD = 256;            // db rows per LDS tile
constexpr int kBfShift = 8;          // log2 kBfD
static_assert(32 * kBfWaves == kBfD, "each wave stages 32 rows of a tile");
// Key of an empty column (a zero row past the db): below every real key
// T s + (T - 1 - c) >= T (-2^22 - 2^21).
constexpr int32_t kBfEmpty = INT_MIN / 2 - (1 << 29);
constexpr int kBfSlots = 512;        // work-groups resident at once (two per CU)

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

// y' = y - 128 (the byte XOR 0x80) of every db row, zero rows up to a whole
// tile, and each row's key bias -T ||y'||^2 + (T - 1 - c), c = g mod T (an
// empty row gets kBfEmpty, below every real key).  Eight lanes per row.
__global__ void k_bf_prep(const uint8_t* D, int nd, int nd_pad, uint8_t* Dp, int32_t* bias) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = t >> 3, piece = t & 7;
  if (g >= nd_pad) return;  // whole rows: the 8 lanes of a row leave together
  u32x4v v = {0u, 0u, 0u, 0u};
  if (g < nd) v = *reinterpret_cast<const u32x4v*>(D + (size_t)g * kDim + 16 * piece) ^ 0x80808080u;
  *reinterpret_cast<u32x4v*>(Dp + (size_t)g * kDim + 16 * piece) = v;
  int32_t nrm = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) nrm = __builtin_amdgcn_sdot4((int)v[w], (int)v[w], nrm, false);
  nrm += __shfl_xor(nrm, 1);
  nrm += __shfl_xor(nrm, 2);
  nrm += __shfl_xor(nrm, 4);
  if (piece == 0) bias[g] = g < nd ? -(nrm << kBfShift) + (kBfD - 1 - (g & (kBfD - 1))) : kBfEmpty;
}

typedef __attribute__((address_space(3))) void lds_void;

// Copies tile rows [tile, tile + kBfD) of y' and their biases into LDS, with
// no registers in between: wave w fills rows 32 w .. 32 w + 31, eight rows
// (1 KB) per instruction, lane L writing bytes 16 L.. of its instruction's
// block.  Row r's piece p (16 bytes) sits at slot p ^ ((r >> 1) & 7), so
// lane L of instruction i loads piece (L % 8) ^ ((4 (i % 2) + L / 16) % 8)
// of row 32 w + 8 i + L / 8: lp[i % 2] is that piece's byte offset from the
// instruction's first row.
__device__ __forceinline__ void bf_stage(const uint8_t* Dp, const int32_t* bias, int tile, uint8_t* sd,
                                         int32_t* sb, int wave, const uint32_t (&lp)[2], uint32_t lb) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r0 = 32 * wave + 8 * i;
    const uint8_t* src = Dp + (size_t)(tile + r0) * kDim;  // uniform
    __builtin_amdgcn_global_load_lds(src + lp[i & 1], (lds_void*)(sd + r0 * kDim), 16, 0, 0);
  }
  if (wave == 0)
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint8_t*>(bias + tile) + lb, (lds_void*)sb, 16, 0, 0);
}

__global__ __launch_bounds__(64 * kBfWaves, 4) void k_bf_partial(const uint8_t* Q, int nq, const uint8_t* Dp,
                                                    const int32_t* bias, int nd, int split_cols, int4* work) {
  __shared__ __attribute__((aligned(16))) uint8_t sD0[kBfD * kDim];
  __shared__ __attribute__((aligned(16))) uint8_t sD1[kBfD * kDim];
  __shared__ __attribute__((aligned(16))) int32_t sB0[kBfD];
  __shared__ __attribute__((aligned(16))) int32_t sB1[kBfD];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
  const uint32_t lp[2] = {(uint32_t)(lane >> 3) * kDim + 16u * (uint32_t)((lane & 7) ^ ((lane >> 4) & 7)),
                          (uint32_t)(lane >> 3) * kDim + 16u * (uint32_t)((lane & 7) ^ ((4 + (lane >> 4)) & 7))};
  const uint32_t lb = 16u * (uint32_t)lane;
  // the lane's db row of a 32-row block is 32 blk + lane % 32; its pieces
  // 2 ks + half sit at slots (2 ks + half) ^ sw: byte koff[ks] + 4096 blk
  const uint32_t sw = ((uint32_t)(lane & 31) >> 1) & 7u;
  uint32_t koff[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
    koff[ks] = (uint32_t)(lane & 31) * kDim + 16u * (((uint32_t)(2 * ks + half)) ^ sw);
  const uint32_t boff = 4u * (uint32_t)(lane & 31);
  auto compute = [&](const uint8_t* sd, const int32_t* sb, int tile) {
    int32_t before[E];
#pragma unroll
    for (int e = 0; e < E; ++e) before[e] = s1[e];
#pragma unroll
    for (int blk = 0; blk < kBfD / 32; ++blk) {
      i32x16v acc[kBfRB];
#pragma unroll
      for (int rb = 0; rb < kBfRB; ++rb) acc[rb] = i32x16v{};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const i32x4v B = *reinterpret_cast<const i32x4v*>(sd + koff[ks] + 32 * kDim * blk);
#pragma unroll
        for (int rb = 0; rb < kBfRB; ++rb)
          acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[rb][ks], B, acc[rb], 0, 0, 0);
      }
      const int32_t bs = *reinterpret_cast<const int32_t*>(reinterpret_cast<const uint8_t*>(sb) + boff + 128 * blk);
#pragma unroll
      for (int rb = 0; rb < kBfRB; ++rb) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int32_t key = (acc[rb][e] << (kBfShift + 1)) + bs;  // T (2 x'.y' - ||y'||^2) + T - 1 - c
          s2[16 * rb + e] = med3i(s1[16 * rb + e], s2[16 * rb + e], key);
          s1[16 * rb + e] = max(s1[16 * rb + e], key);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) t1[e] = s1[e] != before[e] ? tile : t1[e];
  };
  // Two buffers: after the barrier that ends tile k - 1, tile k + 1 streams
  // into the buffer tile k - 1 used while tile k is multiplied.
  if (c0 < c1) bf_stage(Dp, bias, c0, sD0, sB0, wave, lp, lb);
  for (int tile = c0; tile < c1;) {
    __builtin_amdgcn_s_waitcnt(0);  // this lane's copies of the tile have landed
    __syncthreads();                // everyone's have, and the other buffer is free
    if (tile + kBfD < c1) bf_stage(Dp, bias, tile + kBfD, sD1, sB1, wave, lp, lb);
    compute(sD0, sB0, tile);
    tile += kBfD;
    if (tile >= c1) break;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tile + kBfD < c1) bf_stage(Dp, bias, tile + kBfD, sD0, sB0, wave, lp, lb);
    compute(sD1, sB1, tile);
    tile += kBfD;
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

// Splits of the db: work-groups run in rounds of kBfSlots (two per CU of a
// 256-CU MI355X), each taking about (its tiles + 1.5) tile times (the 1.5:
// loading the queries and merging the lanes' lists).  The split count
// minimises rounds x (tiles + 1.5), the fewest splits on ties, over counts
// that give at least one full round (or a tile per work-group).
int bruteforce_splits(int nq, int nd) {
  const int qt = (nq + kBfQ - 1) / kBfQ;
  const int dt = (nd + kBfD - 1) / kBfD;
  if (qt <= 0 || dt <= 1) return 1;
  const int lo = std::min(dt, std::max(1, (kBfSlots + qt - 1) / qt));
  const int hi = std::min(dt, 4 * lo);
  int best = lo;
  double best_cost = 0.0;
  for (int s = lo; s <= hi; ++s) {
    const int tiles = (dt + s - 1) / s;  // tiles per work-group
    const long wg = (long)qt * ((dt + tiles - 1) / tiles);
    const double cost = (double)((wg + kBfSlots - 1) / kBfSlots) * (tiles + 1.5);
    if (s == lo || cost < best_cost - 1e-9) {
      best_cost = cost;
      best = s;
    }
  }
  return best;
}

// Workspace: the per-split partial top-2 (16 B per query and split), then
// y' (128 B per db row, rows padded to a whole tile) and the row biases.
static uint64_t bf_part_bytes(int nq, int nd) {
  return ((uint64_t)bruteforce_splits(nq, nd) * (uint64_t)nq * 16u + 255u) & ~255ull;
}
static uint64_t bf_rows_pad(int nd) { return ((uint64_t)nd + kBfD - 1) / kBfD * kBfD; }

uint64_t bruteforce_work_bytes(int nq, int nd) {
  return bf_part_bytes(nq, nd) + bf_rows_pad(nd) * (kDim + 4);
}

hipError_t launch_bruteforce(const uint8_t* q, int nq, const uint8_t* d, int nd, int ra, int rb,
                             int32_t* out, void* work, int splits, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const int dt = (nd + kBfD - 1) / kBfD;
  const int split_cols = ((dt + splits - 1) / splits) * kBfD;
  int4* w = reinterpret_cast<int4*>(work);
  if (nd > 0) {
    const int nd_pad = (int)bf_rows_pad(nd);
    uint8_t* Dp = reinterpret_cast<uint8_t*>(work) + bf_part_bytes(nq, nd);
    int32_t* bias = reinterpret_cast<int32_t*>(Dp + (size_t)nd_pad * kDim);
    hipLaunchKernelGGL(k_bf_prep, dim3((nd_pad * 8 + 255) / 256), dim3(256), 0, s, d, nd, nd_pad, Dp, bias);
    hipLaunchKernelGGL(k_bf_partial, dim3((nq + kBfQ - 1) / kBfQ, splits), dim3(64 * kBfWaves), 0, s, q, nq,
                       Dp, bias, nd, split_cols, w);
  }
  hipLaunchKernelGGL(k_bf_merge, dim3((nq + 255) / 256), dim3(256), 0, s, w, nd > 0 ? splits : 0, q,
                     nq, nd, ra, rb, out);
  return hipGetLastError();
}

}  // namespace chm

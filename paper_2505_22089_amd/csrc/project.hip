// Long codes and bucket ids (Sec. 2.3.1 steps (1)-(2)): the sign of the
// projection p_r(x) = sum_d W[r][d] (x_d - mu_d) = W_r . x - c_r of every
// descriptor onto every random row r, as an MFMA GEMM per 32-descriptor
// tile (c_r = W_r . mu is exact on the host).
//
// Exactness: x_d is an integer in [0, 255] and W is bfloat16, so both MFMA
// input types (bf16 and fp32) hold the operands exactly and every product is
// exact in fp32; only the fp32 accumulation of W_r . x and the subtraction of
// c_r (rounded to fp32) round.  In any summation order the error is below
// 127 * 2^-24 * (||W_r|| ||x|| + |c_r|) (Cauchy-Schwarz), twice that if the
// accumulator truncates, well under the threshold
// tau_r ||x|| + kappa_r = fixup_rel (||W_r|| ||x|| + |c_r|) for
// fixup_rel >= 1e-4.  Projections under the threshold are listed and
// recomputed in fp64 by k_fixup, which is exact for these operands, so every
// bit equals the sign of the exact value (a zero projection gives 0).
//
// k_project: one work-group of kProjWaves wavefronts shares W in LDS; each
// wavefront loops over 32-descriptor tiles.  A lane's share of the tile is
// converted to MFMA operands once (byte -> float conversions); the 192
// (padded) rows are done in two passes of three 32x32 output blocks.  Codes
// and bucket ids are written from the signs; each wavefront writes the
// borderline (descriptor, row) entries of its tiles into its own region of
// the global fix-up list, without atomics.
// k_fixup: wavefronts walk the regions; each lane recomputes one entry
// exactly in fp64 and patches its bit with a 32-bit atomic.  If a region
// overflowed (adversarial inputs only: the overflow word then holds the
// batch's number), it instead rebuilds every code and bucket id of the
// batch from exact values.
#include "chm_internal.h"

namespace chm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const u32x2 gcu32x2;
typedef __attribute__((address_space(1))) const u32x4 gcu32x4;

#ifndef CHM_PROJ_WAVES
#define CHM_PROJ_WAVES 8
#endif
#ifndef CHM_PROJ_GRID_PER_CU
#define CHM_PROJ_GRID_PER_CU 2
#endif
constexpr int kProjWaves = CHM_PROJ_WAVES;
constexpr int kProjWG = 64 * kProjWaves;

__device__ __forceinline__ uint32_t bf16_bits_of_int(int v) {
  // |v| <= 255 has at most 8 significant bits: the bf16 pattern is the upper
  // half of the fp32 pattern, exactly.
  return __float_as_uint((float)v) >> 16;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// bf16 patterns of bytes 2i and 2i+1 of w (integers 0..255 are exact in
// bf16: the upper half of their fp32 pattern), packed low | high.
__device__ __forceinline__ uint32_t bf16x2_of_bytes(uint32_t w, int i) {
  const float lo = (float)((w >> (16 * i)) & 0xFFu);
  const float hi = (float)((w >> (16 * i + 8)) & 0xFFu);
  return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xFFFF0000u);
}

template <bool FP32>
// waves per SIMD the bf16 variant is compiled for (VGPR budget 512 / this)
#ifndef CHM_PROJ_WAVES_PER_SIMD
#define CHM_PROJ_WAVES_PER_SIMD 4
#endif
__global__ __launch_bounds__(kProjWG, FP32 ? 2 : CHM_PROJ_WAVES_PER_SIMD) void k_project(HashBatch hb,
                                                                                     ProjConsts pc) {
  __shared__ uint16_t sW[kRowsPad * kWStride];
  __shared__ uint32_t sWords[kProjWaves][32 * 6];
  __shared__ float sRow[3][kRowsPad];     // tau_r, kappa_r, c_r (fp32)
  __shared__ float sSx[kProjWaves][32];   // ||x|| (rounded up) of the wave's tile rows

  const int tid = threadIdx.x;
  for (int c = tid; c < kRowsPad * (kDim / 8); c += kProjWG) {
    const int r = c / (kDim / 8), k8 = c % (kDim / 8);
    const uint4 v = *reinterpret_cast<const uint4*>(pc.W + r * kDim + k8 * 8);
    uint32_t* dst = reinterpret_cast<uint32_t*>(sW + r * kWStride + k8 * 8);
    dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
  }
  for (int i = tid; i < 3 * kRowsPad; i += kProjWG) (&sRow[0][0])[i] = pc.tau[i];
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps tile / image in SGPRs
  const int lane = __lane_id();
  const int half = lane >> 5;
  const int col = lane & 31;
  uint32_t* words = sWords[wave];
  // Lane L < 32 collects the words of descriptor L: it is accumulator element
  // e = 4*(L/8) + L%4, in the upper ballot half iff (L/4) is odd.
  const int eL = 4 * ((lane >> 3) & 3) + (lane & 3);
  const bool hiL = (lane >> 2) & 1;

  // this wavefront's region of the fix-up list: [gw * cap_w, (gw + 1) * cap_w)
  const uint32_t gw = blockIdx.x * kProjWaves + wave;
  const uint32_t cap_w = pc.fix_cap / pc.n_waves;
  uint32_t* region = pc.fixlist + 1 + pc.n_waves + (size_t)gw * cap_w;
  uint32_t wcount = 0;

  const int total_tiles = hb.tile_prefix[hb.count];
  int im = 0;  // tiles of a wavefront increase, so the image search resumes
  for (int tile = blockIdx.x * kProjWaves + wave; tile < total_tiles;
       tile += gridDim.x * kProjWaves) {
    while (tile >= hb.tile_prefix[im + 1]) ++im;
    const HashImage I = hash_image(hb, im);
    const int d0 = (tile - hb.tile_prefix[im]) * 32;
    const int dr = d0 + col;
    const bool valid = dr < I.n;
    const uint8_t* xrow = I.desc + (size_t)(valid ? dr : d0) * kDim;

    // The lane's bytes of its descriptor (bf16: k = 16*kb + 8*half .. +7;
    // fp32: the whole row); invalid rows read as zero.  ||x||^2 with dot4.
    uint32_t nx = 0;
    u32x4 abf[8];   // bf16 operands, converted once per tile
    u32x4 rawf[8];
    if (!FP32) {
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const u32x2 w = valid ? *(gcu32x2*)(xrow + 16 * kb + 8 * half) : u32x2{0u, 0u};
        nx = __builtin_amdgcn_udot4(w[0], w[0], nx, false);
        nx = __builtin_amdgcn_udot4(w[1], w[1], nx, false);
        abf[kb] = u32x4{bf16x2_of_bytes(w[0], 0), bf16x2_of_bytes(w[0], 1), bf16x2_of_bytes(w[1], 0),
                        bf16x2_of_bytes(w[1], 1)};
      }
      nx += __shfl_xor(nx, 32);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        rawf[q] = valid ? *(gcu32x4*)(xrow + 16 * q) : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 4; ++j) nx = __builtin_amdgcn_udot4(rawf[q][j], rawf[q][j], nx, false);
      }
    }
    if (lane < 32) sSx[wave][lane] = valid ? sqrtf((float)nx) * 1.000001f : 0.f;
    wave_sync();

    // per lane, borderline accumulator elements: bit 16*(blk&1) + e of bm3[blk>>1]
    uint32_t bm3[3] = {0u, 0u, 0u};
    // elements whose descriptor (8*(e/4) + 4*half + e%4 of the tile) exists
    uint32_t vm = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) vm |= (d0 + 8 * (e >> 2) + 4 * half + (e & 3) < I.n) ? (1u << e) : 0u;
    vm |= vm << 16;
    // One 32x32 block of rows at a time: a single accumulator keeps the
    // register count low enough for four wavefronts per SIMD.
#pragma unroll 1
    for (int blk = 0; blk < 6; ++blk) {
      f32x16 acc;
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] = 0.f;
      const int row = 32 * blk + col;
      if (!FP32) {
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
          const int k0 = 16 * kb + 8 * half;
          const u32x4 bw = *reinterpret_cast<const u32x4*>(sW + row * kWStride + k0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, abf[kb]),
                                                        __builtin_bit_cast(bf16x8, bw), acc, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < 64; ++kk) {
          const int k = 2 * kk + half;
          const float Af = (float)((rawf[kk >> 3][(kk >> 1) & 3] >> (8 * (k & 3))) & 0xFFu);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(Af, bf16_to_f32(sW[row * kWStride + k]), acc, 0, 0, 0);
        }
      }
      const float tau = sRow[0][row], kap = sRow[1][row], cr = sRow[2][row];
      uint32_t word = 0, m = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // descriptors 8q + 4*half + 0..3 of the tile
        const float4 sx4 = *reinterpret_cast<const float4*>(&sSx[wave][8 * q + 4 * half]);
        const float sx[4] = {sx4.x, sx4.y, sx4.z, sx4.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = 4 * q + i;
          const float v = acc[e] - cr;
          const uint64_t bits = __ballot(v > 0.f);
          if (e == eL) word = hiL ? (uint32_t)(bits >> 32) : (uint32_t)bits;
          m |= (fabsf(v) < fmaf(tau, sx[i], kap)) ? (1u << e) : 0u;
        }
      }
      if (lane < 32) words[lane * 6 + blk] = word;
      m <<= 16 * (blk & 1);
      if (blk < 2) bm3[0] |= m;
      else if (blk < 4) bm3[1] |= m;
      else bm3[2] |= m;
    }
    // Borderline entries of the tile go straight to this wavefront's region of
    // the global list (no atomics): lane offsets from a wave prefix sum.
    {
      bm3[0] &= vm;
      bm3[1] &= vm;
      bm3[2] &= vm;
      const int mine = __popc(bm3[0]) + __popc(bm3[1]) + __popc(bm3[2]);
      int incl = mine;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
      }
      const uint32_t tile_n = __builtin_amdgcn_readfirstlane(__shfl(incl, 63));
      uint32_t idx = wcount + (uint32_t)(incl - mine);
#pragma unroll
      for (int w3 = 0; w3 < 3; ++w3) {
        uint32_t m = bm3[w3];
        while (m) {
          const int bit = __builtin_ctz(m);
          m &= m - 1u;
          const int blk = 2 * w3 + (bit >> 4), e = bit & 15;
          const int drel = 8 * (e >> 2) + 4 * half + (e & 3);
          if (idx < cap_w)
            region[idx] = ((uint32_t)im << 24) | ((uint32_t)(32 * blk + col) << 16) | (uint32_t)(d0 + drel);
          ++idx;
        }
      }
      wcount += tile_n;
    }
    wave_sync();
    if (lane < 32 && valid) {
      const uint32_t* w = words + lane * 6;
      I.codes[dr] = make_uint4(w[0], w[1], w[2], w[3]);
      const uint64_t bb = (uint64_t)w[4] | ((uint64_t)w[5] << 32);
      const uint32_t mask = (1u << hb.m) - 1u;
      for (int t = 0; t < hb.L; ++t)
        I.ids[(size_t)t * I.n_pad + dr] = (uint8_t)((uint32_t)(bb >> (hb.m * t)) & mask);
      I.norms[dr] = nx;
    }
    wave_sync();
  }
  if (lane == 0) {
    pc.fixlist[1 + gw] = wcount;
    if (wcount > cap_w) atomicExch(pc.fixlist, hb.seq);
  }
}

// Exact projection p_r(x): sum_k W[r][k] x_k is exact in fp64 (products of
// 8-bit significands, partial sums multiples of 2^-23 below 2^21), so is
// c_r = W_r . mu; four independent partial sums keep each exact.
__device__ __forceinline__ double exact_projection(const uint8_t* xr, const uint16_t* Wr, double c) {
  double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll 2
  for (int k16 = 0; k16 < kDim / 16; ++k16) {
    const u32x4 xv = *(gcu32x4*)(xr + 16 * k16);
    const u32x4 w0 = *(gcu32x4*)(Wr + 16 * k16);
    const u32x4 w1 = *(gcu32x4*)(Wr + 16 * k16 + 8);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t x4 = xv[q];
      const uint32_t wa = q < 2 ? w0[2 * q] : w1[2 * (q - 2)];
      const uint32_t wb = q < 2 ? w0[2 * q + 1] : w1[2 * (q - 2) + 1];
      p0 = fma((double)__uint_as_float(wa << 16), (double)(x4 & 0xFF), p0);
      p1 = fma((double)__uint_as_float(wa & 0xFFFF0000u), (double)((x4 >> 8) & 0xFF), p1);
      p2 = fma((double)__uint_as_float(wb << 16), (double)((x4 >> 16) & 0xFF), p2);
      p3 = fma((double)__uint_as_float(wb & 0xFFFF0000u), (double)(x4 >> 24), p3);
    }
  }
  return ((p0 + p1) + (p2 + p3)) - c;
}

// Sets or clears one bit; true when that changed it.
__device__ __forceinline__ bool set_bit(uint32_t* word, uint32_t bit, bool on) {
  const uint32_t old = on ? atomicOr(word, bit) : atomicAnd(word, ~bit);
  return ((old & bit) != 0) != on;
}

// Exact projection with W read from LDS (row-major bf16, kDim per row) and
// the descriptor row loaded up front.
__device__ __forceinline__ double exact_projection_lds(const uint8_t* xr, const uint16_t* sWr, double c) {
  u32x4 xv[8];
#pragma unroll
  for (int k16 = 0; k16 < kDim / 16; ++k16) xv[k16] = *(gcu32x4*)(xr + 16 * k16);
  double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
  for (int k16 = 0; k16 < kDim / 16; ++k16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint2 wv = *reinterpret_cast<const uint2*>(sWr + 16 * k16 + 4 * q);
      const uint32_t x4 = xv[k16][q];
      p0 = fma((double)__uint_as_float(wv.x << 16), (double)(x4 & 0xFF), p0);
      p1 = fma((double)__uint_as_float(wv.x & 0xFFFF0000u), (double)((x4 >> 8) & 0xFF), p1);
      p2 = fma((double)__uint_as_float(wv.y << 16), (double)((x4 >> 16) & 0xFF), p2);
      p3 = fma((double)__uint_as_float(wv.y & 0xFFFF0000u), (double)(x4 >> 24), p3);
    }
  }
  return ((p0 + p1) + (p2 + p3)) - c;
}

constexpr int kFixWG = 512;

// Without an overflow of the batch's fix-up list: wavefronts walk the
// regions, each lane recomputes one listed projection exactly and patches
// its bit.  After an overflow (adversarial inputs only) every work-group
// instead rebuilds its share of the codes and bucket ids of the batch from
// exact values.  Either way each work-group adds its counts (projections
// recomputed, bits they changed) to the store's counters with one atomic
// per counter.
__global__ __launch_bounds__(kFixWG) void k_fixup(HashBatch hb, ProjConsts pc) {
  __shared__ uint16_t sW[kRowsPad * kWStride];
  __shared__ unsigned long long s_sum[2];
  if (threadIdx.x < 2) s_sum[threadIdx.x] = 0;
  unsigned long long n_fix = 0, n_flip = 0;
  const int lane = __lane_id();
  if (pc.fixlist[0] == hb.seq) {
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int gsize = gridDim.x * blockDim.x;
    const int total = hb.tile_prefix[hb.count] * 32;
    for (int g = gtid; g < total; g += gsize) {
      int im = 0;
      while (g >= hb.tile_prefix[im + 1] * 32) ++im;
      const HashImage I = hash_image(hb, im);
      const int d = g - hb.tile_prefix[im] * 32;
      if (d >= I.n) continue;
      uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
#pragma unroll 1
      for (int r = 0; r < pc.R; ++r) {
        const double p = exact_projection(I.desc + (size_t)d * kDim, pc.W + r * kDim, pc.cmu[r]);
        const uint32_t bit = p > 0.0 ? 1u << (r & 31) : 0u;
        const int slot = r < 128 ? (r >> 5) : 4 + ((r - 128) >> 5);
        w0 |= slot == 0 ? bit : 0u; w1 |= slot == 1 ? bit : 0u; w2 |= slot == 2 ? bit : 0u;
        w3 |= slot == 3 ? bit : 0u; w4 |= slot == 4 ? bit : 0u; w5 |= slot == 5 ? bit : 0u;
      }
      const uint4 old = I.codes[d];
      uint32_t flips = __popc(old.x ^ w0) + __popc(old.y ^ w1) + __popc(old.z ^ w2) + __popc(old.w ^ w3);
      I.codes[d] = make_uint4(w0, w1, w2, w3);
      const uint64_t bb = (uint64_t)w4 | ((uint64_t)w5 << 32);
      const uint32_t mask = (1u << hb.m) - 1u;
      for (int t = 0; t < hb.L; ++t) {
        const uint8_t nb = (uint8_t)((uint32_t)(bb >> (hb.m * t)) & mask);
        flips += __popc((uint32_t)(I.ids[(size_t)t * I.n_pad + d] ^ nb));
        I.ids[(size_t)t * I.n_pad + d] = nb;
      }
      n_fix += (unsigned long long)pc.R;
      n_flip += flips;
    }
  } else {
    for (int c = threadIdx.x; c < kRowsPad * kDim / 8; c += kFixWG) {
      const int r = c / (kDim / 8), k8 = c % (kDim / 8);
      *reinterpret_cast<uint4*>(sW + r * kWStride + 8 * k8) = reinterpret_cast<const uint4*>(pc.W)[c];
    }
    __syncthreads();
    const uint32_t cap_w = pc.fix_cap / pc.n_waves;
    const uint32_t* counts = pc.fixlist + 1;
    const uint32_t* entries = pc.fixlist + 1 + pc.n_waves;
    // a wavefront takes whole regions; its lanes stride inside one
    const int wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kFixWG / 64) + (threadIdx.x >> 6)));
    const int nw = gridDim.x * (kFixWG / 64);
    for (int r = wid; r < pc.n_waves; r += nw) {
      const uint32_t count = counts[r];
      if (lane == 0) n_fix += count;
      for (uint32_t k = lane; k < count; k += 64) {
        const uint32_t ent = entries[(size_t)r * cap_w + k];
        const int im = ent >> 24, row = (ent >> 16) & 0xFF, d = ent & 0xFFFF;
        const HashImage I = hash_image(hb, im);
        const double p = exact_projection_lds(I.desc + (size_t)d * kDim, sW + row * kWStride, pc.cmu[row]);
        bool changed;
        if (row < 128) {
          changed = set_bit(reinterpret_cast<uint32_t*>(I.codes + d) + (row >> 5), 1u << (row & 31), p > 0.0);
        } else {
          const int t = (row - 128) / hb.m, j = (row - 128) % hb.m;
          const size_t byte = (size_t)t * I.n_pad + d;
          uint32_t* w = reinterpret_cast<uint32_t*>(I.ids + (byte & ~(size_t)3));
          changed = set_bit(w, 1u << (8 * (byte & 3) + j), p > 0.0);
        }
        if (changed) ++n_flip;
      }
    }
  }
  __syncthreads();  // s_sum is cleared
  if (n_fix) atomicAdd(&s_sum[0], n_fix);
  if (n_flip) atomicAdd(&s_sum[1], n_flip);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_sum[0]) atomicAdd(pc.fixups, s_sum[0]);
    if (s_sum[1]) atomicAdd(pc.fixups + 1, s_sum[1]);
  }
}

hipError_t launch_project(const HashBatch& hb, const ProjConsts& pc, int fp32, int n_cu,
                          hipStream_t s) {
  const int tiles = hb.tile_prefix[hb.count];
  if (tiles == 0) return hipSuccess;
  int grid = (tiles + kProjWaves - 1) / kProjWaves;
  if (grid > CHM_PROJ_GRID_PER_CU * n_cu) grid = CHM_PROJ_GRID_PER_CU * n_cu;
  if (grid * kProjWaves > kMaxProjWaves) grid = kMaxProjWaves / kProjWaves;
  ProjConsts p2 = pc;
  p2.n_waves = grid * kProjWaves;
  if (fp32)
    hipLaunchKernelGGL(k_project<true>, dim3(grid), dim3(kProjWG), 0, s, hb, p2);
  else
    hipLaunchKernelGGL(k_project<false>, dim3(grid), dim3(kProjWG), 0, s, hb, p2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fixup, dim3(2 * n_cu), dim3(kFixWG), 0, s, hb, p2);
  return hipGetLastError();
}

}  // namespace chm

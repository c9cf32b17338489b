// Long codes and bucket ids (Sec. 2.3.1 steps (1)-(2)): the sign of the
// projection p_r(x) = sum_d W[r][d] (x_d - mu_d) of every descriptor onto
// every random row r, as an MFMA GEMM per 32-descriptor tile.
//
// Exactness: x_d - mu_d is an integer in [-255, 255] and W is bfloat16, so
// both MFMA input types (bf16 and fp32) hold the operands exactly and every
// product is exact in fp32; only the fp32 accumulation rounds.  Its error is
// below ~128 * 2^-24 * ||W_r|| ||x - mu|| (Cauchy-Schwarz), far below the
// threshold tau_r * ||x - mu|| with tau_r = fixup_rel * ||W_r|| (1e-3 by
// default).  Projections under the threshold are listed and recomputed in
// fp64 by k_fixup, which is exact for these operands, so every bit equals the
// sign of the exact value.
//
// k_project: one work-group of kProjWaves wavefronts shares W in LDS; each
// wavefront loops over 32-descriptor tiles.  The 192 (padded) rows are done
// in two passes of three 32x32 output blocks.  Codes and bucket ids are
// written from the fp32 signs; borderline (descriptor, row) entries go to a
// per-wave LDS list and, once per tile, to the global fix-up list.
// k_fixup: a persistent grid over the list; each lane recomputes one entry
// exactly and patches its bit with a 32-bit atomic.  If any list overflowed
// (adversarial inputs only), it recomputes every projection of the batch.
#include "chm_internal.h"

namespace chm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const u32x2 gcu32x2;
typedef __attribute__((address_space(1))) const u32x4 gcu32x4;

constexpr int kProjWaves = 8;
constexpr int kProjWG = 64 * kProjWaves;
constexpr int kTileFixCap = 1024;  // per-wave LDS list for one tile

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

template <bool FP32>
__global__ __launch_bounds__(kProjWG) void k_project(HashBatch hb, ProjConsts pc) {
  __shared__ uint16_t sW[kRowsPad * kWStride];
  __shared__ uint32_t sFix[kProjWaves][kTileFixCap];
  __shared__ uint32_t sWords[kProjWaves][32 * 6];
  __shared__ float sTau[kRowsPad];
  __shared__ float sSd[kProjWaves][32];   // ||x - mu|| of the wave's tile rows
  __shared__ uint8_t sMu[kDim];

  const int tid = threadIdx.x;
  for (int c = tid; c < kRowsPad * (kDim / 8); c += kProjWG) {
    const int r = c / (kDim / 8), k8 = c % (kDim / 8);
    const uint4 v = *reinterpret_cast<const uint4*>(pc.W + r * kDim + k8 * 8);
    uint32_t* dst = reinterpret_cast<uint32_t*>(sW + r * kWStride + k8 * 8);
    dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
  }
  if (tid < kDim) sMu[tid] = pc.mu[tid];
  if (tid < kRowsPad) sTau[tid] = pc.tau[tid];
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps tile / image in SGPRs
  const int lane = __lane_id();
  const int half = lane >> 5;
  const int col = lane & 31;
  uint32_t* fix = sFix[wave];
  uint32_t* words = sWords[wave];
  // Lane L < 32 collects the words of descriptor L: it is accumulator element
  // e = 4*(L/8) + L%4, in the upper ballot half iff (L/4) is odd.
  const int eL = 4 * ((lane >> 3) & 3) + (lane & 3);
  const bool hiL = (lane >> 2) & 1;

  const int total_tiles = hb.tile_prefix[hb.count];
  int im = 0;  // tiles of a wavefront increase, so the image search resumes
  for (int tile = blockIdx.x * kProjWaves + wave; tile < total_tiles;
       tile += gridDim.x * kProjWaves) {
    while (tile >= hb.tile_prefix[im + 1]) ++im;
    const HashImage& I = hb.img[im];
    const int d0 = (tile - hb.tile_prefix[im]) * 32;
    const int dr = d0 + col;
    const bool valid = dr < I.n;
    const uint8_t* xrow = I.desc + (size_t)(valid ? dr : d0) * kDim;

    // Raw bytes of the lane's descriptor (bf16: k = 16*kb + 8*half .. +7;
    // fp32: the whole row), converted to MFMA operands in each pass.
    uint32_t nx = 0, nc = 0;
    u32x2 rawb[8];
    u32x4 rawf[8];
    if (!FP32) {
#pragma unroll
      for (int kb = 0; kb < 8; ++kb)
        rawb[kb] = valid ? *(gcu32x2*)(xrow + 16 * kb + 8 * half) : u32x2{0u, 0u};
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const int k0 = 16 * kb + 8 * half;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int x = (rawb[kb][q >> 2] >> (8 * (q & 3))) & 0xFF;
          const int c = valid ? x - (int)sMu[k0 + q] : 0;
          nx += (uint32_t)(x * x);
          nc += (uint32_t)(c * c);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) rawf[q] = valid ? *(gcu32x4*)(xrow + 16 * q) : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
      for (int kk = 0; kk < 64; ++kk) {
        const int k = 2 * kk + half;
        const int x = (rawf[kk >> 3][(kk >> 1) & 3] >> (8 * (k & 3))) & 0xFF;
        const int c = valid ? x - (int)sMu[k] : 0;
        nx += (uint32_t)(x * x);
        nc += (uint32_t)(c * c);
      }
    }
    nx += __shfl_xor(nx, 32);
    nc += __shfl_xor(nc, 32);
    if (lane < 32) sSd[wave][lane] = valid ? sqrtf((float)nc) * 1.000001f : 0.f;
    wave_sync();

    int nfix = 0;
    float4 sd4;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      f32x16 acc[3];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[b][e] = 0.f;
      if (!FP32) {
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
          const int k0 = 16 * kb + 8 * half;
          const uint2 mu8 = *reinterpret_cast<const uint2*>(sMu + k0);
          u32x4 a;
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const uint32_t w = rawb[kb][p >> 1];
            const uint32_t m = p < 2 ? mu8.x : mu8.y;
            const int s0 = (p & 1) * 16;
            const int c0 = valid ? (int)((w >> s0) & 0xFF) - (int)((m >> s0) & 0xFF) : 0;
            const int c1 = valid ? (int)((w >> (s0 + 8)) & 0xFF) - (int)((m >> (s0 + 8)) & 0xFF) : 0;
            a[p] = bf16_bits_of_int(c0) | (bf16_bits_of_int(c1) << 16);
          }
          const bf16x8 Ab = __builtin_bit_cast(bf16x8, a);
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const int row = 32 * (3 * pass + b) + col;
            const u32x4 bw = *reinterpret_cast<const u32x4*>(sW + row * kWStride + k0);
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ab, __builtin_bit_cast(bf16x8, bw),
                                                            acc[b], 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < 64; ++kk) {
          const int k = 2 * kk + half;
          const int x = (rawf[kk >> 3][(kk >> 1) & 3] >> (8 * (k & 3))) & 0xFF;
          const float Af = valid ? (float)(x - (int)sMu[k]) : 0.f;
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const int row = 32 * (3 * pass + b) + col;
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(Af, bf16_to_f32(sW[row * kWStride + k]),
                                                         acc[b], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int blk = 3 * pass + b;
        const float tau = sTau[32 * blk + col];
        uint32_t word = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          if ((e & 3) == 0) sd4 = *reinterpret_cast<const float4*>(&sSd[wave][8 * (e >> 2) + 4 * half]);
          const float sde = (e & 3) == 0 ? sd4.x : (e & 3) == 1 ? sd4.y : (e & 3) == 2 ? sd4.z : sd4.w;
          const float v = acc[b][e];
          const uint64_t bits = __ballot(v > 0.f);
          if (e == eL) word = hiL ? (uint32_t)(bits >> 32) : (uint32_t)bits;
          const bool border = fabsf(v) < tau * sde;
          const uint64_t bm = __ballot(border);
          if (bm) {
            if (border) {
              const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                  (uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
              const uint32_t idx = (uint32_t)nfix + below;
              const int drel = 8 * (e >> 2) + 4 * half + (e & 3);
              if (idx < kTileFixCap)
                fix[idx] = ((uint32_t)im << 24) | ((uint32_t)(32 * blk + col) << 16) | (uint32_t)(d0 + drel);
            }
            nfix += __popcll(bm);
          }
        }
        if (lane < 32) words[lane * 6 + blk] = word;
      }
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
    if (nfix > 0) {
      // hand the tile's entries to the global list (one atomic per tile)
      uint32_t base = 0;
      if (lane == 0) {
        if (nfix > kTileFixCap) {
          atomicOr(pc.fixlist + 1, 1u);
        } else {
          base = atomicAdd(pc.fixlist, (uint32_t)nfix);
          if (base + (uint32_t)nfix > pc.fix_cap) atomicOr(pc.fixlist + 1, 1u);
        }
      }
      base = __shfl(base, 0);
      if (nfix <= kTileFixCap)
        for (int i = lane; i < nfix; i += 64)
          if (base + (uint32_t)i < pc.fix_cap) pc.fixlist[2 + base + i] = fix[i];
    }
    wave_sync();
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

__device__ __forceinline__ void set_bit(uint32_t* word, uint32_t bit, bool on) {
  if (on) atomicOr(word, bit);
  else atomicAnd(word, ~bit);
}

__global__ __launch_bounds__(256) void k_fixup(HashBatch hb, ProjConsts pc) {
  if (pc.fixlist[1] != 0) return;  // overflow: k_fixup_all rebuilds the batch
  const uint32_t count = pc.fixlist[0];
  const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gsize = gridDim.x * blockDim.x;
  for (uint32_t i = gtid; i < count; i += gsize) {
    const uint32_t ent = pc.fixlist[2 + i];
    const int im = ent >> 24, r = (ent >> 16) & 0xFF, d = ent & 0xFFFF;
    const HashImage& I = hb.img[im];
    const double p = exact_projection(I.desc + (size_t)d * kDim, pc.W + r * kDim, pc.cmu[r]);
    if (r < 128) {
      set_bit(reinterpret_cast<uint32_t*>(I.codes + d) + (r >> 5), 1u << (r & 31), p > 0.0);
    } else {
      const int t = (r - 128) / hb.m, j = (r - 128) % hb.m;
      const size_t byte = (size_t)t * I.n_pad + d;
      uint32_t* w = reinterpret_cast<uint32_t*>(I.ids + (byte & ~(size_t)3));
      set_bit(w, 1u << (8 * (byte & 3) + j), p > 0.0);
    }
  }
  if (gtid == 0) atomicAdd(pc.fixups, (unsigned long long)count);
}

// After an overflow of the fix-up list: rebuild every code and bucket id of
// the batch from exact values (adversarial inputs only).
__global__ __launch_bounds__(256) void k_fixup_all(HashBatch hb, ProjConsts pc) {
  if (pc.fixlist[1] == 0) return;
  const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gsize = gridDim.x * blockDim.x;
  const int total = hb.tile_prefix[hb.count] * 32;
  for (int g = gtid; g < total; g += gsize) {
    int im = 0;
    while (g >= hb.tile_prefix[im + 1] * 32) ++im;
    const HashImage& I = hb.img[im];
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
    I.codes[d] = make_uint4(w0, w1, w2, w3);
    const uint64_t bb = (uint64_t)w4 | ((uint64_t)w5 << 32);
    const uint32_t mask = (1u << hb.m) - 1u;
    for (int t = 0; t < hb.L; ++t)
      I.ids[(size_t)t * I.n_pad + d] = (uint8_t)((uint32_t)(bb >> (hb.m * t)) & mask);
  }
  if (gtid == 0) atomicAdd(pc.fixups, (unsigned long long)total * pc.R);
}

hipError_t launch_project(const HashBatch& hb, const ProjConsts& pc, int fp32, int n_cu,
                          hipStream_t s) {
  const int tiles = hb.tile_prefix[hb.count];
  if (tiles == 0) return hipSuccess;
  hipError_t e = launch_fill_u32(pc.fixlist, 0u, 2, s);
  if (e != hipSuccess) return e;
  int grid = (tiles + kProjWaves - 1) / kProjWaves;
  if (grid > 2 * n_cu) grid = 2 * n_cu;
  if (fp32)
    hipLaunchKernelGGL(k_project<true>, dim3(grid), dim3(kProjWG), 0, s, hb, pc);
  else
    hipLaunchKernelGGL(k_project<false>, dim3(grid), dim3(kProjWG), 0, s, hb, pc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fixup, dim3(4 * n_cu), dim3(256), 0, s, hb, pc);
  hipLaunchKernelGGL(k_fixup_all, dim3(4 * n_cu), dim3(256), 0, s, hb, pc);
  return hipGetLastError();
}

}  // namespace chm

// Long codes and bucket ids (Sec. 2.3.1 steps (1)-(2)): the sign of the
// projection p_r(x) = sum_d W[r][d] (x_d - mu_d) of every descriptor onto
// every random row r, as one MFMA GEMM per 32-descriptor tile.
//
// Exactness: x_d - mu_d is an integer in [-255, 255] and W is bfloat16, so
// both MFMA input types (bf16 and fp32) hold the operands exactly and every
// product is exact in fp32; only the fp32 accumulation rounds.  Its error is
// below ~128 * 2^-24 * ||W_r|| ||x - mu|| (Cauchy-Schwarz), far below the
// threshold tau_r * ||x - mu|| with tau_r = fixup_rel * ||W_r|| (1e-3 by
// default).  Projections under the threshold are recomputed in fp64, which is
// exact for these operands, so every bit equals the sign of the exact value.
#include "chm_internal.h"

namespace chm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kFixCap = 1280;   // per-wave list of borderline (descriptor, row)
constexpr int kProjWaves = 4;

__device__ __forceinline__ uint32_t bf16_bits_of_int(int v) {
  // |v| <= 255 has at most 8 significant bits: the bf16 pattern is the upper
  // half of the fp32 pattern, exactly.
  return __float_as_uint((float)v) >> 16;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

template <bool FP32>
__global__ __launch_bounds__(256) void k_project(HashBatch hb, ProjConsts pc) {
  __shared__ uint16_t sW[kRowsPad * kWStride];
  __shared__ uint32_t sFix[kProjWaves][kFixCap];
  __shared__ uint32_t sWords[kProjWaves][32][6];
  __shared__ uint8_t sMu[kDim];

  const int tid = threadIdx.x;
  // Stage W (kRowsPad x 128 bf16) with padded rows.
  for (int c = tid; c < kRowsPad * (kDim / 8); c += blockDim.x) {
    const int r = c / (kDim / 8), k8 = c % (kDim / 8);
    const uint4 v = *reinterpret_cast<const uint4*>(pc.W + r * kDim + k8 * 8);
    uint32_t* dst = reinterpret_cast<uint32_t*>(sW + r * kWStride + k8 * 8);
    dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
  }
  if (tid < kDim) sMu[tid] = pc.mu[tid];
  __syncthreads();

  const int wave = tid >> 6;
  const int lane = lane_id();
  const int half = lane >> 5;
  const int col = lane & 31;

  float tau[6];
#pragma unroll
  for (int b = 0; b < 6; ++b) tau[b] = pc.tau[32 * b + col];

  const int total_tiles = hb.tile_prefix[hb.count];
  for (int tile = blockIdx.x * kProjWaves + wave; tile < total_tiles;
       tile += gridDim.x * kProjWaves) {
    int im = 0;
    while (tile >= hb.tile_prefix[im + 1]) ++im;
    const HashImage& I = hb.img[im];
    const int d0 = (tile - hb.tile_prefix[im]) * 32;
    const int dr = d0 + col;
    const bool valid = dr < I.n;
    const uint8_t* xrow = I.desc + (size_t)(valid ? dr : 0) * kDim;

    // Norms: ||x||^2 for the re-rank and ||x - mu||^2 for the fix-up threshold.
    uint32_t nx = 0, nc = 0;
    f32x16 acc[6];
#pragma unroll
    for (int b = 0; b < 6; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[b][e] = 0.f;

    if (!FP32) {
      // A operand of the 32x32x16 bf16 MFMA: lane holds row (lane % 32),
      // k = 16*kb + 8*half .. +7.
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const int k0 = 16 * kb + 8 * half;
        uint2 raw = valid ? *reinterpret_cast<const uint2*>(xrow + k0) : make_uint2(0, 0);
        u32x4 a;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const uint32_t w = p < 2 ? raw.x : raw.y;
          const int s0 = (p & 1) * 16;
          const int x0 = (w >> s0) & 0xFF, x1 = (w >> (s0 + 8)) & 0xFF;
          const int c0 = valid ? x0 - (int)sMu[k0 + 2 * p] : 0;
          const int c1 = valid ? x1 - (int)sMu[k0 + 2 * p + 1] : 0;
          nx += (uint32_t)(x0 * x0 + x1 * x1);
          nc += (uint32_t)(c0 * c0 + c1 * c1);
          a[p] = bf16_bits_of_int(c0) | (bf16_bits_of_int(c1) << 16);
        }
        const bf16x8 av = __builtin_bit_cast(bf16x8, a);
#pragma unroll
        for (int b = 0; b < 6; ++b) {
          const u32x4 bw = *reinterpret_cast<const u32x4*>(sW + (32 * b + col) * kWStride + k0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, bw),
                                                          acc[b], 0, 0, 0);
        }
      }
    } else {
      // A operand of the 32x32x2 fp32 MFMA: lane holds row (lane % 32), k = 2*kk + half.
      uint32_t xw[32];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        uint4 v = valid ? *reinterpret_cast<const uint4*>(xrow + 16 * q) : make_uint4(0, 0, 0, 0);
        xw[4 * q] = v.x; xw[4 * q + 1] = v.y; xw[4 * q + 2] = v.z; xw[4 * q + 3] = v.w;
      }
#pragma unroll
      for (int kk = 0; kk < 64; ++kk) {
        const int k = 2 * kk + half;
        const int x = (xw[k >> 2] >> (8 * (k & 3))) & 0xFF;
        const int c = valid ? x - (int)sMu[k] : 0;
        nx += (uint32_t)(x * x);
        nc += (uint32_t)(c * c);
        const float af = (float)c;
#pragma unroll
        for (int b = 0; b < 6; ++b) {
          const float bf = bf16_to_f32(sW[(32 * b + col) * kWStride + k]);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af, bf, acc[b], 0, 0, 0);
        }
      }
    }
    nx += __shfl_xor(nx, 32);
    nc += __shfl_xor(nc, 32);
    // ||x - mu|| of the descriptors this lane's accumulators belong to:
    // acc element e is descriptor 8*(e/4) + 4*half + e%4, row 32*b + col.
    const float sdesc = valid ? sqrtf((float)nc) * 1.000001f : 0.f;
    float sd[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) sd[e] = __shfl(sdesc, 8 * (e >> 2) + 4 * half + (e & 3));

    int nfix = 0;
    uint32_t* fix = sFix[wave];
    // Lane L < 32 collects the words of descriptor L: it is element
    // e = 4*(L/8) + L%4 of the accumulators, in the upper half iff (L/4) is odd.
    const int eL = 4 * ((lane >> 3) & 3) + (lane & 3);
    const bool hiL = (lane >> 2) & 1;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      uint32_t word = 0;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float v = acc[b][e];
        const uint64_t bits = __ballot(v > 0.f);
        if (e == eL) word = hiL ? (uint32_t)(bits >> 32) : (uint32_t)bits;
        const bool border = fabsf(v) < tau[b] * sd[e];
        const uint64_t bm = __ballot(border);
        if (bm) {
          if (border) {
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
            const int drel = 8 * (e >> 2) + 4 * half + (e & 3);
            fix[nfix + below] = ((uint32_t)drel << 8) | (uint32_t)(32 * b + col);
          }
          nfix += __popcll(bm);
        }
      }
      if (lane < 32) sWords[wave][lane][b] = word;
      // Flush the list before it could overflow with the next block's entries.
      const bool last = (b == 5);
      if (nfix > 0 && (last || nfix > kFixCap - 1024)) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int i = lane; i < nfix; i += 64) {
          const uint32_t ent = fix[i];
          const int drel = ent >> 8, r = ent & 0xFF;
          const uint8_t* xr = I.desc + (size_t)(d0 + drel) * kDim;
          double p = 0.0;
          for (int k = 0; k < kDim; ++k)
            p += (double)bf16_to_f32(sW[r * kWStride + k]) * (double)((int)xr[k] - (int)sMu[k]);
          const int slot = r < 128 ? (r >> 5) : 4 + ((r - 128) >> 5);
          const uint32_t bit = 1u << (r & 31);
          if (p > 0.0) atomicOr(&sWords[wave][drel][slot], bit);
          else atomicAnd(&sWords[wave][drel][slot], ~bit);
        }
        if (lane == 0) atomicAdd(pc.fixups, (unsigned long long)nfix);
        nfix = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 32 && valid) {
      const uint32_t* w = sWords[wave][lane];
      I.codes[dr] = make_uint4(w[0], w[1], w[2], w[3]);
      const uint64_t bb = (uint64_t)w[4] | ((uint64_t)w[5] << 32);
      uint32_t lo = 0, hi = 0;
      const uint32_t mask = (1u << hb.m) - 1u;
      for (int t = 0; t < hb.L; ++t) {
        const uint32_t id = (uint32_t)(bb >> (hb.m * t)) & mask;
        if (t < 4) lo |= id << (8 * t);
        else hi |= id << (8 * (t - 4));
      }
      I.ids[dr] = make_uint2(lo, hi);
      I.norms[dr] = nx;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

hipError_t launch_project(const HashBatch& hb, const ProjConsts& pc, int fp32, int n_cu,
                          hipStream_t s) {
  const int tiles = hb.tile_prefix[hb.count];
  if (tiles == 0) return hipSuccess;
  int grid = (tiles + kProjWaves - 1) / kProjWaves;
  const int cap = n_cu * 2;
  if (grid > cap) grid = cap;
  if (fp32)
    hipLaunchKernelGGL(k_project<true>, dim3(grid), dim3(256), 0, s, hb, pc);
  else
    hipLaunchKernelGGL(k_project<false>, dim3(grid), dim3(256), 0, s, hb, pc);
  return hipGetLastError();
}

}  // namespace chm

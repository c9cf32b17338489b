// Long codes and bucket ids (Sec. 2.3.1 steps (1)-(2)): the sign of the
// projection p_r(x) = sum_d W[r][d] (x_d - mu_d) = W_r . x - c_r of every
// descriptor onto every random row r, as an MFMA GEMM per 32-descriptor
// tile (c_r = W_r . mu is exact on the host).
//
// Exactness: x_d is an integer in [0, 255] and W is bfloat16, so both MFMA
// input types (bf16 and fp32) hold the operands exactly and every product is
// exact in fp32.  c_r, rounded to fp32, joins the same accumulation as more
// exact products: its three bf16 parts (truncations: each remainder is
// exact) times 1, or -c_r times 1 in the fp32 variant.  Only the fp32
// accumulation rounds: over at most 144 terms, in any order, the error is
// below 144 * 2^-23 * (||W_r|| ||x|| + |c_r|) (Cauchy-Schwarz; 2^-23 also
// covers a truncating accumulator), plus 2^-24 |c_r| for c_r itself, well
// under tau_r ||x|| + kappa_r = fixup_rel (||W_r|| ||x|| + |c_r|) for
// fixup_rel >= 1e-4.  A tile tests each row against the threshold of the
// largest ||x|| among its descriptors (a larger threshold only lists more),
// never below a tiny positive floor, so an exact zero is always listed.
// Listed projections are recomputed in fp64, which is exact for these
// operands, so every bit equals the sign of the exact value (a zero
// projection gives 0).
//
// k_project: one work-group of kProjWaves wavefronts shares W in LDS, each
// row followed by the bf16 parts of -c_r; each wavefront loops over
// 32-descriptor tiles.  W is the MFMA's A operand and the tile its B
// operand, so a lane holds 16 rows of one descriptor: rows 8q + 4h + i
// (q, i = 0..3) of each 32-row block, h being the lane's half-wave.  Taking
// them in decreasing order, the lane shifts each sign bit into a word with
// v_alignbit, by one bit, or by five (the sign and four bits the other
// half-wave's rows replace) where the other half's four rows lie below, so
// row r lands on bit r; the borderline flags (the sign of |p| minus the
// threshold) go into a second word the same way.  Borderline (descriptor,
// row) entries go to the wavefront's own region of a global list (offsets
// from a running wave-uniform count plus a DPP prefix sum over the
// lanes).  After the last tile the work-group recomputes the entries of its
// regions in fp64 and patches the bits with 32-bit atomics.  A region that
// overflowed (adversarial inputs only) is not read: its wavefront rebuilds
// every code and bucket id of its tiles from exact values instead.
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
// waves per SIMD the bf16 variant is compiled for (VGPR budget 512 / this)
#ifndef CHM_PROJ_WAVES_PER_SIMD
#define CHM_PROJ_WAVES_PER_SIMD 4
#endif
constexpr int kProjWaves = CHM_PROJ_WAVES;
constexpr int kProjWG = 64 * kProjWaves;
// bf16 per LDS row of W: 128 weights, the three bf16 parts of -c_r and 13
// zeros (one more 16-deep MFMA step), then 8 of padding: a 304-byte stride
// puts the 16-byte operand reads of 16 consecutive rows on distinct banks.
constexpr int kWK = kDim + 16;
constexpr int kWStrideX = kWK + 8;

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

// word shifted left by 32 - s bits, the top 32 - s bits of v's pattern
// shifted in (s = 31: v's sign bit; s = 27: the sign, then four bits that
// are overwritten later).
__device__ __forceinline__ uint32_t push_sign(uint32_t word, float v, uint32_t s) {
  return __builtin_amdgcn_alignbit(word, __float_as_uint(v), s);
}

// Exact projection p_r(x): sum_k W[r][k] x_k is exact in fp64 (products of
// 8-bit significands, partial sums multiples of 2^-23 below 2^21), so is
// c_r = W_r . mu; four independent partial sums keep each exact.  W is
// read from LDS (row-major bf16).
__device__ __forceinline__ double exact_projection_lds(const uint8_t* xr, const uint16_t* sWr, double c) {
  u32x4 xv[8];  // the whole row first: one memory round trip
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
    // keep the scheduler from hoisting every LDS read and conversion of W
    __builtin_amdgcn_sched_barrier(0);
  }
  return ((p0 + p1) + (p2 + p3)) - c;
}

// Sets or clears one bit; true when that changed it.
__device__ __forceinline__ bool set_bit(uint32_t* word, uint32_t bit, bool on) {
  const uint32_t old = on ? atomicOr(word, bit) : atomicAnd(word, ~bit);
  return ((old & bit) != 0) != on;
}

template <bool FP32>
__global__ __launch_bounds__(kProjWG, FP32 ? 2 : CHM_PROJ_WAVES_PER_SIMD) void k_project(HashBatch hb,
                                                                                     ProjConsts pc) {
  __shared__ uint16_t sW[kRowsPad * kWStrideX];
  __shared__ float sThr[kProjWaves][kRowsPad];  // the current tile's threshold of each row
  __shared__ float sRow[3][kRowsPad];           // tau_r, kappa_r, c_r (fp32)
  __shared__ uint32_t sCount[kProjWaves];       // entries each wavefront listed
  __shared__ unsigned long long sSum[2];        // the work-group's fix-ups and changed bits

  const int tid = threadIdx.x;
  for (int i = tid; i < 3 * kRowsPad; i += kProjWG) (&sRow[0][0])[i] = pc.tau[i];
  for (int c = tid; c < kRowsPad * (kWK / 8); c += kProjWG) {
    const int r = c / (kWK / 8), k8 = c % (kWK / 8);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (k8 < kDim / 8) {
      v = *reinterpret_cast<const uint4*>(pc.W + r * kDim + k8 * 8);
    } else if (k8 == kDim / 8) {
      // -c_r = -(hi + mid + lo): truncating to the upper 16 bits leaves an
      // exact fp32 remainder, and the last one has at most 8 significant bits
      const float c = pc.tau[2 * kRowsPad + r];
      const float hi = __uint_as_float(__float_as_uint(c) & 0xFFFF0000u);
      const float r1 = c - hi;
      const float mid = __uint_as_float(__float_as_uint(r1) & 0xFFFF0000u);
      const float lo = r1 - mid;
      v.x = (__float_as_uint(-hi) >> 16) | (__float_as_uint(-mid) & 0xFFFF0000u);
      v.y = __float_as_uint(-lo) >> 16;
    }
    uint32_t* dst = reinterpret_cast<uint32_t*>(sW + r * kWStrideX + k8 * 8);
    dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
  }
  if (tid < 2) sSum[tid] = 0;
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps tile / image in SGPRs
  const int lane = __lane_id();
  const int h = lane >> 5;
  const int col = lane & 31;
  // shift at the lowest row of the lane's lowest group: five bits where
  // the other half's rows 0..3 lie below (h = 1)
  const uint32_t s_low = h ? 27u : 31u;
  const uint32_t own = h ? 0xF0F0F0F0u : 0x0F0F0F0Fu;  // this half's bits of a block word
  // bf16 B operand of the -c_r step: x = 1 at k = 128, 129, 130
  const u32x4 ones = h ? u32x4{0u, 0u, 0u, 0u} : u32x4{0x3F803F80u, 0x3F80u, 0u, 0u};
  const int R = pc.R;

  // this wavefront's region of the fix-up list: [gw * cap_w, (gw + 1) * cap_w)
  const uint32_t gw = blockIdx.x * kProjWaves + wave;
  const uint32_t cap_w = pc.fix_cap / pc.n_waves;
  uint32_t* region = pc.fixlist + (size_t)gw * cap_w;
  uint32_t wcnt = 0;  // entries this wavefront listed so far (uniform; sCount[wave] after the tiles)

  const int total_tiles = hb.tile_prefix[hb.count];
  const int tile_step = gridDim.x * kProjWaves;
  int im = 0;  // tiles of a wavefront increase, so the image search resumes
  for (int tile = gw; tile < total_tiles; tile += tile_step) {
    while (tile >= hb.tile_prefix[im + 1]) ++im;
    const HashImage I = hash_image(hb, im);
    const int d0 = (tile - hb.tile_prefix[im]) * 32;
    const int dr = d0 + col;
    const bool valid = dr < I.n;
    const uint8_t* xrow = I.desc + (size_t)(valid ? dr : d0) * kDim;

    // The lane's bytes of its descriptor (bf16: k = 16*kb + 8*h .. +7;
    // fp32: the whole row); invalid rows read as zero.  ||x||^2 with dot4.
    uint32_t nx = 0;
    u32x4 abf[8];   // bf16 operands, converted once per tile
    u32x4 rawf[8];
    if (!FP32) {
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const u32x2 w = valid ? *(gcu32x2*)(xrow + 16 * kb + 8 * h) : u32x2{0u, 0u};
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
    // the tile's largest ||x|| (rounded up), then each row's threshold
    float sx = valid ? sqrtf((float)nx) * 1.000001f : 0.f;
    {
      // the largest over the 64 lanes (each half holds the tile's 32
      // norms) by DPP: running maxima inside each 16-lane row, then across
      // rows, read from lane 63; sx >= 0, so its bit pattern orders like
      // the value
      uint32_t v = __float_as_uint(sx);
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true));   // row_shr:1
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true));   // row_shr:2
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true));   // row_shr:4
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true));   // row_shr:8
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
      sx = __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)v, 63));
    }
    for (int r = lane; r < kRowsPad; r += 64)
      sThr[wave][r] = r < R ? fmaxf(fmaf(sRow[0][r], sx, sRow[1][r]), 1e-30f) : -1.f;
    wave_sync();

    uint32_t w4 = 0u;  // block 4's word, kept for the bucket ids
    // unrolled: the scheduler may start a block's W reads and MFMA chain
    // beside the previous block's epilogue
#pragma unroll
    for (int blk = 0; blk < 6; ++blk) {
      f32x16 acc;
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] = 0.f;
      const int row = 32 * blk + col;  // the A operand row this lane supplies
      if (!FP32) {
        const uint16_t* wr = sW + row * kWStrideX + 8 * h;
#pragma unroll
        for (int kb = 0; kb < 9; ++kb) {
          const u32x4 aw = *reinterpret_cast<const u32x4*>(wr + 16 * kb);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, aw),
                                                        __builtin_bit_cast(bf16x8, kb < 8 ? abf[kb] : ones),
                                                        acc, 0, 0, 0);
        }
      } else {
        const uint16_t* wr = sW + row * kWStrideX;
#pragma unroll
        for (int kk = 0; kk < 64; ++kk) {
          const int k = 2 * kk + h;
          const float xv = (float)((rawf[kk >> 3][(kk >> 1) & 3] >> (8 * (k & 3))) & 0xFFu);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(bf16_to_f32(wr[k]), xv, acc, 0, 0, 0);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(h ? 0.f : -sRow[2][row], h ? 0.f : 1.f, acc, 0, 0, 0);
      }
      // acc[4q + i] is row 32 blk + 8q + 4h + i of descriptor col
      const float4* tp = reinterpret_cast<const float4*>(&sThr[wave][32 * blk + 4 * h]);
      uint32_t sg = 0u, bd = 0u;
#pragma unroll
      for (int q = 3; q >= 0; --q) {
        const float4 t4 = tp[2 * q];
        const float th[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
        for (int i = 3; i >= 0; --i) {
          const int e = 4 * q + i;
          const uint32_t sh = i ? 31u : q ? 27u : s_low;
          sg = push_sign(sg, acc[e], sh);
          bd = push_sign(bd, fabsf(acc[e]) - th[i], sh);
        }
      }
      // the block word: this half's rows from this lane, the other half's
      // from its partner (lane ^ 32); bit r = 1 for a positive projection
      const uint32_t o = __shfl_xor(sg, 32);
      const uint32_t word = ~((sg & own) | (o & ~own));
      if (blk < 4) {
        if (h == 0 && valid) reinterpret_cast<uint32_t*>(I.codes + dr)[blk] = word;
      } else if (blk == 4) {
        w4 = word;
      } else if (h == 0 && valid) {
        const uint64_t bb = (uint64_t)w4 | ((uint64_t)word << 32);
        const uint32_t mask = (1u << hb.m) - 1u;
        for (int t = 0; t < hb.L; ++t)
          I.ids[(size_t)t * I.n_pad + dr] = (uint8_t)((uint32_t)(bb >> (hb.m * t)) & mask);
      }
      // borderline entries of this half's rows (rows >= R have threshold -1
      // and are never flagged) go to the wavefront's region
      bd = valid ? (bd & own) : 0u;
      if (__ballot(bd != 0u)) {  // consecutive slots: a DPP prefix sum of the lanes' counts
        const uint32_t nb = (uint32_t)__popc(bd);
        const uint32_t incl = wave_incl_add(nb);
        uint32_t idx = wcnt + incl - nb;
        wcnt += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        while (bd) {
          const int bit = __builtin_ctz(bd);
          bd &= bd - 1u;
          if (idx < cap_w) region[idx] = ((uint32_t)im << 24) | ((uint32_t)(32 * blk + bit) << 16) | (uint32_t)dr;
          ++idx;
        }
      }
    }
    if (h == 0 && valid) I.norms[dr] = nx;
    wave_sync();  // sThr is rewritten by the next tile
  }
  if (lane == 0) sCount[wave] = wcnt;

  // Fix-up of the work-group's listed entries (regions concatenated in
  // wavefront order; a region that overflowed counts as empty), 64 entries
  // per wavefront at a time.  The barrier also makes the codes and entries
  // written above visible to the other wavefronts of the work-group.
  __syncthreads();
  const uint32_t wcount = sCount[wave];
  unsigned long long n_fix = 0, n_flip = 0;
  {
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kProjWaves; ++w) total += sCount[w] <= cap_w ? sCount[w] : 0u;
    for (uint32_t k = (uint32_t)wave * 64u + (uint32_t)lane; k < total; k += kProjWaves * 64u) {
      int w = 0;
      uint32_t base = 0;
      for (;; ++w) {
        const uint32_t c = sCount[w] <= cap_w ? sCount[w] : 0u;
        if (k < base + c) break;
        base += c;
      }
      const uint32_t ent = pc.fixlist[(size_t)(blockIdx.x * kProjWaves + w) * cap_w + (k - base)];
      const int eim = ent >> 24, row = (ent >> 16) & 0xFF, d = ent & 0xFFFF;
      const HashImage I = hash_image(hb, eim);
      const double p = exact_projection_lds(I.desc + (size_t)d * kDim, sW + row * kWStrideX, pc.cmu[row]);
      bool changed;
      if (row < 128) {
        changed = set_bit(reinterpret_cast<uint32_t*>(I.codes + d) + (row >> 5), 1u << (row & 31), p > 0.0);
      } else {
        const int t = (row - 128) / hb.m, j = (row - 128) % hb.m;
        const size_t byte = (size_t)t * I.n_pad + d;
        uint32_t* wd = reinterpret_cast<uint32_t*>(I.ids + (byte & ~(size_t)3));
        changed = set_bit(wd, 1u << (8 * (byte & 3) + j), p > 0.0);
      }
      n_fix += 1;
      if (changed) ++n_flip;
    }
  }
  if (wcount > cap_w) {
    // Overflow: rebuild every code and bucket id of this wavefront's tiles
    // from exact values.  Lane (col, h) computes rows 96 h .. 96 h + 95 of
    // descriptor col (words 3h .. 3h + 2); its partner supplies the rest.
    im = 0;
    for (int tile = gw; tile < total_tiles; tile += tile_step) {
      while (tile >= hb.tile_prefix[im + 1]) ++im;
      const HashImage I = hash_image(hb, im);
      const int dr = (tile - hb.tile_prefix[im]) * 32 + col;
      const bool valid = dr < I.n;
      uint32_t w3[3] = {0u, 0u, 0u};
      if (valid) {
        const uint8_t* xr = I.desc + (size_t)dr * kDim;
#pragma unroll 1
        for (int r = 96 * h; r < 96 * h + 96 && r < R; ++r) {
          const double p = exact_projection_lds(xr, sW + r * kWStrideX, pc.cmu[r]);
          const int k = (r - 96 * h) >> 5;
          const uint32_t bit = p > 0.0 ? 1u << (r & 31) : 0u;
          w3[0] |= k == 0 ? bit : 0u;
          w3[1] |= k == 1 ? bit : 0u;
          w3[2] |= k == 2 ? bit : 0u;
        }
        n_fix += (unsigned long long)(min(96 * h + 96, R) - min(96 * h, R));
      }
      uint32_t o3[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) o3[k] = __shfl_xor(w3[k], 32);
      if (h == 0 && valid) {
        const uint32_t w[6] = {w3[0], w3[1], w3[2], o3[0], o3[1], o3[2]};
        const uint4 old = I.codes[dr];
        uint32_t flips = __popc(old.x ^ w[0]) + __popc(old.y ^ w[1]) + __popc(old.z ^ w[2]) + __popc(old.w ^ w[3]);
        I.codes[dr] = make_uint4(w[0], w[1], w[2], w[3]);
        const uint64_t bb = (uint64_t)w[4] | ((uint64_t)w[5] << 32);
        const uint32_t mask = (1u << hb.m) - 1u;
        for (int t = 0; t < hb.L; ++t) {
          const uint8_t nb = (uint8_t)((uint32_t)(bb >> (hb.m * t)) & mask);
          flips += __popc((uint32_t)(I.ids[(size_t)t * I.n_pad + dr] ^ nb));
          I.ids[(size_t)t * I.n_pad + dr] = nb;
        }
        n_flip += flips;
      }
    }
  }
  if (n_fix) atomicAdd(&sSum[0], n_fix);
  if (n_flip) atomicAdd(&sSum[1], n_flip);
  __syncthreads();
  if (tid == 0) {
    if (sSum[0]) atomicAdd(pc.fixups, sSum[0]);
    if (sSum[1]) atomicAdd(pc.fixups + 1, sSum[1]);
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
  return hipGetLastError();
}

}  // namespace chm

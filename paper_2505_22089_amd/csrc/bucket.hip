// Lookup tables of Sec. 2.3.1 step (1): for every image and table, the 2^m
// buckets as a stable counting sort of the bucket ids (CSR: offsets +
// members, members ascending inside each bucket).  One work-group per
// (image, table); the stable scatter ranks equal ids inside a wavefront with
// ballots and across wavefronts with per-wave counts in LDS.
#include "chm_internal.h"

namespace chm {

constexpr int kBucketWG = 256;
constexpr int kBucketWaves = kBucketWG / 64;

__device__ __forceinline__ uint32_t id_byte(uint2 v, int t) {
  return ((t < 4 ? v.x >> (8 * t) : v.y >> (8 * (t - 4)))) & 0xFFu;
}

__global__ __launch_bounds__(kBucketWG) void k_buckets(HashBatch hb) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kBucketWaves][256];

  const int im = blockIdx.x / hb.L;
  const int t = blockIdx.x % hb.L;
  const HashImage& I = hb.img[im];
  const int n = I.n;
  const int nb = 1 << hb.m;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = __lane_id();

  hist[tid] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += kBucketWG) atomicAdd(&hist[id_byte(I.ids[i], t)], 1u);
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int b = 0; b < nb; ++b) {
      base[b] = run;
      I.offsets[t * (nb + 1) + b] = (int32_t)run;
      run += hist[b];
    }
    I.offsets[t * (nb + 1) + nb] = (int32_t)run;
  }
  __syncthreads();

  uint16_t* mem = I.members + (size_t)t * I.n_pad;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int c = 0; c < n; c += kBucketWG) {
    const int i = c + tid;
    const bool valid = i < n;
    const uint32_t b = valid ? id_byte(I.ids[i], t) : 0u;
#pragma unroll
    for (int w = 0; w < kBucketWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < hb.m; ++bit) {
      const bool set = (b >> bit) & 1u;
      const uint64_t bm = __ballot(valid && set);
      peers &= set ? bm : ~bm;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[wave][b] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[b] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][b];
      mem[pos] = (uint16_t)i;
    }
    __syncthreads();
    if (tid < nb) {
      uint32_t add = 0;
#pragma unroll
      for (int w = 0; w < kBucketWaves; ++w) add += wcnt[w][tid];
      base[tid] += add;
    }
    __syncthreads();
  }
  for (int i = n + tid; i < I.n_pad; i += kBucketWG) mem[i] = 0;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_buckets(const HashBatch& hb, hipStream_t s) {
  if (hb.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_buckets, dim3(hb.count * hb.L), dim3(kBucketWG), 0, s, hb);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace chm

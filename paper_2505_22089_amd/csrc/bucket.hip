// Lookup tables of Sec. 2.3.1 step (1): for every image and table, the 2^m
// buckets as a stable counting sort of the bucket ids (CSR: offsets +
// members, members ascending inside each bucket).
//
// A member is stored as 16 j, the byte offset of db point j's long code, so
// a matching lane addresses the code with no arithmetic.  Each bucket's
// range of the members array is padded to a multiple of 8 entries with
// copies of the bucket's first (smallest) member, and starts at a multiple
// of 8: a matching lane then reads whole aligned 32-byte blocks of 8 members
// and needs no bounds test per entry (a repeated member is a candidate
// already seen, which the set semantics of the candidate list drop).
// offsets[t][b] .. offsets[t][b + 1] is the padded range and counts[t][b]
// the bucket's members without pads.
//
// k_buckets: one work-group per (image, table).  The table's ids are staged
// in LDS once; each wavefront owns a contiguous segment of descriptors.
// Pass 1 counts per (wavefront, bucket) and finds each bucket's first
// member; a scan turns the counts into each wavefront's starting position
// inside each bucket; pass 2 scatters, ranking equal ids inside a 64-lane
// chunk by the lanes' bits in a per-wavefront LDS mask of each bucket (each
// lane ORs its bit in: the rank is the count of lower lanes with the same
// id), so the order inside a bucket is the descriptor order; the pads are
// written last.  k_buckets_small does the same for images of up to
// kSmallMaxN descriptors with the table assembled in LDS and written out
// in whole 16-byte stores.
//
// k_tcodes: for images too large for the query-major kernel's LDS code
// stage, the codes again in bucket order (tcodes[t][pos] = codes[j] for
// members[t][pos] = 16 j), so that a block's 8 codes are one contiguous 128
// bytes.  Written in order (coalesced), the codes gathered from L2.
#include "chm_internal.h"

namespace chm {

constexpr int kBucketWG = 1024;
constexpr int kBucketWaves = kBucketWG / 64;
constexpr int kBucketMaxN = 65536;

// Lanes of this wavefront's 64-element chunk holding the same bucket id as
// this lane: every valid lane ORs its bit into the wavefront's mask of its
// bucket, reads the mask back, and the mask is cleared again after all
// lanes have read it (a wavefront's LDS operations run in program order).
__device__ __forceinline__ uint64_t peers_of(unsigned long long* mask, uint32_t b, bool valid) {
  const int lane = __lane_id();
  if (valid) atomicOr(&mask[b], 1ull << lane);
  __builtin_amdgcn_wave_barrier();
  const uint64_t peers = valid ? mask[b] : 0ull;
  __builtin_amdgcn_wave_barrier();
  if (valid && (peers & ((1ull << lane) - 1ull)) == 0) mask[b] = 0ull;
  __builtin_amdgcn_wave_barrier();
  return peers;
}

__global__ __launch_bounds__(kBucketWG) void k_buckets(HashBatch hb) {
  extern __shared__ uint8_t sId[];  // the table's ids (dynamic: the batch's largest n_pad)
  __shared__ uint32_t cnt[kBucketWaves][256];
  __shared__ unsigned long long peer[kBucketWaves][256];  // per wavefront, zero between chunks
  __shared__ uint32_t first[256];   // smallest member of each bucket
  __shared__ uint32_t real[256];    // members of each bucket
  __shared__ uint32_t pbase[256];   // padded start of each bucket
  __shared__ uint32_t s_total;      // padded length of the table

  const int im = blockIdx.x / hb.L;
  const int t = blockIdx.x % hb.L;
  const HashImage I = hash_image(hb, im);
  const int n = I.n;
  const int nb = 1 << hb.m;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = __lane_id();
  const uint8_t* ids = I.ids + (size_t)t * I.n_pad;

  // stage ids (n_pad is a multiple of 8 and the table start is 8-byte aligned)
  for (int i = tid; i < I.n_pad / 8; i += kBucketWG)
    reinterpret_cast<uint2*>(sId)[i] = reinterpret_cast<const uint2*>(ids)[i];
  for (int i = tid; i < kBucketWaves * 256; i += kBucketWG) {
    (&cnt[0][0])[i] = 0;
    (&peer[0][0])[i] = 0ull;
  }
  for (int i = tid; i < 256; i += kBucketWG) first[i] = 0xFFFFFFFFu;
  __syncthreads();

  // each wavefront: a contiguous segment of whole 64-lane chunks
  const int chunks = (n + 63) / 64;
  const int per = (chunks + kBucketWaves - 1) / kBucketWaves;
  const int c0 = wave * per, c1 = min(chunks, c0 + per);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  for (int c = c0; c < c1; ++c) {
    const int i = c * 64 + lane;
    const bool valid = i < n;
    const uint32_t b = valid ? sId[i] : 0u;
    const uint64_t peers = peers_of(peer[wave], b, valid);
    if (valid && (peers & lt) == 0) {
      cnt[wave][b] += (uint32_t)__popcll(peers);
      atomicMin(&first[b], (uint32_t)i);
    }
  }
  __syncthreads();

  // padded offsets of the table, and each wavefront's start inside each bucket
  if (tid < 64) {
    // scan over buckets: lane handles buckets 4*lane .. 4*lane+3
    uint32_t tot[4], run = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = 4 * lane + k;
      uint32_t s = 0;
      if (b < nb)
        for (int w = 0; w < kBucketWaves; ++w) s += cnt[w][b];
      if (b < nb) {
        real[b] = s;
        I.counts[t * nb + b] = (int32_t)s;
      }
      tot[k] = (s + 7u) & ~7u;
      run += tot[k];
    }
    const uint32_t incl = wave_incl_add(run);
    uint32_t base = incl - run;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = 4 * lane + k;
      if (b < nb) {
        I.offsets[t * (nb + 1) + b] = (int32_t)base;
        pbase[b] = base;
        uint32_t pos = base;
        for (int w = 0; w < kBucketWaves; ++w) {
          const uint32_t c = cnt[w][b];
          cnt[w][b] = pos;
          pos += c;
        }
      }
      base += tot[k];
    }
    if (lane == 63) {
      I.offsets[t * (nb + 1) + nb] = (int32_t)incl;
      s_total = incl;
    }
  }
  __syncthreads();

  uint32_t* mem = I.members + (size_t)t * I.m_stride;
  for (int c = c0; c < c1; ++c) {
    const int i = c * 64 + lane;
    const bool valid = i < n;
    const uint32_t b = valid ? sId[i] : 0u;
    const uint64_t peers = peers_of(peer[wave], b, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t start = valid ? cnt[wave][b] : 0u;
    if (valid) mem[start + rank] = 16u * (uint32_t)i;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) cnt[wave][b] = start + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  // pads (positions no scattered member takes) and the unused tail
  for (int b = tid; b < nb; b += kBucketWG) {
    const uint32_t c = real[b], pc = (c + 7u) & ~7u;
    for (uint32_t k = c; k < pc; ++k) mem[pbase[b] + k] = 16u * first[b];
  }
  for (int i = (int)s_total + tid; i < I.m_stride; i += kBucketWG) mem[i] = 0;
}

// Images up to kSmallMaxN descriptors: the same table built in LDS and
// written out with whole 16-byte stores.  Scattering each member straight
// to global memory (one 4-byte store per member, a different line per
// lane) took about half of the kernel.  The counting pass also keeps each
// member's rank inside its (wavefront, bucket) run, so the scatter needs no
// second ranking.  Dynamic LDS: the ids, the ranks (2 B), then one region
// that holds the peer masks during the counting pass and the bucket-ordered
// members afterwards; with 16-bit counts the work-group stays within half a
// CU's LDS.
constexpr int kSmallMaxN = 8192;
constexpr int kSmallMemMax = kSmallMaxN + 7 * 256;          // members per table, at most
constexpr int kSmallRankOff = kSmallMaxN;                   // byte offsets in dynamic LDS
constexpr int kSmallUnionOff = 3 * kSmallMaxN;
constexpr int kSmallUnionBytes = (kBucketWaves * 256 * 8 > 4 * kSmallMemMax) ? kBucketWaves * 256 * 8
                                                                             : 4 * kSmallMemMax;
constexpr int kSmallDynBytes = kSmallUnionOff + kSmallUnionBytes;

__global__ __launch_bounds__(kBucketWG) void k_buckets_small(HashBatch hb) {
  extern __shared__ __attribute__((aligned(16))) uint8_t sDyn[];
  __shared__ uint16_t cnt[kBucketWaves][256];
  __shared__ uint32_t first[256];
  __shared__ uint32_t real[256];
  __shared__ uint32_t pbase[256];
  __shared__ uint32_t s_total;
  uint8_t* sId = sDyn;
  uint16_t* sRank = reinterpret_cast<uint16_t*>(sDyn + kSmallRankOff);
  unsigned long long(*peer)[256] = reinterpret_cast<unsigned long long(*)[256]>(sDyn + kSmallUnionOff);
  uint32_t* sMem = reinterpret_cast<uint32_t*>(sDyn + kSmallUnionOff);

  const int im = blockIdx.x / hb.L;
  const int t = blockIdx.x % hb.L;
  const HashImage I = hash_image(hb, im);
  const int n = I.n;
  const int nb = 1 << hb.m;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = __lane_id();
  const uint8_t* ids = I.ids + (size_t)t * I.n_pad;

  for (int i = tid; i < I.n_pad / 8; i += kBucketWG)
    reinterpret_cast<uint2*>(sId)[i] = reinterpret_cast<const uint2*>(ids)[i];
  for (int i = tid; i < kBucketWaves * 256; i += kBucketWG) {
    (&cnt[0][0])[i] = 0;
    (&peer[0][0])[i] = 0ull;
  }
  for (int i = tid; i < 256; i += kBucketWG) first[i] = 0xFFFFFFFFu;
  __syncthreads();

  const int chunks = (n + 63) / 64;
  const int per = (chunks + kBucketWaves - 1) / kBucketWaves;
  const int c0 = wave * per, c1 = min(chunks, c0 + per);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int c = c0; c < c1; ++c) {
    const int i = c * 64 + lane;
    const bool valid = i < n;
    const uint32_t b = valid ? sId[i] : 0u;
    const uint64_t peers = peers_of(peer[wave], b, valid);
    if (valid) sRank[i] = (uint16_t)(cnt[wave][b] + (uint32_t)__popcll(peers & lt));
    if (valid && (peers & lt) == 0) {  // after every peer has read the count (program order)
      cnt[wave][b] = (uint16_t)(cnt[wave][b] + (uint32_t)__popcll(peers));
      atomicMin(&first[b], (uint32_t)i);
    }
  }
  __syncthreads();  // the peer masks are dead from here: the region holds the members

  if (tid < 64) {
    uint32_t tot[4], run = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = 4 * lane + k;
      uint32_t s = 0;
      if (b < nb)
        for (int w = 0; w < kBucketWaves; ++w) s += cnt[w][b];
      if (b < nb) {
        real[b] = s;
        I.counts[t * nb + b] = (int32_t)s;
      }
      tot[k] = (s + 7u) & ~7u;
      run += tot[k];
    }
    const uint32_t incl = wave_incl_add(run);
    uint32_t base = incl - run;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = 4 * lane + k;
      if (b < nb) {
        I.offsets[t * (nb + 1) + b] = (int32_t)base;
        pbase[b] = base;
        uint32_t pos = base;
        for (int w = 0; w < kBucketWaves; ++w) {
          const uint32_t c = cnt[w][b];
          cnt[w][b] = (uint16_t)pos;
          pos += c;
        }
      }
      base += tot[k];
    }
    if (lane == 63) {
      I.offsets[t * (nb + 1) + nb] = (int32_t)incl;
      s_total = incl;
    }
  }
  __syncthreads();

  // members into LDS: wavefront start in the bucket plus the rank; then the
  // pads (copies of each bucket's first member) and the unused tail
  for (int i = tid; i < n; i += kBucketWG) sMem[cnt[(i >> 6) / per][sId[i]] + sRank[i]] = 16u * (uint32_t)i;
  for (int b = tid; b < nb; b += kBucketWG) {
    const uint32_t c = real[b], pc = (c + 7u) & ~7u;
    for (uint32_t k = c; k < pc; ++k) sMem[pbase[b] + k] = 16u * first[b];
  }
  for (int i = (int)s_total + tid; i < I.m_stride; i += kBucketWG) sMem[i] = 0;
  __syncthreads();
  uint4* mem = reinterpret_cast<uint4*>(I.members + (size_t)t * I.m_stride);  // m_stride: a multiple of 8
  for (int i = tid; i < I.m_stride / 4; i += kBucketWG) mem[i] = reinterpret_cast<const uint4*>(sMem)[i];
}

// Bucket-ordered code copies.  Work-groups are dealt to the XCDs
// round-robin; work-group w = x + n_xcd k (XCD x) copies slice k % slices
// of batch image x + n_xcd (k / slices): entries [s kTcPer, (s + 1) kTcPer)
// of its L x m_stride.  All slices of an image thus run on one XCD, whose
// L2 holds the image's codes for the gathers.  Images without a copy, and
// work-groups past the batch, return at once.  A thread takes groups of 4
// consecutive entries (one 16-byte load of their members, 4 code gathers,
// 4 stores), two groups per pass.
constexpr int kTcWG = 256;
constexpr int kTcPer = 8192;

__global__ __launch_bounds__(kTcWG) void k_tcodes(HashBatch hb, int slices, int n_xcd) {
  const int x = (int)(blockIdx.x % (unsigned)n_xcd);
  const int k = (int)(blockIdx.x / (unsigned)n_xcd);
  const int im = x + n_xcd * (k / slices);
  if (im >= hb.count) return;
  const HashImage I = hash_image(hb, im);
  if (!I.tcodes) return;
  const uint32_t total = (uint32_t)hb.L * (uint32_t)I.m_stride;  // a multiple of 8
  const uint32_t s0 = (uint32_t)(k % slices) * (uint32_t)kTcPer;
  const uint32_t s1 = min(total, s0 + (uint32_t)kTcPer);
  const char* codes = reinterpret_cast<const char*>(I.codes);
  // two groups of 4 entries per pass (both member loads, then the eight
  // gathers, then the stores), then one left over
  uint32_t pos = s0 + 4 * threadIdx.x;
  for (; pos + 4 * kTcWG < s1; pos += 8 * kTcWG) {
    const uint4 m = *reinterpret_cast<const uint4*>(I.members + pos);
    const uint4 n = *reinterpret_cast<const uint4*>(I.members + pos + 4 * kTcWG);
    const uint4 c0 = *reinterpret_cast<const uint4*>(codes + m.x);
    const uint4 c1 = *reinterpret_cast<const uint4*>(codes + m.y);
    const uint4 c2 = *reinterpret_cast<const uint4*>(codes + m.z);
    const uint4 c3 = *reinterpret_cast<const uint4*>(codes + m.w);
    const uint4 d0 = *reinterpret_cast<const uint4*>(codes + n.x);
    const uint4 d1 = *reinterpret_cast<const uint4*>(codes + n.y);
    const uint4 d2 = *reinterpret_cast<const uint4*>(codes + n.z);
    const uint4 d3 = *reinterpret_cast<const uint4*>(codes + n.w);
    I.tcodes[pos] = c0;
    I.tcodes[pos + 1] = c1;
    I.tcodes[pos + 2] = c2;
    I.tcodes[pos + 3] = c3;
    I.tcodes[pos + 4 * kTcWG] = d0;
    I.tcodes[pos + 4 * kTcWG + 1] = d1;
    I.tcodes[pos + 4 * kTcWG + 2] = d2;
    I.tcodes[pos + 4 * kTcWG + 3] = d3;
  }
  if (pos < s1) {
    const uint4 m = *reinterpret_cast<const uint4*>(I.members + pos);
    const uint4 c0 = *reinterpret_cast<const uint4*>(codes + m.x);
    const uint4 c1 = *reinterpret_cast<const uint4*>(codes + m.y);
    const uint4 c2 = *reinterpret_cast<const uint4*>(codes + m.z);
    const uint4 c3 = *reinterpret_cast<const uint4*>(codes + m.w);
    I.tcodes[pos] = c0;
    I.tcodes[pos + 1] = c1;
    I.tcodes[pos + 2] = c2;
    I.tcodes[pos + 3] = c3;
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_buckets(const HashBatch& hb, int n_xcd, hipStream_t s) {
  if (hb.count == 0) return hipSuccess;
  // LDS for the ids sized to the batch, so that small images leave room for
  // several work-groups per CU
  int n_pad = 8;
  for (int i = 0; i < hb.count; ++i) n_pad = max(n_pad, (hb.img[i].n + 7) / 8 * 8);
  if (n_pad > kBucketMaxN) return hipErrorInvalidValue;
  hipError_t e;
  if (n_pad <= kSmallMaxN) {
    hipLaunchKernelGGL(k_buckets_small, dim3(hb.count * hb.L), dim3(kBucketWG), (size_t)kSmallDynBytes, s, hb);
  } else {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_buckets), hipFuncAttributeMaxDynamicSharedMemorySize,
                            kBucketMaxN);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_buckets, dim3(hb.count * hb.L), dim3(kBucketWG), (size_t)n_pad, s, hb);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int slices = 0;
  for (int i = 0; i < hb.count; ++i) {
    const ImageLayout l = image_layout(hb.L, hb.m, hb.img[i].n);
    if (l.has_tcodes) slices = max(slices, (hb.L * l.m_stride + kTcPer - 1) / kTcPer);
  }
  if (slices == 0) return hipSuccess;
  if (n_xcd < 1) n_xcd = 1;
  const int per_xcd = (hb.count + n_xcd - 1) / n_xcd;
  hipLaunchKernelGGL(k_tcodes, dim3(n_xcd * per_xcd * slices), dim3(kTcWG), 0, s, hb, slices, n_xcd);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace chm

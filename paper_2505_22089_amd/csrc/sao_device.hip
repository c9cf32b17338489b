// SAO local geometric constraint (Sec. 2.3.3, Fig. 4) on the device: the same
// scores as the host implementation, for up to 8 neighbours.
//
// Pairs go in batches, each with its own scratch in the caller's work buffer.
//  1. k_sao_build, one work-group per pair: the matched query rows are
//     compacted in row order (a block scan of the match flags), so a compact
//     index orders like the query row that labels the match; then, for the
//     query image and for the db image, the matched keypoints are
//     counting-sorted into a uniform grid of about two points per cell.
//  2. k_sao_search, one thread per match: in each image an exact ring
//     search over the cells finds the N nearest other matches (64-bit
//     squared distances, ties by compact index), stopping once the next
//     ring's distance bound reaches the N-th distance; the two neighbour
//     lists are sorted by angle (half-plane, then the sign of a 64-bit cross
//     product) and their labels compared by the cyclic edit distance, the
//     least Levenshtein distance over the rotations of one list (Maes, 1990).
// All geometry is exact for coordinates below 2^30 in magnitude.  A pair
// whose input breaks the contract (a db row outside the db image, or a
// coordinate out of range) keeps no match and is counted in the first word
// of the work buffer; every index stays inside its buffer whatever the input.
#include <algorithm>
#include <vector>

#include "chm.h"
#include "chm_host.h"
#include "chm_internal.h"

namespace chm {

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s);

namespace {

constexpr int kSaoWG = 256;                        // search: one thread per match
constexpr int kSaoBuildWG = 256;                   // build: one work-group per pair
constexpr int kSaoBuildWaves = kSaoBuildWG / 64;
constexpr int kSaoMaxN = kSaoMaxNeighbors;
constexpr int kSaoBatch = 512;  // pairs per launch pair (scratch is per pair)
// grid density, points per cell on average (4 per cell: the same time on
// the benchmark workload's matches; 8: 21% slower)
constexpr double kSaoPointsPerCell = 2.0;
constexpr int64_t kSaoCoordLimit = int64_t(1) << 30;
constexpr int64_t kSaoSqrtMax = 3037000499LL;  // floor(sqrt(2^63 - 1))

struct SaoPair {
  const int32_t* kq;  // query keypoints (x, y) per row
  const int32_t* kd;  // db keypoints
  int32_t nq, nd;
  int64_t off;        // first query row's position in the match arrays
};

struct GridInfo {
  int64_t x0, y0, cell, nx, ny;
};

struct PairInfo {  // 128 bytes at the head of a pair's scratch
  int32_t M, bad, pad0, pad1;
  GridInfo g[2];
  int32_t pad[4];
};
static_assert(sizeof(PairInfo) <= 128, "pair info fits its 128 bytes");

struct SaoArgs {
  const SaoPair* pairs;  // this batch's pairs
  int32_t n_pairs;
  int32_t n_max;         // rows of the largest query image (scratch capacity)
  const int32_t* match;
  int32_t* out;
  int32_t* ced;          // may be null
  int32_t nn, num, den;
  uint8_t* scratch;
  uint64_t scratch_bytes;  // per pair
  int32_t* errors;
};

__host__ __device__ inline uint64_t round16(uint64_t v) { return (v + 15) & ~uint64_t(15); }
__host__ __device__ inline int64_t sao_cells_max(int64_t n) { return 4 * n + 64; }

// A pair's scratch for capacity n: info, rows[n], and per image pts[n]
// (int4: x, y, compact index; in cell order), cell[C + 1] (cell ends) and
// xy[n] (the keypoint of each compact match: one load instead of three
// dependent ones through rows, the matches and the keypoints).
struct PairScratch {
  PairInfo* info;
  int32_t* rows;
  int4* pts[2];
  int32_t* cell[2];
  int2* xy[2];
};

__host__ __device__ inline uint64_t pair_scratch_bytes(int64_t n) {
  const int64_t C = sao_cells_max(n);
  return 128 + round16(4 * n) + 2 * (round16(16 * n) + round16(4 * (C + 1)) + round16(8 * n));
}

__device__ inline PairScratch scratch_at(const SaoArgs& a, int pair) {
  const int64_t n = a.n_max, C = sao_cells_max(n);
  uint8_t* p = a.scratch + a.scratch_bytes * (uint64_t)pair;
  PairScratch s;
  s.info = reinterpret_cast<PairInfo*>(p);
  p += 128;
  s.rows = reinterpret_cast<int32_t*>(p);
  p += round16(4 * n);
  for (int side = 0; side < 2; ++side) {
    s.pts[side] = reinterpret_cast<int4*>(p);
    p += round16(16 * n);
    s.cell[side] = reinterpret_cast<int32_t*>(p);
    p += round16(4 * (C + 1));
    s.xy[side] = reinterpret_cast<int2*>(p);
    p += round16(8 * n);
  }
  return s;
}

// Exclusive prefix of v over the work-group; *total receives the sum.
template <int WAVES>
__device__ inline int block_exclusive(int v, int* s_tmp, int* total) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const int incl = (int)wave_incl_add((uint32_t)v);
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  int before = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const int t = s_tmp[w];
    before += w < wave ? t : 0;
    sum += t;
  }
  __syncthreads();
  *total = sum;
  return before + incl - v;
}

// Barrier between phases that hand data through global memory (plain
// stores and L2 atomics of other waves of the work-group): the release
// completes this wave's writes, and the agent-scope acquire invalidates the
// CU's L1, so no wave reads a line cached before the phase.
__device__ inline void phase_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores and atomics have completed
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ inline bool lex_less(uint64_t d1, int32_t i1, uint64_t d2, int32_t i2) {
  return d1 < d2 || (d1 == d2 && i1 < i2);
}

// The 8 nearest candidates seen so far, ascending by (squared distance,
// compact index); empty slots hold (UINT64_MAX, INT32_MAX).
struct NearList {
  uint64_t d[kSaoMaxN];
  int32_t i[kSaoMaxN];
};

// Inserts (d, idx), which the caller has checked to be below the n-th entry.
__device__ inline void near_insert(NearList& L, uint64_t d, int32_t idx) {
  bool lt[kSaoMaxN];
#pragma unroll
  for (int k = 0; k < kSaoMaxN; ++k) lt[k] = lex_less(d, idx, L.d[k], L.i[k]);
#pragma unroll
  for (int k = kSaoMaxN - 1; k >= 1; --k) {
    if (lt[k]) {
      L.d[k] = lt[k - 1] ? L.d[k - 1] : d;
      L.i[k] = lt[k - 1] ? L.i[k - 1] : idx;
    }
  }
  if (lt[0]) {
    L.d[0] = d;
    L.i[0] = idx;
  }
}

// A grid in global memory (the build kernel's output).
struct GlobalGrid {
  const int32_t* cell;  // cell ends
  const int4* pts;      // x, y, compact index, in cell order
  __device__ int32_t end(int64_t cid) const { return cell[cid]; }
  __device__ int4 pt(int32_t k) const { return pts[k]; }
};

// The n nearest other points of compact point c (at x, y): their compact
// indices in out[0..n), ascending by (squared distance, index).  With
// PACKED (every |dx|, |dy| below 2^23 and indices below 2^16) the two parts
// travel as one 64-bit key (d2 << 16 | index), which orders the same way.
template <bool PACKED, class Grid>
__device__ inline void ring_search(const Grid& G, const GridInfo& g, int64_t x, int64_t y, int32_t c, int n,
                                   int32_t (&out)[kSaoMaxN]) {
  NearList L;        // general keys
  uint64_t K[kSaoMaxN];  // packed keys
#pragma unroll
  for (int k = 0; k < kSaoMaxN; ++k) {
    L.d[k] = ~uint64_t(0);
    L.i[k] = INT32_MAX;
    K[k] = ~uint64_t(0);
  }
  // cell counts are at most 4 M + 64, so cell coordinates fit 32 bits
  const int32_t nx = (int32_t)g.nx, ny = (int32_t)g.ny;
  const int32_t ix = (int32_t)min(max((x - g.x0) / g.cell, int64_t(0)), g.nx - 1);
  const int32_t iy = (int32_t)min(max((y - g.y0) / g.cell, int64_t(0)), g.ny - 1);
  const int32_t rmax = max(max(ix, nx - 1 - ix), max(iy, ny - 1 - iy));
  const int32_t xs = (int32_t)x, ys = (int32_t)y;
  uint64_t wd = ~uint64_t(0);  // the n-th entry (the last one kept)
  int32_t wi = INT32_MAX;
  uint64_t wk = ~uint64_t(0);
  int found = 0;
  for (int32_t r = 0; r <= rmax; ++r) {
    for (int32_t j = max(iy - r, 0); j <= min(iy + r, ny - 1); ++j) {
      const bool edge = r == 0 || j == iy - r || j == iy + r;
      const int32_t step = edge ? 1 : 2 * r;
      for (int32_t i = ix - r; i <= ix + r; i += step) {
        if (i < 0 || i >= nx) continue;
        const int32_t cid = j * nx + i;
        const int32_t b = cid ? G.end(cid - 1) : 0, e = G.end(cid);
        for (int32_t k = b; k < e; ++k) {
          const int4 p = G.pt(k);
          if (p.z == c) continue;
          // |dx|, |dy| < 2^31: squares as 32 x 32 -> 64-bit products
          const uint32_t ax = (uint32_t)abs(p.x - xs), ay = (uint32_t)abs(p.y - ys);
          const uint64_t d2 = (uint64_t)ax * ax + (uint64_t)ay * ay;
          ++found;
          if (PACKED) {
            const uint64_t key = (d2 << 16) | (uint32_t)p.z;
            if (key >= wk) continue;
            bool lt[kSaoMaxN];
#pragma unroll
            for (int q = 0; q < kSaoMaxN; ++q) lt[q] = key < K[q];
#pragma unroll
            for (int q = kSaoMaxN - 1; q >= 1; --q)
              if (lt[q]) K[q] = lt[q - 1] ? K[q - 1] : key;
            if (lt[0]) K[0] = key;
#pragma unroll
            for (int q = 0; q < kSaoMaxN; ++q)
              if (q == n - 1) wk = K[q];
          } else {
            if (!lex_less(d2, p.z, wd, wi)) continue;
            near_insert(L, d2, p.z);
#pragma unroll
            for (int q = 0; q < kSaoMaxN; ++q)
              if (q == n - 1) {
                wd = L.d[q];
                wi = L.i[q];
              }
          }
        }
      }
    }
    if (found >= n) {
      // every point not yet seen lies outside the block of cells scanned so
      // far, at least as far as the block's nearest edge inside the grid
      const int64_t inf = INT64_MAX;
      const int64_t dl = ix - r > 0 ? x - (g.x0 + (int64_t)(ix - r) * g.cell) : inf;
      const int64_t dr = ix + r < nx - 1 ? g.x0 + (int64_t)(ix + r + 1) * g.cell - x : inf;
      const int64_t dd = iy - r > 0 ? y - (g.y0 + (int64_t)(iy - r) * g.cell) : inf;
      const int64_t du = iy + r < ny - 1 ? g.y0 + (int64_t)(iy + r + 1) * g.cell - y : inf;
      const int64_t lb = min(min(dl, dr), min(dd, du));
      const uint64_t worst = PACKED ? (wk >> 16) : wd;
      if (lb > kSaoSqrtMax || (uint64_t)(lb * lb) > worst) break;  // a point at lb could still tie
    }
  }
#pragma unroll
  for (int k = 0; k < kSaoMaxN; ++k) out[k] = PACKED ? (int32_t)(K[k] & 0xFFFFu) : L.i[k];
}

struct Polar {
  int32_t dx, dy;
  int32_t label;
};

__device__ inline int half_plane(int32_t dx, int32_t dy) {
  if (dx == 0 && dy == 0) return -1;
  return (dy > 0 || (dy == 0 && dx > 0)) ? 0 : 1;
}

__device__ inline bool angle_less(const Polar& u, const Polar& v) {
  const int hu = half_plane(u.dx, u.dy), hv = half_plane(v.dx, v.dy);
  if (hu != hv) return hu < hv;
  if (hu >= 0) {
    const int64_t cross = (int64_t)u.dx * v.dy - (int64_t)u.dy * v.dx;
    if (cross != 0) return cross > 0;
  }
  // same direction: nearer first (the squared lengths only on this rare path)
  const uint64_t du = (uint64_t)((int64_t)u.dx * u.dx + (int64_t)u.dy * u.dy);
  const uint64_t dv = (uint64_t)((int64_t)v.dx * v.dx + (int64_t)v.dy * v.dy);
  if (du != dv) return du < dv;
  return u.label < v.label;
}

// Sorts the first n entries by angle (odd-even transposition, fixed indices).
__device__ inline void sort_by_angle(Polar (&e)[kSaoMaxN], int n) {
#pragma unroll
  for (int pass = 0; pass < kSaoMaxN; ++pass) {
#pragma unroll
    for (int j = pass & 1; j + 1 < kSaoMaxN; j += 2) {
      if (j + 1 < n && angle_less(e[j + 1], e[j])) {
        const Polar t = e[j];
        e[j] = e[j + 1];
        e[j + 1] = t;
      }
    }
  }
}

// Least Levenshtein distance between a and the rotations of b (length n).
__device__ inline int cyclic_edit_distance(const int32_t (&a)[kSaoMaxN], int32_t (&b)[kSaoMaxN], int n) {
  int best = n;
#pragma unroll 1
  for (int s = 0; s < n; ++s) {
    int row[kSaoMaxN + 1];
#pragma unroll
    for (int j = 0; j <= kSaoMaxN; ++j) row[j] = j;
#pragma unroll
    for (int i = 1; i <= kSaoMaxN; ++i) {
      if (i <= n) {
        int diag = row[0];
        row[0] = i;
#pragma unroll
        for (int j = 1; j <= kSaoMaxN; ++j) {
          if (j <= n) {
            const int up = row[j];
            row[j] = min(min(up + 1, row[j - 1] + 1), diag + (a[i - 1] != b[j - 1] ? 1 : 0));
            diag = up;
          }
        }
      }
    }
    int dist = 0;
#pragma unroll
    for (int j = 0; j <= kSaoMaxN; ++j)
      if (j == n) dist = row[j];
    best = min(best, dist);
    const int32_t first = b[0];  // rotate the first n entries left by one
#pragma unroll
    for (int k = 0; k + 1 < kSaoMaxN; ++k)
      if (k + 1 < n) b[k] = b[k + 1];
      else if (k + 1 == n) b[k] = first;
    if (n == kSaoMaxN) b[kSaoMaxN - 1] = first;
  }
  return best;
}

typedef int32_t v2i __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const v2i gcv2i;
typedef __attribute__((address_space(1))) const int32_t gci32;

__device__ inline int2 ldg_xy(const int32_t* p) {
  const v2i v = *(gcv2i*)p;
  return make_int2(v.x, v.y);
}

__device__ inline int2 xy_at(const int2* xy, int32_t c) {
  return ldg_xy(reinterpret_cast<const int32_t*>(xy + c));
}

// Keypoint of compact match c in image `side` (0 query, 1 db).
__device__ inline int2 point_of(const SaoArgs& a, const SaoPair& P, const int32_t* rows, int side,
                                int32_t c) {
  const int32_t row = *(gci32*)(rows + c);
  if (side == 0) return ldg_xy(P.kq + 2 * (int64_t)row);
  const int32_t m = *(gci32*)(a.match + P.off + row);  // validated during compaction
  return ldg_xy(P.kd + 2 * (int64_t)m);
}

__global__ __launch_bounds__(kSaoBuildWG) void k_sao_build(SaoArgs a) {
  __shared__ int s_tmp[kSaoBuildWaves];
  __shared__ int s_M, s_bad;
  __shared__ int s_red[4][kSaoBuildWaves];
  __shared__ GridInfo s_grid;
  const int p = blockIdx.x;
  const PairScratch S = scratch_at(a, p);
  const SaoPair P = a.pairs[p];
  const int tid = threadIdx.x;
  const int nq = min(max(P.nq, 0), a.n_max);
  if (tid == 0) {
    s_M = 0;
    s_bad = P.nq > a.n_max || P.nq < 0 ? 1 : 0;
  }
  phase_barrier();
  // compaction of the matched rows in row order (and every output starts
  // at -1): each thread counts its own segment of rows, one block scan
  // gives the segments' starts, then each thread writes its rows
  const int seg = (nq + kSaoBuildWG - 1) / kSaoBuildWG;
  const int r0 = min(tid * seg, nq), r1 = min(r0 + seg, nq);
  int mine = 0;
  for (int i = r0; i < r1; ++i) {
    const int32_t m = a.match[P.off + i];
    if (m >= P.nd) s_bad = 1;
    mine += (m >= 0 && m < P.nd) ? 1 : 0;
  }
  int total;
  int pos = block_exclusive<kSaoBuildWaves>(mine, s_tmp, &total);
  for (int i = r0; i < r1; ++i) {
    const int32_t m = a.match[P.off + i];
    a.out[P.off + i] = -1;
    if (a.ced) a.ced[P.off + i] = -1;
    if (m >= 0 && m < P.nd) S.rows[pos++] = i;
  }
  if (tid == 0) s_M = total;
  phase_barrier();
  const int M = s_M;
  // a grid per image
  for (int side = 0; side < 2 && M > 1; ++side) {
    int xmin = INT32_MAX, ymin = INT32_MAX, xmax = INT32_MIN, ymax = INT32_MIN;
    for (int c = tid; c < M; c += kSaoBuildWG) {
      const int2 q = point_of(a, P, S.rows, side, c);
      S.xy[side][c] = q;
      if (q.x <= -kSaoCoordLimit || q.x >= kSaoCoordLimit || q.y <= -kSaoCoordLimit || q.y >= kSaoCoordLimit)
        s_bad = 1;
      xmin = min(xmin, q.x);
      ymin = min(ymin, q.y);
      xmax = max(xmax, q.x);
      ymax = max(ymax, q.y);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      xmin = min(xmin, __shfl_xor(xmin, d));
      ymin = min(ymin, __shfl_xor(ymin, d));
      xmax = max(xmax, __shfl_xor(xmax, d));
      ymax = max(ymax, __shfl_xor(ymax, d));
    }
    if (__lane_id() == 0) {
      s_red[0][tid >> 6] = xmin;
      s_red[1][tid >> 6] = ymin;
      s_red[2][tid >> 6] = xmax;
      s_red[3][tid >> 6] = ymax;
    }
    phase_barrier();
    if (tid == 0) {
      int64_t x0 = INT32_MAX, y0 = INT32_MAX, x1 = INT32_MIN, y1 = INT32_MIN;
      for (int w = 0; w < kSaoBuildWaves; ++w) {
        x0 = min(x0, (int64_t)s_red[0][w]);
        y0 = min(y0, (int64_t)s_red[1][w]);
        x1 = max(x1, (int64_t)s_red[2][w]);
        y1 = max(y1, (int64_t)s_red[3][w]);
      }
      const double w = double(x1 - x0) + 1.0, h = double(y1 - y0) + 1.0;
      int64_t cell = max(int64_t(1), (int64_t)ceil(sqrt(w * h * kSaoPointsPerCell / double(M))));
      int64_t nx, ny;
      for (;;) {  // at most 4 M + 64 cells, so the cell array always fits
        nx = (x1 - x0) / cell + 1;
        ny = (y1 - y0) / cell + 1;
        if ((double)nx * (double)ny <= 4.0 * (double)M + 64.0) break;
        cell *= 2;
      }
      s_grid = GridInfo{x0, y0, cell, nx, ny};
      S.info->g[side] = s_grid;
    }
    phase_barrier();
    const GridInfo g = s_grid;
    const int64_t ncell = g.nx * g.ny;
    int32_t* cell = S.cell[side];
    for (int64_t k = tid; k <= ncell; k += kSaoBuildWG) cell[k] = 0;
    phase_barrier();
    for (int c = tid; c < M; c += kSaoBuildWG) {
      const int2 q = S.xy[side][c];
      const int64_t cx = min(max(((int64_t)q.x - g.x0) / g.cell, int64_t(0)), g.nx - 1);
      const int64_t cy = min(max(((int64_t)q.y - g.y0) / g.cell, int64_t(0)), g.ny - 1);
      atomicAdd(&cell[cy * g.nx + cx], 1);
    }
    phase_barrier();
    int run = 0;  // exclusive scan: cell[k] = first slot of cell k
    for (int64_t base = 0; base < ncell; base += kSaoBuildWG) {
      const int64_t k = base + tid;
      const int v = k < ncell ? cell[k] : 0;
      int total;
      const int ex = block_exclusive<kSaoBuildWaves>(v, s_tmp, &total);
      if (k < ncell) cell[k] = run + ex;
      run += total;
    }
    phase_barrier();
    // scatter; afterwards cell[k] is the end of cell k (the start of k + 1)
    int4* pts = S.pts[side];
    for (int c = tid; c < M; c += kSaoBuildWG) {
      const int2 q = S.xy[side][c];
      const int64_t cx = min(max(((int64_t)q.x - g.x0) / g.cell, int64_t(0)), g.nx - 1);
      const int64_t cy = min(max(((int64_t)q.y - g.y0) / g.cell, int64_t(0)), g.ny - 1);
      const int32_t slot = atomicAdd(&cell[cy * g.nx + cx], 1);
      pts[min(max(slot, 0), M - 1)] = make_int4(q.x, q.y, c, 0);
    }
    phase_barrier();
  }
  if (tid == 0) {
    S.info->M = M;
    S.info->bad = s_bad;
    if (s_bad) atomicAdd(a.errors, 1);
  }
}

__global__ __launch_bounds__(kSaoWG) void k_sao_search(SaoArgs a) {
  const int p = blockIdx.y;
  const PairScratch S = scratch_at(a, p);
  const int M = S.info->M;
  if ((int)(blockIdx.x * kSaoWG) >= M || S.info->bad) return;  // uniform over the work-group
  // threads take the matches in the query image's cell order, so the lanes
  // of a wavefront search neighbouring cells (one match: no grid, row order)
  const int32_t t = (int32_t)(blockIdx.x * kSaoWG + threadIdx.x);
  const bool active = t < M;
  const int32_t c = !active ? 0 : M > 1 ? min(max(S.pts[0][t].z, 0), M - 1) : t;
  const SaoPair P = a.pairs[p];
  const int n = min(a.nn, M - 1);
  int dist = 0;
  if (n > 0) {
    int32_t lab[2][kSaoMaxN];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const GridInfo g = S.info->g[side];
      if (active) {
        const int2 o = xy_at(S.xy[side], c);  // n > 0: M > 1, so the build wrote xy
        int32_t nn_idx[kSaoMaxN];
        const GlobalGrid G{S.cell[side], S.pts[side]};
        // packed keys when every coordinate difference is below 2^23
        if (g.nx * g.cell < (int64_t(1) << 23) && g.ny * g.cell < (int64_t(1) << 23) && M <= 65536)
          ring_search<true>(G, g, o.x, o.y, c, n, nn_idx);
        else
          ring_search<false>(G, g, o.x, o.y, c, n, nn_idx);
        Polar e[kSaoMaxN];
#pragma unroll
        for (int k = 0; k < kSaoMaxN; ++k) {
          const int32_t nb = k < n ? min(max(nn_idx[k], 0), M - 1) : c;
          const int2 q = xy_at(S.xy[side], nb);
          e[k] = Polar{q.x - o.x, q.y - o.y, nb};
        }
        sort_by_angle(e, n);
#pragma unroll
        for (int k = 0; k < kSaoMaxN; ++k) lab[side][k] = e[k].label;
      }
    }
    if (active) dist = cyclic_edit_distance(lab[0], lab[1], n);
  }
  if (active) {
    const int32_t row = S.rows[c];
    const int32_t m = a.match[P.off + row];
    if ((int64_t)dist * a.den <= (int64_t)a.num * n) a.out[P.off + row] = m;
    if (a.ced) a.ced[P.off + row] = dist;
  }
}

}  // namespace

uint64_t sao_work_bytes(int32_t n_pairs, int32_t max_rows) {
  const int64_t B = std::min<int64_t>(std::max(n_pairs, 1), kSaoBatch);
  return 256 + round16(sizeof(SaoPair) * (uint64_t)std::max(n_pairs, 1)) +
         (uint64_t)B * pair_scratch_bytes(std::max(max_rows, 1));
}

hipError_t sao_upload(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                      const int32_t* h_n_feats, const int64_t* h_starts, void* d_work, hipStream_t s) {
  std::vector<SaoPair> hp((size_t)n_pairs);
  for (int32_t p = 0; p < n_pairs; ++p) {
    const int32_t q = h_pairs[2 * p], d = h_pairs[2 * p + 1];
    hp[(size_t)p] = SaoPair{d_kp[q], d_kp[d], h_n_feats[q], h_n_feats[d], h_starts[p]};
  }
  SaoPair* dp = reinterpret_cast<SaoPair*>(static_cast<uint8_t*>(d_work) + 256);
  hipError_t e = hipSuccess;
  if (n_pairs > 0) e = hipMemcpyAsync(dp, hp.data(), sizeof(SaoPair) * hp.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // hp is freed on return
  return e;
}

hipError_t sao_run(int32_t first, int32_t count, int32_t table_pairs, int32_t n_max, const int32_t* d_match,
                   int32_t nn, int32_t num, int32_t den, int32_t* d_out, int32_t* d_ced, void* d_work,
                   hipStream_t s) {
  uint8_t* w = static_cast<uint8_t*>(d_work);
  SaoPair* dp = reinterpret_cast<SaoPair*>(w + 256);
  SaoArgs a;
  a.n_max = std::max(n_max, 1);
  a.match = d_match;
  a.out = d_out;
  a.ced = d_ced;
  a.nn = nn;
  a.num = num;
  a.den = den;
  a.scratch = w + 256 + round16(sizeof(SaoPair) * (uint64_t)table_pairs);
  a.scratch_bytes = pair_scratch_bytes(a.n_max);
  a.errors = reinterpret_cast<int32_t*>(w);
  const unsigned chunks = (unsigned)((a.n_max + kSaoWG - 1) / kSaoWG);
  for (int32_t b0 = 0; b0 < count; b0 += kSaoBatch) {
    a.pairs = dp + first + b0;
    a.n_pairs = std::min(kSaoBatch, count - b0);
    hipLaunchKernelGGL(k_sao_build, dim3(a.n_pairs), dim3(kSaoBuildWG), 0, s, a);
    hipLaunchKernelGGL(k_sao_search, dim3(chunks, a.n_pairs), dim3(kSaoWG), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sao(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                      const int32_t* h_n_feats, const int64_t* h_offs, const int32_t* d_match, int32_t nn,
                      int32_t num, int32_t den, int32_t* d_out, int32_t* d_ced, void* d_work, bool clear_errors,
                      hipStream_t s) {
  int32_t n_max = 1;
  for (int32_t p = 0; p < n_pairs; ++p) n_max = std::max(n_max, h_n_feats[h_pairs[2 * p]]);
  hipError_t e = clear_errors ? launch_fill_u32(static_cast<uint32_t*>(d_work), 0u, 1, s) : hipSuccess;
  if (e == hipSuccess) e = sao_upload(n_pairs, h_pairs, d_kp, h_n_feats, h_offs, d_work, s);
  if (e == hipSuccess) e = sao_run(0, n_pairs, n_pairs, n_max, d_match, nn, num, den, d_out, d_ced, d_work, s);
  return e;
}

}  // namespace chm

extern "C" chm_status chm_sao_work_bytes(int32_t n_pairs, int32_t max_query_rows, uint64_t* out_bytes) {
  chm::clear_error();
  if (!out_bytes || n_pairs < 0 || max_query_rows < 0) return chm::fail(CHM_E_INVALID_ARG, "bad arguments");
  *out_bytes = chm::sao_work_bytes(n_pairs, max_query_rows);
  return CHM_OK;
}

extern "C" chm_status chm_sao_filter_device(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* d_kp,
                                            const int32_t* h_n_feats, int32_t n_images, const int64_t* h_offs,
                                            const int32_t* d_match, int32_t n_neighbors, int32_t score_num,
                                            int32_t score_den, int32_t* d_out, int32_t* d_ced, void* d_work,
                                            uint64_t work_bytes, void* stream) {
  using namespace chm;
  clear_error();
  if (n_pairs < 0 || n_images < 0) return fail(CHM_E_INVALID_ARG, "negative count");
  if (n_pairs == 0) return CHM_OK;
  if (!h_pairs || !d_kp || !h_n_feats || !h_offs || !d_match || !d_out || !d_work)
    return fail(CHM_E_INVALID_ARG, "NULL array");
  if (n_neighbors < 1 || n_neighbors > kSaoMaxN)
    return fail(CHM_E_INVALID_ARG, "n_neighbors must be 1..%d on the device", kSaoMaxN);
  if (score_num < 0 || score_den <= 0) return fail(CHM_E_INVALID_ARG, "bad score threshold");
  if (d_out == d_match || (d_ced && (const int32_t*)d_ced == d_match))
    return fail(CHM_E_INVALID_ARG, "d_out and d_ced must not be d_match");
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
  const uint64_t need = sao_work_bytes(n_pairs, n_max);
  if (work_bytes < need)
    return fail(CHM_E_CAPACITY, "work buffer holds %llu bytes, %llu needed", (unsigned long long)work_bytes,
                (unsigned long long)need);
  const hipError_t e = launch_sao(n_pairs, h_pairs, d_kp, h_n_feats, h_offs, d_match, n_neighbors, score_num,
                                  score_den, d_out, d_ced, d_work, true, (hipStream_t)stream);
  if (e != hipSuccess) return fail(CHM_E_HIP, "SAO launch failed: %s", hipGetErrorString(e));
  return CHM_OK;
}

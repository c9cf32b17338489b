/*
 * Plain CPU oracle for cascade-hashing feature matching.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load, link or
 * call this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the HIP
 * library.
 *
 * It follows the four steps of cascade hashing as the paper states them in
 * Sec. 2.3.1 (hashing lookup with L tables of 2^m buckets, remapping to n-bit
 * codes and Hamming distances, ranking to the top K, Euclidean distance and
 * ratio test), with these readings where the text is silent:
 *   - the LSH family is the sign of a random projection of the centred
 *     descriptor x - mu; rows 0..n-1 give the long code, rows n + m*t .. give
 *     the m bits of bucket table t (independent rows);
 *   - projections are evaluated exactly (fp64 is exact for bf16 weights of
 *     magnitude in [2^-16, 32) or zero times integers in [-255, 255]);
 *   - bit = 1 iff the projection is > 0 (a zero projection gives bit 0);
 *   - bit r of the code sits in word r/32 at position r%32; bit j of a bucket
 *     id comes from row n + m*t + j at position j (least significant first);
 *   - the candidates of a query are the SET union over tables of the db
 *     points sharing its bucket;
 *   - the top K are the min(K, |C|) candidates with the smallest
 *     (Hamming distance, db index) pairs in lexicographic order; with
 *     `whole` set (the other reading of "until K are returned") every
 *     candidate as close as the K-th in Hamming distance is re-ranked too;
 *   - the ratio test dis(q1) < t_r * dis(q2) is taken on squared integer
 *     distances with t_r = a/b as b^2 d1 < a^2 d2; fewer than two candidates
 *     means no match, unless `single` is set: then a lone candidate has an
 *     infinite second distance and is accepted (the other reading).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_DIM 128
#define ORC_CODE_BITS 128
#define ORC_CODE_WORDS 4

typedef struct orc_image {
  const uint8_t *desc;      /* n x 128 */
  const uint32_t *codes;    /* n x 4 */
  const uint8_t *ids;       /* n x L */
  const int32_t *offsets;   /* L x (2^m + 1) */
  const int32_t *members;   /* L x n */
  int64_t n;
} orc_image;

static double bf16_value(uint16_t bits) {
  uint32_t u = (uint32_t)bits << 16;
  float f;
  memcpy(&f, &u, sizeof f);
  return (double)f;
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Projection of every descriptor onto every row: p_r(x) = sum_d W[r][d] (x_d - mu_d).
 * Sec. 2.3.1 steps (1)-(2): the LSH functions behind both the short and the long codes. */
void orc_project(const uint8_t *X, int64_t n, const uint16_t *W, int32_t R,
                 const uint8_t *mu, double *P) {
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < n; ++i) {
    for (int r = 0; r < R; ++r) {
      double s = 0.0;
      for (int d = 0; d < ORC_DIM; ++d)
        s += bf16_value(W[(int64_t)r * ORC_DIM + d]) * (double)((int)X[i * ORC_DIM + d] - (int)mu[d]);
      P[i * R + r] = s;
    }
  }
}

/* Codes and bucket ids of one image (steps (1)-(2) of Sec. 2.3.1). */
void orc_hash(const uint8_t *X, int64_t n, const uint16_t *W, const uint8_t *mu,
              int32_t L, int32_t m, uint32_t *codes, uint8_t *ids) {
  const int R = ORC_CODE_BITS + L * m;
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < n; ++i) {
    double p[ORC_CODE_BITS + 8 * 8];
    for (int r = 0; r < R; ++r) {
      double s = 0.0;
      for (int d = 0; d < ORC_DIM; ++d)
        s += bf16_value(W[(int64_t)r * ORC_DIM + d]) * (double)((int)X[i * ORC_DIM + d] - (int)mu[d]);
      p[r] = s;
    }
    for (int w = 0; w < ORC_CODE_WORDS; ++w) {
      uint32_t word = 0;
      for (int k = 0; k < 32; ++k)
        if (p[32 * w + k] > 0.0) word |= (uint32_t)1 << k;
      codes[i * ORC_CODE_WORDS + w] = word;
    }
    for (int t = 0; t < L; ++t) {
      int b = 0;
      for (int j = 0; j < m; ++j)
        if (p[ORC_CODE_BITS + m * t + j] > 0.0) b |= 1 << j;
      ids[i * L + t] = (uint8_t)b;
    }
  }
}

/* Lookup tables of step (1): for each table, 2^m buckets listing the points
 * whose bucket id is that bucket, in ascending index order. */
void orc_tables(const uint8_t *ids, int64_t n, int32_t L, int32_t m,
                int32_t *offsets, int32_t *members) {
  const int nb = 1 << m;
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
  for (int t = 0; t < L; ++t) {
    int32_t *off = offsets + (int64_t)t * (nb + 1);
    for (int b = 0; b <= nb; ++b) off[b] = 0;
    for (int64_t i = 0; i < n; ++i) off[ids[i * L + t] + 1] += 1;
    for (int b = 0; b < nb; ++b) off[b + 1] += off[b];
    for (int b = 0; b < nb; ++b) fill[b] = off[b];
    for (int64_t i = 0; i < n; ++i) {
      int b = ids[i * L + t];
      members[(int64_t)t * n + fill[b]] = (int32_t)i;
      fill[b] += 1;
    }
  }
  free(fill);
}

typedef struct cand { int32_t h; int32_t j; } cand;

static int cand_less(const void *pa, const void *pb) {
  const cand *a = (const cand *)pa, *b = (const cand *)pb;
  if (a->h != b->h) return a->h < b->h ? -1 : 1;
  if (a->j != b->j) return a->j < b->j ? -1 : 1;
  return 0;
}

static int hamming(const uint32_t *a, const uint32_t *b) {
  int h = 0;
  for (int w = 0; w < ORC_CODE_WORDS; ++w) h += __builtin_popcount(a[w] ^ b[w]);
  return h;
}

static int64_t sq_euclid(const uint8_t *x, const uint8_t *y) {
  int64_t e = 0;
  for (int d = 0; d < ORC_DIM; ++d) {
    int64_t diff = (int64_t)x[d] - (int64_t)y[d];
    e += diff * diff;
  }
  return e;
}

/* Steps (1)-(4) of Sec. 2.3.1 for every query of image q against db image d.
 * out[i] = matched db index or -1; topk (optional, nq x K) = keys h<<24 | j of the
 * ranked candidates, 0xFFFFFFFF where fewer than K exist.  Returns the number of
 * (unique) candidates evaluated. */
static int64_t match_pair_impl(const orc_image *q, const orc_image *d, int L, int m, int K,
                               int ra, int rb, int single, int whole, int32_t *out, uint32_t *topk,
                               int32_t *stamp, cand *buf) {
  const int nb = 1 << m;
  int64_t total = 0;
  for (int64_t j = 0; j < d->n; ++j) stamp[j] = -1;
  for (int64_t i = 0; i < q->n; ++i) {
    /* (1) candidates: union over tables of the query's bucket in image d */
    int64_t nc = 0;
    for (int t = 0; t < L; ++t) {
      int b = q->ids[i * L + t];
      const int32_t *off = d->offsets + (int64_t)t * (nb + 1);
      for (int32_t s = off[b]; s < off[b + 1]; ++s) {
        int32_t j = d->members[(int64_t)t * d->n + s];
        if (stamp[j] != (int32_t)i) {
          stamp[j] = (int32_t)i;
          buf[nc].j = j;
          /* (2) Hamming distance of the long codes */
          buf[nc].h = hamming(q->codes + i * ORC_CODE_WORDS, d->codes + (int64_t)j * ORC_CODE_WORDS);
          ++nc;
        }
      }
    }
    total += nc;
    /* (3) rank by Hamming distance, ties by db index, keep the first K */
    qsort(buf, (size_t)nc, sizeof(cand), cand_less);
    int64_t nt = nc < K ? nc : K;
    if (topk) {
      for (int k = 0; k < K; ++k)
        topk[i * K + k] = k < nt ? ((uint32_t)buf[k].h << 24) | (uint32_t)buf[k].j : 0xFFFFFFFFu;
    }
    /* (4) Euclidean re-rank of the top K (or of every candidate within the
       K-th's Hamming distance) and ratio test */
    if (whole && nt > 0)
      while (nt < nc && buf[nt].h == buf[nt - 1].h) ++nt;
    if (nt < 2) { out[i] = (nt == 1 && single) ? buf[0].j : -1; continue; }
    int64_t d1 = -1, d2 = -1;
    int32_t j1 = -1;
    for (int64_t k = 0; k < nt; ++k) {
      int64_t e = sq_euclid(q->desc + i * ORC_DIM, d->desc + (int64_t)buf[k].j * ORC_DIM);
      if (d1 < 0 || e < d1) { d2 = d1; d1 = e; j1 = buf[k].j; }
      else if (d2 < 0 || e < d2) { d2 = e; }
    }
    out[i] = ((int64_t)rb * rb * d1 < (int64_t)ra * ra * d2) ? j1 : -1;
  }
  return total;
}

int64_t orc_match_pair(const orc_image *q, const orc_image *d, int32_t L, int32_t m, int32_t K,
                       int32_t ra, int32_t rb, int32_t single, int32_t whole, int32_t *out,
                       uint32_t *topk) {
  int32_t *stamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d->n > 0 ? d->n : 1));
  cand *buf = (cand *)malloc(sizeof(cand) * (size_t)(d->n > 0 ? d->n : 1));
  int64_t c = match_pair_impl(q, d, L, m, K, ra, rb, single, whole, out, topk, stamp, buf);
  free(stamp);
  free(buf);
  return c;
}

/* Every directed pair (pairs[2p], pairs[2p+1]) of a pair list; results of pair p at
 * out + out_offsets[p].  Pairs run in parallel; each pair is the plain loop above.
 * Returns the total number of candidates evaluated. */
int64_t orc_match_pairs(const orc_image *images, const int32_t *pairs, int64_t P,
                        const int64_t *out_offsets, int32_t L, int32_t m, int32_t K,
                        int32_t ra, int32_t rb, int32_t single, int32_t whole, int32_t *out,
                        uint32_t *topk) {
  int64_t nmax = 1;
  for (int64_t p = 0; p < P; ++p) {
    int64_t nd = images[pairs[2 * p + 1]].n;
    if (nd > nmax) nmax = nd;
  }
  int64_t total = 0;
#pragma omp parallel reduction(+ : total)
  {
    int32_t *stamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)nmax);
    cand *buf = (cand *)malloc(sizeof(cand) * (size_t)nmax);
    int64_t p;
#pragma omp for schedule(dynamic, 1)
    for (p = 0; p < P; ++p) {
      total += match_pair_impl(&images[pairs[2 * p]], &images[pairs[2 * p + 1]], L, m, K, ra, rb, single, whole,
                               out + out_offsets[p],
                               topk ? topk + out_offsets[p] * K : NULL, stamp, buf);
    }
    free(stamp);
    free(buf);
  }
  return total;
}

/* Exhaustive nearest-neighbour matching with the same ratio test: d1 <= d2 are
 * the two smallest squared distances over every db descriptor, j1 the first
 * index reaching d1. */
void orc_bruteforce(const uint8_t *Xq, int64_t nq, const uint8_t *Xd, int64_t nd,
                    int32_t ra, int32_t rb, int32_t *out) {
  int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
  for (i = 0; i < nq; ++i) {
    int64_t d1 = -1, d2 = -1;
    int32_t j1 = -1;
    for (int64_t j = 0; j < nd; ++j) {
      int64_t e = sq_euclid(Xq + i * ORC_DIM, Xd + j * ORC_DIM);
      if (d1 < 0 || e < d1) { d2 = d1; d1 = e; j1 = (int32_t)j; }
      else if (d2 < 0 || e < d2) { d2 = e; }
    }
    if (nd < 2) { out[i] = -1; continue; }
    out[i] = ((int64_t)rb * rb * d1 < (int64_t)ra * ra * d2) ? j1 : -1;
  }
}

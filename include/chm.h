/*
 * chm.h -- C-ABI of the MI355X (gfx950) cascade-hashing feature matcher.
 *
 * The library implements, as hand-written HIP kernels, cascade-hashing
 * matching of image pairs (paper Sec. 2.3.1, steps (1)-(4)): sign-of-random-
 * projection codes of n = 128 bits and L tables of 2^m buckets per image,
 * same-bucket candidate lookup, Hamming ranking to the top K, exact integer
 * Euclidean re-rank of those K and the ratio test; the block-row pipeline of
 * Sec. 2.3.2 (load descriptors and build codes/tables on load, match the
 * pairs of a block, free what the next block row no longer needs); and the
 * host-side MBR block schedule of Sec. 2.2 with GPS ordering (Appendix A).
 *
 * Conventions shared by every call:
 *  - Descriptors are 128-d uint8 rows (SIFT, Sec. 2.4), row-major, 128 B each.
 *  - "d_" pointers are device (HBM) pointers, "h_" pointers are host pointers.
 *    Device memory is owned by the caller: the library never allocates device
 *    memory, it sub-allocates inside the arena the caller hands to
 *    chm_store_create.  Streams are passed as void* (a hipStream_t; NULL is
 *    the null stream).  Work is enqueued on the given stream; host arrays are
 *    only read during the call.
 *  - Every call returns a chm_status (0 = CHM_OK).  On error, outputs are
 *    unspecified and chm_last_error() returns a message for the calling
 *    thread.  HIP runtime failures map to CHM_E_HIP; asynchronous kernel
 *    faults surface at a later call or at stream synchronisation.
 *  - Results never depend on the match mode, the stream, the tuning or the
 *    schedule: they are the unique output of the method as specified below.
 */
#ifndef CHM_H
#define CHM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHM_ABI_VERSION 2
#define CHM_DIM 128       /* descriptor dimension (SIFT) */
#define CHM_CODE_BITS 128 /* n, bits of the long code (Sec. 2.3.1 step (2), n = 128) */
#define CHM_MAX_FEATS 65535

typedef enum chm_status {
  CHM_OK = 0,
  CHM_E_INVALID_ARG = -1,  /* a size, pointer or parameter is out of range */
  CHM_E_UNSUPPORTED = -2,  /* a valid request the library does not support */
  CHM_E_CAPACITY = -3,     /* the arena (or a cap) cannot hold what was asked */
  CHM_E_NOT_RESIDENT = -4, /* a pair names an image that is not loaded */
  CHM_E_HIP = -5,          /* a HIP runtime call failed */
  CHM_E_INTERNAL = -6
} chm_status;

enum { CHM_PROJ_BF16 = 0, CHM_PROJ_FP32 = 1 };
enum { CHM_MATCH_PLAIN = 0, CHM_MATCH_BATCHED = 1 };

/* Parameters of cascade hashing (Sec. 2.3.1; defaults in the paper:
 * L = 6, m = 8, n = 128, K = 8; ratio threshold t_r, Sec. 3.2). */
typedef struct chm_config {
  uint32_t abi_version;   /* must be CHM_ABI_VERSION */
  int32_t num_tables;     /* L, 1..8 */
  int32_t bucket_bits;    /* m, 0..8 (0 = one bucket: every db point is a candidate) */
  int32_t top_k;          /* K, 1..32: candidates kept by Hamming ranking */
  int32_t ratio_num;      /* t_r = ratio_num / ratio_den, 0 < num <= den <= 46340 */
  int32_t ratio_den;
  int32_t proj_precision; /* CHM_PROJ_BF16 or CHM_PROJ_FP32 (MFMA input type) */
  int32_t flags;          /* CHM_ACCEPT_SINGLE | CHM_WHOLE_LAST_BUCKET, or 0 */
  double fixup_rel;       /* a projection p_r(x) = W_r.x - c_r (c_r = W_r.mu) is
                             recomputed in fp64 when its fp32 value v has
                             |v| < fixup_rel * (||W_r||_2 * ||x||_2 + |c_r|);
                             must lie in [1e-4, 0.5].  The fp32 sum of the
                             128 exact products minus c_r errs by at most
                             127 * 2^-24 * (||W_r||_2 ||x||_2 + |c_r|) (twice
                             that if the accumulator truncated), so every
                             value in the range keeps every bit exact; 1e-4
                             (the default) recomputes the fewest */
} chm_config;

/* Flag of chm_config.flags.  The ratio test needs a second candidate; by
 * default a query with a single candidate gets no match.  With this flag its
 * second distance counts as infinite and the single candidate is accepted
 * (the other reading of Sec. 2.3.1 step (4)). */
#define CHM_ACCEPT_SINGLE 1
/* Flag of chm_config.flags.  Step (3) keeps the first K candidates in
 * (Hamming distance, db index) order; with this flag every candidate as
 * close in Hamming distance as the K-th is re-ranked as well (the other
 * reading of checking buckets until K are returned).  The top-K keys
 * written by a plan are the first K either way. */
#define CHM_WHOLE_LAST_BUCKET 2

/* Fills *cfg with the paper's defaults (L=6, m=8, K=8, t_r=4/5, BF16, 1e-4). */
void chm_config_default(chm_config *cfg);

/* Message of the last failing call on this thread ("" if none). */
const char *chm_last_error(void);

/* ABI version of the loaded library (CHM_ABI_VERSION it was built with). */
int32_t chm_abi_version(void);

/* Test hook for the CHM_E_HIP error path: the n-th HIP runtime call the
 * library checks on the calling thread after this call (n >= 1) is not
 * made and reports a failure, so the entry point making it returns
 * CHM_E_HIP (its outputs are then unspecified, as for any error); n = 0
 * cancels a pending failure.  Later calls run normally. */
void chm_debug_fail_hip(int32_t n);

/* ------------------------------------------------------------------ store
 * A store keeps images resident in a caller-owned device arena: the raw
 * descriptors and everything step (1)-(2) of Sec. 2.3.1 builds for them
 * (long codes, bucket ids, lookup tables), as Sec. 2.3.2 step (1) loads a
 * block's descriptors and computes their codes and bucket ids on load.
 */
typedef struct chm_store chm_store;

/* Bytes of arena one image of n_feats descriptors occupies (descriptors,
 * codes, bucket ids, norms, tables; 256-byte aligned sections). */
chm_status chm_image_bytes(const chm_config *cfg, int32_t n_feats, uint64_t *out_bytes);

/* Bytes of arena the store itself needs (projection matrix, counters). */
chm_status chm_store_overhead_bytes(const chm_config *cfg, uint64_t *out_bytes);

/* Creates a store.
 *   cfg      : parameters (copied).
 *   h_W      : host, (128 + L*m) x 128 bfloat16 bit patterns, row r is the
 *              r-th random projection (rows 0..127 the long code, row
 *              128 + m*t + j bit j of table t's bucket id).  Every value must
 *              be 0 or of magnitude in [2^-16, 32) (the fp64 recompute is then
 *              exact); otherwise CHM_E_INVALID_ARG.
 *   h_mu     : host, 128 uint8, the centring vector subtracted before projection.
 *   d_arena  : device, 256-byte aligned, arena_bytes long, owned by the caller
 *              and not touched by anyone else while the store lives.
 *   out      : receives the store.  The store copies W and mu into the arena
 *              (enqueued on the null stream and completed before returning). */
chm_status chm_store_create(const chm_config *cfg, const uint16_t *h_W, const uint8_t *h_mu,
                            void *d_arena, uint64_t arena_bytes, chm_store **out);

/* Destroys a store (synchronises the device first).  NULL is ignored. */
void chm_store_destroy(chm_store *store);

/* Loads `count` images (Sec. 2.3.2 step (1), Algorithm 1 "load"): copies each
 * image's descriptors into the arena (host->device if descs_on_device == 0,
 * device->device otherwise) and builds its long codes, bucket ids and
 * lookup tables, with batched kernel launches for all images of the call.
 *   image_ids : host, count distinct ids >= 0 not already resident.
 *   descs     : host array of count pointers to n_feats[i] x 128 uint8 rows
 *               (host memory should be pinned for an asynchronous copy).
 *   n_feats   : host, 0..CHM_MAX_FEATS each.
 * Errors: CHM_E_INVALID_ARG (duplicates, resident ids, bad sizes),
 * CHM_E_CAPACITY (arena full; nothing of the call is loaded). */
chm_status chm_store_load(chm_store *store, int32_t count, const int32_t *image_ids,
                          const void *const *descs, const int32_t *n_feats,
                          int32_t descs_on_device, void *stream);

/* Rebuilds codes, bucket ids and tables of resident images from their
 * descriptors (the hashing stage alone).  CHM_E_NOT_RESIDENT if one is not. */
chm_status chm_store_rehash(chm_store *store, int32_t count, const int32_t *image_ids,
                            void *stream);

/* Frees resident images (Algorithm 1 "free"); their arena space is reused by
 * later work on the same stream.  Plans that use them become invalid. */
chm_status chm_store_evict(chm_store *store, int32_t count, const int32_t *image_ids);

/* n_feats of a resident image, or -1 in *out if it is not resident. */
chm_status chm_store_image_feats(const chm_store *store, int32_t image_id, int32_t *out);

typedef struct chm_stats {
  uint64_t h2d_bytes;        /* descriptor bytes copied host -> device */
  uint64_t d2d_bytes;        /* descriptor bytes copied device -> device */
  uint64_t resident_bytes;   /* arena bytes held by resident images now */
  uint64_t resident_peak;    /* maximum of resident_bytes so far */
  uint64_t fixups;           /* projections recomputed in fp64 (synchronises) */
  int64_t images_loaded;
  int64_t images_evicted;
  int32_t resident_images;
  int32_t reserved;
  uint64_t fixup_flips;      /* recomputed projections whose bit the MFMA sign had wrong */
} chm_stats;

chm_status chm_store_stats(chm_store *store, chm_stats *out);

/* Copies an image's internal arrays to caller device buffers (for tests):
 *   d_codes   : n x 4 uint32 (bit r of the long code in word r/32, bit r%32)
 *   d_ids     : L x n uint8, table-major: bucket id of each descriptor in
 *               table t, bit j of it from projection row 128 + m*t + j
 *   d_offsets : L x (2^m + 1) int32, bucket b of table t holds
 *               members[t][offsets[t][b] .. offsets[t][b+1])
 *   d_members : L x n uint16 db indices, ascending inside each bucket
 *   d_norms   : n uint32, squared norm of each descriptor
 * Any pointer may be NULL to skip that array.  offsets and members are the
 * plain tables of Sec. 2.3.1 step (1); the device keeps each bucket padded to
 * a multiple of 8 entries, so asking for either synchronises the stream and
 * stages them through host memory (CHM_E_INTERNAL if the device tables are
 * inconsistent). */
chm_status chm_debug_image(chm_store *store, int32_t image_id, uint32_t *d_codes, uint8_t *d_ids,
                           int32_t *d_offsets, uint16_t *d_members, uint32_t *d_norms,
                           void *stream);

/* ------------------------------------------------------------------ matching
 * Steps (1)-(4) of Sec. 2.3.1 for directed pairs (query image q, db image d):
 * for every descriptor x_i of q, the candidates are the set union over the L
 * tables of d's points in x_i's bucket; they are ranked by (Hamming distance
 * of the long codes, db index) and the first min(K, |C_i|) are kept; their
 * squared Euclidean distances are computed exactly in integers; with d1 <= d2
 * the two smallest and j1 the db index reaching d1, the output is j1 if
 * ratio_den^2 * d1 < ratio_num^2 * d2 and -1 otherwise (also -1 when fewer
 * than two candidates exist).
 */
typedef struct chm_plan chm_plan;

/* Builds an executable plan for a pair list.
 *   h_pairs       : host, n_pairs x 2 int32 (query image, db image), both
 *                   resident (else CHM_E_NOT_RESIDENT); self pairs allowed.
 *   h_out_offsets : host, n_pairs + 1 int64; pair p writes its n_q results to
 *                   d_out[h_out_offsets[p] .. h_out_offsets[p+1]) which must
 *                   have exactly n_q elements (else CHM_E_INVALID_ARG).
 *   d_out         : device int32 output (db index or -1 per query descriptor).
 *   d_topk        : device, NULL or K uint32 per output element: the ranked
 *                   candidates as keys (hamming << 24) | db_index, 0xFFFFFFFF
 *                   where fewer than K candidates exist (for tests).
 *   mode          : CHM_MATCH_PLAIN (one launch per pair, host loop) or
 *                   CHM_MATCH_BATCHED (all pairs in one persistent launch
 *                   replayed from a captured HIP graph).
 * The plan keeps its work list in the arena (CHM_E_CAPACITY if full) and
 * stays valid until one of its images is evicted or the plan is destroyed. */
chm_status chm_plan_create(chm_store *store, const int32_t *h_pairs, int32_t n_pairs,
                           const int64_t *h_out_offsets, int32_t *d_out, uint32_t *d_topk,
                           int32_t mode, void *stream, chm_plan **out);

/* Enqueues the plan's matching on `stream`.  CHM_E_NOT_RESIDENT if an image
 * of the plan was evicted since the plan was built. */
chm_status chm_plan_execute(chm_plan *plan, void *stream);

/* Frees the plan (synchronises the streams it ran on).  NULL is ignored. */
void chm_plan_destroy(chm_plan *plan);

/* One-shot matching: create + execute + destroy (synchronous). */
chm_status chm_match_pairs(chm_store *store, const int32_t *h_pairs, int32_t n_pairs,
                           const int64_t *h_out_offsets, int32_t *d_out, int32_t mode,
                           void *stream);

/* Launch-shape tuning of the match kernels (chosen by the autotuner; any
 * valid value gives identical results). */
typedef struct chm_tuning {
  int32_t queries_per_item; /* queries per batched work item, multiple of 64,
                               64..8192 (default 2048).  Batched plans shrink
                               items where a larger one would not sort in LDS,
                               cap them at 512 in launches that stage no db
                               image, and halve those ending each XCD bin's
                               work. */
  int32_t wg_threads;       /* 256 or 1024 */
  int32_t lds_codes;        /* 1: stage the db image's codes in LDS when they fit */
  int32_t grid_per_cu;      /* persistent work-groups per compute unit when no db
                               image of a batched plan is staged in LDS, 1..8 (a
                               launch that stages runs one per compute unit) */
  int32_t match_kernel;     /* batched plans: CHM_KERNEL_QUERY_MAJOR (one lane per
                               query walking its own buckets, the fields above)
                               for every pair, or CHM_KERNEL_BUCKET_MAJOR
                               (default): pairs whose db image has at least
                               bm_min_db_feats points run bucket major (one
                               launch per table, the lanes of a wavefront
                               sharing one db bucket), the others query major
                               (with CHM_WHOLE_LAST_BUCKET, and when the kept
                               lists do not fit the arena, all run query major) */
  int32_t bm_min_db_feats;  /* see match_kernel, 0..65536 (default 10176, the
                               first size above the query-major LDS code stage) */
  int32_t group_queries;    /* bucket major: pairs with the same db image are
                               grouped while their query images hold at most this
                               many descriptors together (at most 32 pairs),
                               1..1048576 (default 98304) */
  int32_t tail_percent;     /* query major, batched: the items making up the last
                               tail_percent of each XCD bin's work are halved,
                               0..50 (default 8) */
  int32_t hbm_item_queries; /* query major, batched launches that stage no db
                               image in LDS: queries per item, multiple of 64,
                               64..8192 (default 512) */
} chm_tuning;

enum { CHM_KERNEL_QUERY_MAJOR = 0, CHM_KERNEL_BUCKET_MAJOR = 1 };

chm_status chm_store_get_tuning(const chm_store *store, chm_tuning *out);
chm_status chm_store_set_tuning(chm_store *store, const chm_tuning *tuning);

/* ------------------------------------------------------------------ brute force
 * Exhaustive matching (every db descriptor is a candidate) with the same
 * exact squared distances and ratio test; the dense distance step runs as an
 * int8 MFMA GEMM with int32 accumulation.  It is the exactness and roofline
 * reference of the GPU nearest-neighbour matchers the paper compares with
 * (Table 2, ColMap-GPU).
 *   d_q, d_d   : device, nq x 128 and nd x 128 uint8.
 *   d_out      : device, nq int32 (j1 or -1).
 *   d_work     : device scratch of chm_bruteforce_work_bytes(nq, nd) bytes.
 * nq, nd in 0..2^24-1. */
chm_status chm_bruteforce_work_bytes(int32_t nq, int32_t nd, uint64_t *out_bytes);
chm_status chm_bruteforce(const uint8_t *d_q, int32_t nq, const uint8_t *d_d, int32_t nd,
                          int32_t ratio_num, int32_t ratio_den, int32_t *d_out, void *d_work,
                          uint64_t work_bytes, void *stream);

/* chm_bruteforce for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same computation and output, with the workspace taken from a fixed
 * 32 MiB device array the library holds on each GPU (until the process
 * ends) instead of a caller buffer.  It allocates nothing and calls no
 * hipMalloc/hipFree.  Sizes whose chm_bruteforce_work_bytes exceed 32 MiB
 * (about 2 million queries at one db split; a 40,000 x 40,000 pair needs
 * 9.1 MB) are rejected with CHM_E_CAPACITY.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and give undefined results; calls ordered on one stream are
 * safe.  The first call on a device resolves its copy of the array. */
chm_status chm_bruteforce_noalloc(const uint8_t *d_q, int32_t nq, const uint8_t *d_d, int32_t nd,
                                  int32_t ratio_num, int32_t ratio_den, int32_t *d_out, void *stream);

/* ------------------------------------------------------------------ schedule
 * Host-only MBR block schedule (Sec. 2.2 steps (1)-(5), Algorithm 1, GPS of
 * Appendix A).  Usable without a GPU.
 *   pairs       : host, n_pairs x 2 int32 directed pairs over images 0..n_images-1.
 *   image_bytes : host, n_images uint64, arena bytes of each image.
 *   cap_bytes   : residency cap (Size_gpu); every pair's two images must fit
 *                 together (else CHM_E_CAPACITY).
 *   blk_images  : Size_blk, images per schedule segment (>= 1).
 * The schedule is a list of steps; step s frees `evict`, loads `load` and
 * then matches the directed pairs `pairs` (indices into the input list); the
 * resident set never exceeds cap_bytes and every pair appears exactly once. */
typedef struct chm_schedule chm_schedule;

chm_status chm_schedule_mbr(int32_t n_images, const int32_t *pairs, int32_t n_pairs,
                            const uint64_t *image_bytes, uint64_t cap_bytes, int32_t blk_images,
                            chm_schedule **out);
/* A schedule given step by step, for running other data schedules (the
 * per-pair, load/free-list and graph-partition schedules Sec. 2.2 compares
 * MBR with, Fig. 2b) through chm_run_schedule.  Step k frees
 * evict_ids[evict_offs[k] .. evict_offs[k+1]), loads load_ids[load_offs[k]
 * ..] and matches the pairs (indices into `pairs`) pair_ids[pair_offs[k]
 * ..]; each offsets array has n_steps + 1 entries starting at 0.  The call
 * replays the residency and rejects (CHM_E_INVALID_ARG, naming the step) an
 * eviction of an absent image, a load of a resident one, resident bytes
 * above cap_bytes after a step's loads, a pair listed twice or in no step,
 * or a pair whose images are not resident at its step. */
chm_status chm_schedule_from_steps(int32_t n_images, int32_t n_pairs, const int32_t *pairs,
                                   const uint64_t *image_bytes, uint64_t cap_bytes, int32_t n_steps,
                                   const int32_t *evict_offs, const int32_t *evict_ids,
                                   const int32_t *load_offs, const int32_t *load_ids,
                                   const int32_t *pair_offs, const int32_t *pair_ids, chm_schedule **out);
int32_t chm_schedule_num_steps(const chm_schedule *s);
/* Pointers stay valid until chm_schedule_free. */
chm_status chm_schedule_step(const chm_schedule *s, int32_t step, const int32_t **evict,
                             int32_t *n_evict, const int32_t **load, int32_t *n_load,
                             const int32_t **pairs, int32_t *n_pairs);
/* iterations, pairs handled one per step after a stalled iteration, and per
 * iteration the matrix dimension and bandwidth (arrays of `iterations`). */
chm_status chm_schedule_info(const chm_schedule *s, int32_t *iterations, int32_t *fallback_pairs,
                             const int32_t **dims, const int32_t **bandwidths);
void chm_schedule_free(chm_schedule *s);

/* GPS ordering (Appendix A, Algorithm 2) of `nodes` in the undirected graph
 * given by n_edges x 2 `edges` over ids 0..n-1; order_out receives n_nodes ids. */
chm_status chm_gps_order(int32_t n, const int32_t *edges, int32_t n_edges, const int32_t *nodes,
                         int32_t n_nodes, int32_t *order_out);

/* Runs a schedule end to end (Algorithm 1, CascadeHashingMatching): for each
 * step, evicts, loads the new images from host memory (h_descs[image],
 * h_n_feats[image]; pinned memory makes the copies DMA transfers), builds
 * their codes and tables, and matches the step's pairs in one batched launch.
 * Kernels go on `stream`; descriptor copies go on a second stream the call
 * creates, so step k+1's copies overlap step k's matching when the arena has
 * room for them beside what step k still reads (slots evicted at step k+1
 * are held until step k ends; when room runs short the call waits for that
 * and frees them first).  Work queued on `stream` before the call finishes
 * before any copy starts.  The call returns when both streams are done; host
 * buffers must stay valid until then.  Outputs as in chm_plan_create for the
 * schedule's pair list.  The store's arena must hold cap_bytes of images plus
 * a step's work list (tens of bytes per work item); what it holds beyond
 * that is used to copy ahead. */
chm_status chm_run_schedule(chm_store *store, const chm_schedule *s, const int32_t *h_pairs,
                            int32_t n_pairs, const void *const *h_descs,
                            const int32_t *h_n_feats, const int64_t *h_out_offsets,
                            int32_t *d_out, void *stream);

/* SAO local geometric constraint (Sec. 2.3.3, Fig. 4): outlier removal of
 * initial matches on host threads (the paper runs it on the CPU beside the
 * GPU matching).  Host memory only; no GPU call.
 *
 * For every directed pair p (query image h_pairs[2p], db image h_pairs[2p+1])
 * the initial matches are h_match[h_offs[p] .. h_offs[p+1]), one per query
 * row (db row or -1), the layout the matcher writes.  Each match i -> m(i)
 * of a pair with M matches is scored as follows.
 *   - N = min(n_neighbors, M - 1).
 *   - O_p holds the N other matches whose query keypoints are nearest to
 *     query keypoint i, by squared distance, ties by the smaller query row.
 *   - O_q likewise holds the N other matches whose db keypoints are nearest
 *     to db keypoint m(i); a db keypoint matched by several queries is one
 *     point per match.
 *   - Both lists are put in angular order around their centre:
 *     counter-clockwise from +x, angles in [0, 2 pi), a neighbour on the
 *     centre first, equal angles by distance then row.
 *   - CED is the cyclic edit distance between the two lists of query rows:
 *     the least Levenshtein distance (unit costs) over their rotations.
 *   - The match is kept when the dissimilarity CED / N is at most
 *     score_num / score_den, that is CED * score_den <= score_num * N
 *     (N = 0 keeps it, with CED 0).
 *
 *   h_kp[img]   : h_n_feats[img] x 2 int32 keypoint coordinates (x, y) of
 *                 image img, any unit, |x|, |y| < 2^30 (all comparisons are
 *                 exact integer arithmetic).
 *   n_images    : entries of h_kp and h_n_feats.
 *   h_offs      : n_pairs + 1 non-decreasing offsets; pair p's range has the
 *                 query image's row count.
 *   n_neighbors : 1..32 (the paper's figure uses 6).
 *   n_threads   : worker threads; <= 0 uses every hardware thread.
 *   h_out       : filtered matches (the match or -1); may be h_match itself.
 *   h_ced       : optional (NULL), CED per query row, -1 where unmatched.
 * Errors: CHM_E_INVALID_ARG for a NULL array, an image id or db row out of
 * range, a coordinate out of range, or bad offsets or parameters. */
chm_status chm_sao_filter(int32_t n_pairs, const int32_t *h_pairs, const int32_t *const *h_kp,
                          const int32_t *h_n_feats, int32_t n_images, const int64_t *h_offs,
                          const int32_t *h_match, int32_t n_neighbors, int32_t score_num,
                          int32_t score_den, int32_t n_threads, int32_t *h_out, int32_t *h_ced);

/* SAO on the device: the scores and verdicts of chm_sao_filter for
 * n_neighbors 1..8, one work-group per pair (Sec. 2.3.3, Fig. 4).
 *   d_kp        : host array of n_images device pointers; d_kp[img] holds
 *                 h_n_feats[img] x 2 int32 keypoints, |x|, |y| < 2^30.
 *   h_pairs, h_n_feats, h_offs : as in chm_sao_filter (host memory).
 *   d_match     : device matches laid out by h_offs (the matcher's output).
 *   d_out       : device filtered matches; d_ced (optional) device CED per
 *                 query row (-1 where unmatched).  Neither may be d_match.
 *   d_work      : 256-byte aligned device scratch of chm_sao_work_bytes
 *                 (n_pairs, largest query image) bytes (CHM_E_CAPACITY if
 *                 smaller).  When the work completes, its first int32
 *                 holds the number of pairs whose input broke the contract
 *                 (a db row outside the db image, a coordinate out of
 *                 range); such pairs keep no match.
 * The call uploads the pair list (synchronising `stream` once) and then
 * enqueues the kernel on `stream`. */
chm_status chm_sao_work_bytes(int32_t n_pairs, int32_t max_query_rows, uint64_t *out_bytes);
chm_status chm_sao_filter_device(int32_t n_pairs, const int32_t *h_pairs, const int32_t *const *d_kp,
                                 const int32_t *h_n_feats, int32_t n_images, const int64_t *h_offs,
                                 const int32_t *d_match, int32_t n_neighbors, int32_t score_num,
                                 int32_t score_den, int32_t *d_out, int32_t *d_ced, void *d_work,
                                 uint64_t work_bytes, void *stream);

/* chm_run_schedule with outlier removal beside the block rows (Algorithm 1):
 * after each step's batched matching, the device SAO filter of that step's
 * pairs runs on the same stream and writes d_filtered (laid out like d_out).
 *   n_images   : entries of h_descs, h_n_feats and d_kp.
 *   d_kp, n_neighbors, score_num, score_den : as in chm_sao_filter_device.
 *   d_work     : 256-byte aligned, chm_sao_work_bytes(n_pairs, largest
 *                query image) bytes; its first int32 counts, over the whole
 *                run, the pairs whose SAO input broke the contract. */
chm_status chm_run_schedule_sao(chm_store *store, const chm_schedule *s, const int32_t *h_pairs,
                                int32_t n_pairs, const void *const *h_descs, const int32_t *h_n_feats,
                                int32_t n_images, const int64_t *h_out_offsets, int32_t *d_out,
                                const int32_t *const *d_kp, int32_t n_neighbors, int32_t score_num,
                                int32_t score_den, int32_t *d_filtered, void *d_work,
                                uint64_t work_bytes, void *stream);

/* chm_run_schedule_sao with RANSAC of every block row on host threads,
 * beside the device (Algorithm 1: outlier removal runs asynchronously with
 * the matching of the next block rows): once a step's device work (its
 * matching and SAO) ends, a worker thread copies the step's SAO output to
 * h_filtered and runs chm_ransac_filter's verification of the step's pairs
 * into h_verified, while the device goes on with the next steps.  The call
 * returns when the device work and every step's RANSAC are done.
 *   h_kp         : host array of n_images host keypoint arrays (the same
 *                  points as d_kp), |x|, |y| < 2^19.
 *   h_words, iterations, thr, min_inliers, n_threads : as in
 *                  chm_ransac_filter, h_words indexed by the pair's position
 *                  in h_pairs.
 *   h_filtered   : host memory laid out like d_out (pinned memory makes the
 *                  copies DMA transfers): receives the SAO output.
 *   h_verified   : host memory laid out like d_out: the verified matches.
 * Other arguments as in chm_run_schedule_sao.  A keypoint out of range, or a
 * db row outside its image, fails the call with CHM_E_INVALID_ARG. */
chm_status chm_run_schedule_verify(chm_store *store, const chm_schedule *s, const int32_t *h_pairs,
                                   int32_t n_pairs, const void *const *h_descs, const int32_t *h_n_feats,
                                   int32_t n_images, const int64_t *h_out_offsets, int32_t *d_out,
                                   const int32_t *const *d_kp, int32_t n_neighbors, int32_t score_num,
                                   int32_t score_den, int32_t *d_filtered, void *d_work, uint64_t work_bytes,
                                   const int32_t *const *h_kp, const uint32_t *h_words, int32_t iterations,
                                   int32_t thr, int32_t min_inliers, int32_t n_threads, int32_t *h_filtered,
                                   int32_t *h_verified, void *stream);

/* RANSAC global verification (Sec. 2.3.3) of each pair's matches on host
 * threads, with a 2D similarity as the two-view model (q = z (p - p_i) + q_i
 * in complex notation, fixed by two matches).  Host memory only.
 *   h_pairs, h_kp, h_n_feats, n_images, h_offs, h_match : as in
 *                  chm_sao_filter; coordinates must satisfy |x|, |y| < 2^19.
 *   h_words      : n_pairs x iterations x 2 random 32-bit words (the
 *                  caller's generator): hypothesis t of pair p takes match
 *                  i = u mod M and j = v mod (M - 1) (+1 when j >= i) of its
 *                  M matches, in query-row order.
 *   thr          : inlier distance in coordinate units, 0..2^20-1; match k
 *                  is an inlier when |q_k - z (p_k - p_i) - q_i| <= thr,
 *                  tested exactly in integers.
 *   min_inliers  : the best hypothesis (most inliers, the earlier on ties)
 *                  verifies the pair only with at least this many.
 *   h_out        : verified matches (the best hypothesis' inliers), -1
 *                  otherwise; may be h_match itself.
 *   h_best_counts: optional, inlier count of each pair's best hypothesis.
 * A pair with fewer than two matches verifies nothing. */
chm_status chm_ransac_filter(int32_t n_pairs, const int32_t *h_pairs, const int32_t *const *h_kp,
                             const int32_t *h_n_feats, int32_t n_images, const int64_t *h_offs,
                             const int32_t *h_match, const uint32_t *h_words, int32_t iterations,
                             int32_t thr, int32_t min_inliers, int32_t n_threads, int32_t *h_out,
                             int32_t *h_best_counts);

/* RANSAC on the device: the verification of chm_ransac_filter (Sec. 2.3.3;
 * the same hypotheses from the same words, the same exact integer test, the
 * same verified matches and best counts), one work-group per pair.
 *   d_kp         : host array of n_images device pointers; d_kp[img] holds
 *                  h_n_feats[img] x 2 int32 keypoints, |x|, |y| < 2^19.
 *   h_pairs, h_n_feats, h_offs : as in chm_ransac_filter (host memory).
 *   d_match      : device matches laid out by h_offs.
 *   d_words      : device n_pairs x iterations x 2 uint32 (the caller's
 *                  generator), as h_words of chm_ransac_filter.
 *   iterations, thr, min_inliers : as in chm_ransac_filter.
 *   d_out        : device verified matches; may be d_match itself.
 *   d_best_counts: optional device int32 per pair (best inlier count).
 *   d_work       : 256-byte aligned device scratch of chm_ransac_work_bytes
 *                  (n_pairs, largest query image) bytes (CHM_E_CAPACITY if
 *                  smaller).  When the work completes, its first int32
 *                  holds the number of pairs whose input broke the contract
 *                  (a db row outside the db image, a coordinate out of
 *                  range): such pairs verify nothing, where the host call
 *                  fails instead.
 * The call uploads the pair list (synchronising `stream` once) and then
 * enqueues the kernel on `stream`. */
chm_status chm_ransac_work_bytes(int32_t n_pairs, int32_t max_query_rows, uint64_t *out_bytes);
chm_status chm_ransac_filter_device(int32_t n_pairs, const int32_t *h_pairs, const int32_t *const *d_kp,
                                    const int32_t *h_n_feats, int32_t n_images, const int64_t *h_offs,
                                    const int32_t *d_match, const uint32_t *d_words, int32_t iterations,
                                    int32_t thr, int32_t min_inliers, int32_t *d_out, int32_t *d_best_counts,
                                    void *d_work, uint64_t work_bytes, void *stream);

/* chm_run_schedule_sao with device RANSAC of every block row on the same
 * stream (Algorithm 1's outlier removal entirely on the device): after each
 * step's matching and SAO, chm_ransac_filter_device's verification of the
 * step's pairs reads d_filtered and writes d_verified (laid out like d_out).
 *   d_words, iterations, thr, min_inliers : as in chm_ransac_filter_device,
 *                  d_words indexed by the pair's position in h_pairs.
 *   d_rwork      : 256-byte aligned, chm_ransac_work_bytes(n_pairs, largest
 *                  query image) bytes; its first int32 counts, over the
 *                  whole run, the pairs whose RANSAC input broke the
 *                  contract.
 * Other arguments as in chm_run_schedule_sao (d_work is the SAO's). */
chm_status chm_run_schedule_verify_device(chm_store *store, const chm_schedule *s, const int32_t *h_pairs,
                                          int32_t n_pairs, const void *const *h_descs, const int32_t *h_n_feats,
                                          int32_t n_images, const int64_t *h_out_offsets, int32_t *d_out,
                                          const int32_t *const *d_kp, int32_t n_neighbors, int32_t score_num,
                                          int32_t score_den, int32_t *d_filtered, void *d_work,
                                          uint64_t work_bytes, const uint32_t *d_words, int32_t iterations,
                                          int32_t thr, int32_t min_inliers, int32_t *d_verified, void *d_rwork,
                                          uint64_t rwork_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CHM_H */

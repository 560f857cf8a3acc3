/*
 * mask.h - C ABI of the MI355X (gfx950) implementation of the MASK hot path
 * (multilevel approximate similarity search with k-means, arXiv 2208.02734).
 *
 * Two operations sit behind this boundary:
 *   build  - Algorithm 1 (multilevel index construction): split the data into
 *            groups, run k-means in every group, summarise the prototypes of
 *            one level with k-means again, bottom-up;
 *   query  - Algorithm 2 (k-NN search) and Section 3.3 (searching): descend
 *            from the top level through the prototypes nearest to the query,
 *            generalised from the single nearest prototype to a beam of the r
 *            nearest at every level, and rank the data points under the
 *            chosen leaves.
 * The inputs follow the problem statement of Section 1: a dataset, a
 * dissimilarity delta, the level sizes, the queries, k and the probe width r.
 *
 * Conventions for every call:
 *   - every call returns a mask_status; none throws, aborts or prints;
 *     mask_last_error() returns a thread-local description of the last
 *     failure on the calling thread;
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary CPU memory;
 *   - the caller owns every buffer it passes in; the library never frees
 *     them and keeps no pointer to them after the call returns (build) or
 *     after the stream reaches the enqueued work (query);
 *   - invalid arguments return MASK_ERR_INVALID before anything is
 *     allocated or enqueued; an allocation failure returns MASK_ERR_NOMEM
 *     after releasing what the call allocated; a HIP runtime error returns
 *     MASK_ERR_DEVICE.
 */
#ifndef MASK_H
#define MASK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MASK_OK = 0,
  MASK_ERR_INVALID = 1,     /* bad argument; nothing was allocated or enqueued */
  MASK_ERR_NOMEM = 2,       /* device allocation failed */
  MASK_ERR_DEVICE = 3,      /* a HIP runtime call failed */
  MASK_ERR_UNSUPPORTED = 4, /* valid request this build does not implement */
  MASK_ERR_BUSY = 5,        /* a request that can never fit the serving arena */
  MASK_ERR_SHUTDOWN = 6     /* the server is shutting down */
} mask_status;

/* The dissimilarity delta (Section 1, Minkowski family).  Euclidean is the
 * one every experiment of the paper uses; ranking uses the squared distance
 * and the Euclidean distance is reported.  L1 ranks and reports sum |a-b|. */
typedef enum { MASK_L2 = 0, MASK_L1 = 1 } mask_metric;

/* Arithmetic of the distance screening.  MASK_FP32 is the plain form.
 * MASK_BF16: the build screens on BF16 MFMA; the descent reads BF16 rows at
 * every level.  MASK_FP8_E4M3: rows quantised to OCP e4m3 with one FP32
 * scale per row (s = max|x| / 448); the build screens on FP8 MFMA; the
 * descent reads the data layer in FP8 and prototype levels in FP32.  Both
 * re-rank the data layer's best candidates in FP32 (see mask_query) and keep
 * FP64 sums; L2 metric only. */
typedef enum { MASK_FP32 = 0, MASK_BF16 = 1, MASK_FP8_E4M3 = 2 } mask_precision;

/* Optional device allocator (for instance PyTorch's caching allocator).
 * alloc returns NULL on failure; free receives the size that was allocated.
 * A NULL mask_allocator* means hipMalloc / hipFree. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* hip_stream);
  void (*free)(void* ctx, void* ptr, size_t bytes, void* hip_stream);
} mask_allocator;

typedef enum { MASK_DENSE = 0, MASK_CSR = 1 } mask_layout;

/* A matrix of n rows (points or queries) with dim columns, device memory.
 * DENSE: x is row-major n x dim float32 with row stride ld floats
 *        (ld == 0 means ld = dim).
 * CSR:   indptr int64[n+1] rising from 0 to nnz, indices int32[nnz]
 *        (column ids strictly increasing within a row, each < dim), values
 *        float32[nnz]; nnz < 2^31, dim <= 16384.  CSR data (Section 4.3: the
 *        high-dimensional sparse setting) builds a CSR index: L2 metric, FP32
 *        form, distances |x|^2 + |c|^2 - 2 x.c evaluated in float64; its
 *        queries are CSR as well.  mask_build, mask_import and mask_kmeans
 *        check the structure on the device (MASK_ERR_INVALID); queries are
 *        not checked. */
typedef struct {
  int32_t layout;
  int64_t n;
  int32_t dim;
  int32_t ld;
  const float* x;
  const int64_t* indptr;
  const int32_t* indices;
  const float* values;
  int64_t nnz;
} mask_matrix;

/* Most levels an index has. */
#define MASK_MAX_LEVELS 16

/* One level of the index, bottom-up: the items of the level below (the data
 * for levels[0]) are split into n_chunks contiguous groups of nearly equal
 * size (Algorithm 1, split) and k-means with k prototypes runs in each. */
typedef struct {
  int32_t n_chunks;
  int32_t k;
} mask_level;

typedef struct {
  int32_t metric;        /* mask_metric */
  int32_t precision;     /* mask_precision */
  int32_t n_levels;      /* 1..16 */
  const mask_level* levels; /* host array [n_levels], bottom-up */
  int32_t lloyd_iters;   /* Lloyd iterations per level (>= 0) */
  uint64_t seed;         /* seeds the level-0 permutation */
  int32_t rerank_factor; /* precision forms: FP32 re-rank of rerank_factor*k
                            candidates; a negative value -f re-ranks f*k*r1
                            (r1: the query's level-1 beam, the leaves probed);
                            0: 4 for BF16, 48 for FP8 */
  const int32_t* perm;   /* optional device int32[n]: level-0 order; NULL = from seed */
  const int64_t* group_off; /* optional host int64[levels[0].n_chunks + 1]: level-0 group
                               boundaries in that order, rising strictly from 0 to n (as
                               mask_relocate writes them); NULL = split (dense data only) */
  int32_t init;             /* mask_init; k-means++ draws use seed and the level number */
} mask_build_params;

/* Initial prototypes of every group's Lloyd iterations. */
typedef enum {
  MASK_INIT_FIRST = 0,    /* the group's first k members (cyclically if fewer) */
  MASK_INIT_KMEANSPP = 1  /* k-means++ seeding (mask_kmeanspp), dense L2 only */
} mask_init;

typedef struct mask_index mask_index;

typedef struct {
  int64_t n;
  int32_t dim;
  int32_t n_levels;
  int32_t metric;
  int32_t precision;
  int64_t level_size[16];    /* prototypes per level, bottom-up */
  int64_t device_bytes;      /* device memory held by the index */
  int64_t refined_last_level;/* points re-scored in direct form by the last
                                assignment of the build (plain form) */
  int32_t layout;            /* mask_layout of the data (CSR index or dense) */
  int64_t nnz;               /* non-zeros of the data (CSR index) */
} mask_info;

/* Level schedule of Algorithm 1: ngroups = n / length_group (floor); every
 * level summarises the previous one with n_centroids prototypes per group;
 * stop once fewer than one full group remains.  Writes up to cap levels to
 * out (host) and the count to *n_levels.  MASK_ERR_INVALID when the schedule
 * does not shrink (n_centroids >= length_group) or does not fit cap. */
mask_status mask_plan_levels(int64_t n, int32_t length_group, int32_t n_centroids,
                             mask_level* out, int32_t cap, int32_t* n_levels);

/* Algorithm 1.  data: device matrix (DENSE with dim <= 256 for the MFMA
 * assignment, or CSR: every level's prototypes are then dense rows, and the
 * items of the next level are those prototypes with their zeros dropped).
 * Level 0 is permuted by the argsort of the SplitMix64
 * outputs h(seed, i) (or by p->perm) and split into levels[0].n_chunks
 * groups (or cut at p->group_off); each group runs lloyd_iters Lloyd
 * iterations starting from its first k members (taken cyclically when the
 * group holds fewer than k: the repeated copies lose every tie and stay
 * empty) or from its k-means++ seeds (p->init), then a final assignment.  Every chunk must hold at least one item.  The index copies what it needs: data may be freed after the call.
 * Work runs on hip_stream (NULL = the null stream); the call returns after it
 * completes.  On success *out owns device memory until mask_free. */
mask_status mask_build(const mask_matrix* data, const mask_build_params* p,
                       const mask_allocator* a, void* hip_stream, mask_index** out);

/* Algorithm 2 with a beam: for each of the q->n queries (device, DENSE, or
 * CSR for a CSR index; dim equal to the index's) keep the r nearest prototypes of the top level,
 * then at each level below the r nearest children of those, then return the
 * k nearest data points under the kept level-1 prototypes.  Ranking key:
 * (distance, original id).  out_ids: device int32[q->n * k] (original data
 * row ids), out_dist: device float32[q->n * k], rows ascending; slots beyond
 * the candidate count hold id -1 and +inf.  1 <= k <= 2048, 1 <= r <= 2048;
 * on a CSR index of at most 12,288 columns r may reach 3072 (sparse rows need
 * a larger share of the leaves probed for the same recall).
 * Precision forms (index built with MASK_BF16 or MASK_FP8_E4M3): rows are
 * compared in the low precision and the data layer's R = min(rerank_factor *
 * k, C) nearest by that distance (R = min(f * k * r1, C) for rerank_factor =
 * -f, r1 the level-1 beam)
 * are re-ranked in FP32 direct form on the FP32 rows, where C = 512 when k
 * and every beam are at most 512 and 2048 otherwise (all candidates in FP32
 * when they are no more than R, or when R <= k).
 * Asynchronous on hip_stream; allocates nothing.  Each query's result does
 * not depend on the other queries of the batch. */
mask_status mask_query(const mask_index* ix, const mask_matrix* q, int32_t k, int32_t r,
                       int32_t* out_ids, float* out_dist, void* hip_stream);

/* mask_query with a beam per level: r_levels (host int32[n_levels], top
 * level first) gives the number of prototypes kept at each level, each in
 * [1, 2048] (in [1, 3072] on a CSR index of at most 12,288 columns).  The
 * uniform-beam descent is r_levels = {r, ..., r}. */
mask_status mask_query_beams(const mask_index* ix, const mask_matrix* q, int32_t k,
                             const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                             void* hip_stream);

/* mask_query_beams for an index in the BF16 form, with the small
 * prototype levels (at most 16,384 prototypes; usually the top levels)
 * screened for the whole batch at once: one BF16 MFMA GEMM per such level
 * gives every query's squared distance to every prototype of the level, as
 * |q|^2 + |c~|^2 - 2 q.c~ (c~ the BF16 row, q in FP32 split into two BF16
 * terms, FP32 accumulation, clamped at 0), and the descent reads those
 * instead of the rows.  Larger levels and the data layer are as in
 * mask_query_beams.  workspace: device memory of workspace_bytes (256-byte
 * aligned) that the call owns until it completes on hip_stream; queries are
 * processed in slices that fit it (mask_screen_bytes gives the bytes per
 * query; at least one query must fit).  The queries of a slice are
 * launched in the order of their greedy path through the screened levels,
 * so that queries in one subtree share the cache of one XCD; each query's
 * result does not depend on that order.  Results are the screened
 * distances' ranking, not bit-equal to mask_query_beams.
 * MASK_ERR_UNSUPPORTED for other forms.  Asynchronous; allocates nothing. */
mask_status mask_query_screened(const mask_index* ix, const mask_matrix* q, int32_t k,
                                const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                                void* workspace, int64_t workspace_bytes, void* hip_stream);

/* mask_query_screened plus the prototypes kept at every level (as
 * mask_query_beams_debug writes them: sel is device int32[q->n * n_levels *
 * rmax], rmax the largest beam), so that the screened selections can be
 * checked against distances computed elsewhere. */
mask_status mask_query_screened_debug(const mask_index* ix, const mask_matrix* q, int32_t k,
                                      const int32_t* r_levels, int32_t* out_ids,
                                      float* out_dist, int32_t* sel, void* workspace,
                                      int64_t workspace_bytes, void* hip_stream);

/* mask_query_screened with the data layer (Algorithm 2's scan of the kept
 * leaves) evaluated leaf by leaf, for an index in the BF16 form with dim at
 * most 256: the prototype levels are descended first and keep each query's
 * level-1 prototypes; the (leaf, query) pairs are sorted by leaf, and a
 * workgroup takes 32 of them at a time and computes the BF16 distance of
 * every row of each leaf to each of its queries there (the descent's own
 * arithmetic), so a leaf's rows are read once per 32 queries that kept it
 * instead of once per query; a last pass ranks those distances (the
 * re-rank set, the FP32 re-rank, the k nearest).  The level and ranking
 * passes take one wave per query when k and the re-rank set are at most 192
 * and every beam at most 192 (the level-1 beam at most 128), else a
 * workgroup per query.  Results equal mask_query_screened's bit for bit.  workspace: device memory of
 * workspace_bytes (256-byte aligned) that the call owns until it completes
 * on hip_stream; queries are processed in slices that fit it
 * (mask_batched_bytes gives the bytes of a slice; one query must fit).
 * MASK_ERR_UNSUPPORTED for other forms or dim above 256.  Asynchronous;
 * allocates nothing. */
mask_status mask_query_batched(const mask_index* ix, const mask_matrix* q, int32_t k,
                               const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                               void* workspace, int64_t workspace_bytes, void* hip_stream);

/* mask_query_batched plus the prototypes kept at every level, laid out as
 * mask_query_screened_debug writes them: the same sets, each in an order of
 * its own. */
mask_status mask_query_batched_debug(const mask_index* ix, const mask_matrix* q, int32_t k,
                                     const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                                     int32_t* sel, void* workspace, int64_t workspace_bytes,
                                     void* hip_stream);

/* Workspace bytes of mask_query_batched for one slice of n_queries queries
 * (in [1, 2^20]) at beams r_levels (top level first): the screened scores
 * and launch order, r1 kept-leaf slots per query and the distances of at
 * most the rows of the index's r1 largest leaves per query (r1 the level-1
 * beam), and the buffers of the pair sort. */
mask_status mask_batched_bytes(const mask_index* ix, const int32_t* r_levels,
                               int64_t n_queries, int64_t* bytes);

/* Size of the device scratch of mask_query_screened_noalloc: 64 MiB, held
 * by every GPU the library runs on from its first call there until the
 * process ends. */
#define MASK_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)

/* mask_query_screened for callers that cannot allocate device memory or
 * take a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the score rows and launch order live
 * in a static device array of MASK_NOALLOC_SCRATCH_BYTES per GPU, so the
 * call takes no workspace; queries are processed in slices that fit it.
 * The caller still passes the queries and the outputs.  The array's
 * address is looked up once per device, on the first call with that device
 * current; the call itself allocates nothing.  MASK_ERR_INVALID when one
 * query's screened scores (mask_screen_bytes) exceed the scratch.  Results
 * equal mask_query_screened's with any workspace.  Every call on one GPU
 * shares its array: calls that overlap on one GPU (other streams, other
 * host threads) race and must be ordered by the caller. */
mask_status mask_query_screened_noalloc(const mask_index* ix, const mask_matrix* q, int32_t k,
                                        const int32_t* r_levels, int32_t* out_ids,
                                        float* out_dist, void* hip_stream);

/* Workspace bytes per query of mask_query_screened: 4 bytes per prototype
 * of every screened level, each level's count rounded up to a multiple of
 * 32, plus 8 bytes for the launch order (0 when nothing is screened). */
mask_status mask_screen_bytes(const mask_index* ix, int64_t* bytes_per_query);

/* Ragged batch: query i uses k_i[i] and r_i[i] (device int32[q->n], each in
 * [1, k_max] / [1, r_max]) and writes its k_i[i] results at out_ids +
 * out_off[i] / out_dist + out_off[i] (device int64[q->n]).  k_max, r_max <=
 * 2048 are host values bounding the per-query ones (they size the launch).
 * beam_eighths: NULL (query i keeps r_i[i] prototypes at every level, as
 * mask_query), or a beam profile, host int32[n_levels] top level first:
 * query i keeps ceil(r_i[i] * beam_eighths[d] / 8) prototypes at level d
 * (0 keeps r_i[i]); each such beam at r_max must be at most 2048.
 * Otherwise as mask_query; each query's result equals what mask_query (or,
 * with a profile, mask_query_beams with the query's own beams) returns for
 * it alone with the same k (in the precision forms the re-rank cap C
 * follows the query's own k and beams). */
mask_status mask_query_ragged(const mask_index* ix, const mask_matrix* q, const int32_t* k_i,
                              const int32_t* r_i, const int64_t* out_off, int32_t k_max,
                              int32_t r_max, const int32_t* beam_eighths, int32_t* out_ids,
                              float* out_dist, void* hip_stream);

/* mask_query_beams plus the prototypes kept at every level: sel is device
 * int32[q->n * n_levels * rmax] (rmax the largest of r_levels), level-major
 * from the top level down, each set of chunk-major prototype ids in no
 * particular order, padded with -1.  Parity checks replay a descent on
 * these selections (Algorithm 2, the per-level choice). */
mask_status mask_query_beams_debug(const mask_index* ix, const mask_matrix* q, int32_t k,
                                   const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                                   int32_t* sel, void* hip_stream);

/* mask_query plus the prototypes kept at every level: sel is device
 * int32[q->n * n_levels * r], level-major from the top level down, each set
 * of chunk-major prototype ids in no particular order, padded with -1. */
mask_status mask_query_debug(const mask_index* ix, const mask_matrix* q, int32_t k,
                             int32_t r, int32_t* out_ids, float* out_dist, int32_t* sel,
                             void* hip_stream);

/* Range search (Algorithm 3): for each query, the prototypes within
 * radius[i] (device float32[q->n]; a negative or NaN radius finds nothing)
 * are kept at the top level and, among the children of the kept ones, at
 * every level below (at most level_cap per level: the nearest, by (distance,
 * id)); the answer is the data points within radius[i] under the kept
 * level-1 prototypes.  out_ids / out_dist (device, q->n x max_out): the
 * nearest max_out of them ascending, padded with (-1, +inf); out_count
 * (device int32[q->n]): how many are within the radius (may exceed
 * max_out).  Distances compare as squared L2 against radius^2 in float32.
 * Plain FP32 form (dense or CSR), L2 metric; 1 <= max_out, level_cap <=
 * 2048.  Asynchronous on hip_stream. */
mask_status mask_query_range(const mask_index* ix, const mask_matrix* q, const float* radius,
                             int32_t max_out, int32_t level_cap, int32_t* out_ids,
                             float* out_dist, int32_t* out_count, void* hip_stream);

/* Point query (Section 3.3): the nearest prototype at the top level, then
 * at each level the nearest child of the one chosen above (r = 1, ranking
 * key (distance, id)); a full scan of the data rows under the level-1
 * prototype reached (the leaf) gives the answer.  Per query i (device
 * arrays of q->n): out_ids[i] / out_dist[i] = the nearest row of the leaf
 * (as mask_query with k = r = 1; -1 / +inf when the leaf is empty or an
 * empty prototype was chosen above it), out_leaf[i] = the leaf's
 * chunk-major id (-1 when none was reached), out_match[i] = the lowest id of
 * a row of the leaf equal to the query in every coordinate (float
 * comparison), else -1.  Dense indexes, any form.  Asynchronous; allocates
 * nothing. */
mask_status mask_point_query(const mask_index* ix, const mask_matrix* q, int32_t* out_ids,
                             float* out_dist, int32_t* out_leaf, int32_t* out_match,
                             void* hip_stream);

/* Dynamic insertion (Section 3.3): each row of points (device, DENSE, dim
 * as the index) descends greedily -- the nearest prototype at the top
 * level, then the nearest child at each level, skipping prototypes without
 * children above level 1 -- and joins the data rows of the level-1
 * prototype it reaches; out_leaf (device int32[points->n]) receives that
 * prototype's chunk-major id.  The new rows take ids n, n+1, ... in order
 * (n = the index's row count before the call) and join the level-0 group of
 * their leaf, after its members.  When max_leaf > 0, every level-0 group
 * that then holds a leaf of more than max_leaf rows is built again
 * locally: the build's lloyd_iters Lloyd iterations over the group's
 * current rows, starting from its current prototypes, then a final
 * assignment; the prototypes keep their places in the levels above.
 * *n_rebuilt = the number of groups rebuilt.  Index built by mask_build
 * from dense data only (MASK_ERR_UNSUPPORTED otherwise).  Must not race with
 * queries or with a server on the index.  Synchronous. */
mask_status mask_insert(mask_index* ix, const mask_matrix* points, int32_t max_leaf,
                        int32_t* out_leaf, int32_t* n_rebuilt, const mask_allocator* a,
                        void* hip_stream);

/* One relocation step (Sections 4.1-4.2, the relocation table): every data
 * row i with wrong[i] != 0 whose point query reached leaf[i] >= 0 joins the
 * level-0 group that produced that leaf (leaf[i] / levels[0].k); the others
 * stay.  leaf and wrong: device int32[n] in data row order (mask_point_query
 * over all data rows gives leaf; the caller decides what is wrong).  Each
 * group keeps its staying rows in their old order followed by the rows that
 * join it in their old order; groups left empty are dropped.  Writes the
 * new level-0 order to perm_out (device int32[n]) and its group boundaries
 * to group_off_out (host, *n_groups + 1 entries; cap >= levels[0].n_chunks
 * + 1), ready for mask_build's perm and group_off.  Needs an index built by
 * mask_build from dense data (MASK_ERR_UNSUPPORTED otherwise);
 * MASK_ERR_INVALID when a leaf lies outside level 1.  Synchronous. */
mask_status mask_relocate(const mask_index* ix, const int32_t* leaf, const int32_t* wrong,
                          int32_t* perm_out, int64_t* group_off_out, int32_t cap,
                          int32_t* n_groups, const mask_allocator* a, void* hip_stream);

/* Releases the index (NULL is allowed).  Must not race with queries. */
mask_status mask_free(mask_index* ix);

mask_status mask_index_info(const mask_index* ix, mask_info* out);

/* Copies level `level` (1 = first prototype level, n_levels = top) to host
 * memory: protos_host float32[n_l * dim] in chunk-major id order, and, when
 * parent_host is not NULL, parent_host int32[n_{l-1}] = chunk-major id of the
 * level-l prototype of each item one level down (original data row order
 * for level 1).  Synchronous. */
mask_status mask_export_level(const mask_index* ix, int32_t level, float* protos_host,
                              int32_t* parent_host);

/* Builds an index from prototypes and parents computed elsewhere (host
 * arrays laid out as mask_export_level writes them), so that a query can be
 * compared on an index shared with another implementation.  data as in
 * mask_build; p supplies metric and precision. */
mask_status mask_import(const mask_matrix* data, int32_t n_levels, const mask_level* levels,
                        const float* const* protos_host, const int32_t* const* parents_host,
                        const mask_build_params* p, const mask_allocator* a, void* hip_stream,
                        mask_index** out);

/* k-means++ seeding (Arthur and Vassilvitskii 2007, named in Section 3.1)
 * of every group: items (device, DENSE, n x dim, dim <= 256) are split into
 * n_chunks groups as mask_kmeans splits them.  In group c, draw t takes u =
 * (top 53 bits of the SplitMix64 output at counter level * 2^40 + c * k + t
 * from state seed) * 2^-53; draw 0 picks member floor(u * m); draw t > 0
 * picks the first member, in group order, whose running sum of D^2 exceeds
 * u * sum D^2 (D^2: squared distance to the nearest seed so far, float64
 * direct form); a zero sum picks uniformly as draw 0, and a target that
 * rounding leaves unreached picks the last member with D^2 > 0.  Outputs
 * (device): centroids float32[n_chunks*k*dim] (the chosen rows), chosen
 * int32[n_chunks*k] (their item indices; may be NULL).  mask_build with
 * init = MASK_INIT_KMEANSPP seeds level l this way with level = l.
 * Synchronous. */
mask_status mask_kmeanspp(const mask_matrix* items, int32_t n_chunks, int32_t k, uint64_t seed,
                          int32_t level, float* centroids, int32_t* chosen,
                          const mask_allocator* a, void* hip_stream);

/* The batched per-group k-means of Algorithm 1 on its own (the build's
 * inner loop): items (device, DENSE or CSR, n x dim) are split into n_chunks
 * contiguous groups of nearly equal size; group c uses prototypes
 * centroids[c*k .. c*k+k-1].  init: device float32[n_chunks*k*dim] starting
 * prototypes, or NULL for the first k items of each group.  Runs `iters`
 * Lloyd iterations, then a final assignment.  Outputs (device): centroids
 * float32[n_chunks*k*dim], labels int32[n] (chunk-major prototype ids of the
 * final assignment), inertia float64[iters*n_chunks] (sum over the group of
 * delta(x, c^t_{a^t}) at iteration t; may be NULL).  Synchronous. */
mask_status mask_kmeans(const mask_matrix* items, int32_t n_chunks, int32_t k, int32_t iters,
                        int32_t metric, const float* init, float* centroids, int32_t* labels,
                        double* inertia, const mask_allocator* a, void* hip_stream);

const char* mask_last_error(void);

/* ------------------------------------------------------------- serving ---
 * A request loop against a resident index (the serving form): requests are
 * queued by mask_server_submit; a scheduler thread admits them in arrival
 * order into ragged batches while they fit a batch-size limit and a free
 * block of the device arena (memory admission), and keeps up to n_streams
 * batches in flight, so requests arriving while others run join the next
 * batch as soon as a stream and arena space are free (continuous batching).
 * Each query's result equals mask_query's for it alone with the same k, r
 * (with a beam profile, mask_query_beams's with the profile's beams). */
typedef struct mask_server mask_server;

typedef struct {
  int64_t arena_bytes;       /* device memory for in-flight batches (>= 4096) */
  int32_t max_batch_queries; /* largest number of queries in one batch */
  int32_t n_streams;         /* batches in flight at once, 1..16 */
  int32_t batch_window_us;   /* a batch that is not full launches once its oldest
                                request has been queued this long (0: at once) */
  int32_t beam_eighths[MASK_MAX_LEVELS]; /* beam profile, top level first: a request
                                with probe width r keeps ceil(r * beam_eighths[d] / 8)
                                prototypes at level d (0 keeps r); all zero: r at
                                every level */
} mask_server_params;

typedef struct {
  int64_t submitted_requests, submitted_queries;
  int64_t completed_requests, completed_queries;
  int64_t batches, batched_queries;
  int64_t peak_arena_bytes, arena_used_bytes;
  int64_t queued_requests, inflight_batches;
} mask_server_stats;

/* Seconds on the steady clock the server stamps completions with; callers
 * give arrival times on the same clock, so latency = t_done - t_arrival. */
double mask_clock(void);

/* The index must outlive the server.  The arena comes from the allocator
 * (NULL: hipMalloc); staging memory of the same size is pinned host memory.
 * Dense indexes only (MASK_ERR_UNSUPPORTED for a CSR index). */
mask_status mask_server_create(const mask_index* ix, const mask_server_params* p,
                               const mask_allocator* a, mask_server** out);

/* Queues n_q query rows (host, n_q x dim, copied before return) with k and r
 * and the caller's arrival time.  MASK_ERR_BUSY when the request could never
 * fit the arena or the batch limit; MASK_ERR_SHUTDOWN during destroy. */
mask_status mask_server_submit(mask_server* s, const float* q_host, int32_t n_q, int32_t k,
                               int32_t r, double t_arrival, uint64_t* ticket);

/* *done = 1 when the request has finished: then ids_host (int32[n_q*k]) and
 * dist_host (float[n_q*k]) receive the rows (either may be NULL), *t_done
 * the completion time, and the ticket is released.  *done = 0 otherwise. */
mask_status mask_server_poll(mask_server* s, uint64_t ticket, int32_t* done, int32_t* ids_host,
                             float* dist_host, double* t_done);

mask_status mask_server_stats_get(mask_server* s, mask_server_stats* out);

/* Open-loop load generator for measuring the serving loop: from the calling
 * thread, submits request i at t0 + t_offset[i] seconds (t0 = the call's
 * start plus 1 ms; t_offset non-decreasing) with rows pool_off[i] ..
 * pool_off[i] + n_q[i] - 1 of pool_host (host, pool_rows x dim), k[i] and
 * r[i], with that scheduled time as its arrival; polls completions in
 * between (results are discarded) and returns once every request is done.
 * latency[i] (host double[n_req]) = completion - scheduled arrival in
 * seconds; *span = last completion - t0 (may be NULL).  Submission errors
 * (MASK_ERR_BUSY for a request that can never fit) end the replay. */
mask_status mask_server_replay(mask_server* s, const float* pool_host, int64_t pool_rows,
                               int64_t n_req, const double* t_offset, const int32_t* n_q,
                               const int64_t* pool_off, const int32_t* k, const int32_t* r,
                               double* latency, double* span);

/* Serves every queued request, then stops the scheduler and frees the
 * server.  Requests not polled are dropped. */
mask_status mask_server_destroy(mask_server* s);

/* Kernel timing for measurement: while enabled, the library's main kernels
 * (assignment, refinement, update, member sort, descent) record HIP events
 * on the stream they are launched on.  Enabling (or disabling) discards what
 * was recorded.  Adds event records to every instrumented launch. */
mask_status mask_timing_enable(int32_t on);

/* Writes one line per kernel name, "name launches total_ms", plus the
 * counters "descent_rows <candidate rows evaluated by the descent> 0",
 * "refine_small_points <n> 0" and "refine_full_points <n> 0" (points the
 * assignment re-scored in direct form on 2-3 prototypes / on the whole
 * group), to buf (host,
 * NUL-terminated, truncated to cap); *needed receives the full size.
 * Waits for the recorded events. */
mask_status mask_timing_report(char* buf, int64_t cap, int64_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* MASK_H */

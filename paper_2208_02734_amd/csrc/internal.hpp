// Internal declarations shared by the host runtime and the kernel files.
// Everything here targets gfx950 (CDNA4): 64-lane wavefronts, MFMA, 160 KB
// LDS per compute unit, 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mask.h"

namespace mask {

constexpr int kWave = 64;
constexpr int kMaxLevels = 16;
constexpr int kMaxDenseDim = 256;   // MFMA assignment keeps point rows in registers
constexpr int kMaxQueryDim = 4096;  // the descent stages one query row in LDS
constexpr int kMaxBeam = 2048;      // r and k limit of one descent workgroup
// A CSR index keeps up to 3,072 prototypes per level (a wider LDS class, which
// fits beside the dense query vector for up to 12,288 columns): sparse rows
// need a larger share of the leaves probed for the same recall.
constexpr int kMaxBeamCsr = 3072;
constexpr int kMaxCsrWideDim = 12288;
constexpr int kMaxRerank = 2048;    // largest FP32 re-rank set of the BF16 form
constexpr int kMaxSparseDim = 16384; // CSR columns: the descent scatters a query row in LDS

// ------------------------------------------------------------------ errors

void set_error(const std::string& msg);

struct Error {
  mask_status status;
  std::string msg;
};

#define MASK_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::mask::Error{MASK_ERR_DEVICE, std::string(#call) + ": " +              \
                                               hipGetErrorString(e_)};              \
  } while (0)

#define MASK_CHECK(cond, msg)                                                       \
  do {                                                                              \
    if (!(cond)) throw ::mask::Error{MASK_ERR_INVALID, (msg)};                      \
  } while (0)

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    throw Error{MASK_ERR_DEVICE, std::string("launch ") + what + ": " + hipGetErrorString(e)};
}

// ------------------------------------------------------------------ timing
// When enabled (mask_timing_enable), instrumented launches record a pair of
// HIP events on their stream; mask_timing_report sums the elapsed times per
// kernel name.  Disabled, a ScopedTiming costs one branch.
bool timing_enabled();
// "<prefix><level>" as a string that lives as long as the library (a
// timing scope name), for levels 0 .. kMaxLevels.
const char* level_scope_name(const char* prefix, int level);
void timing_record(const char* name, hipStream_t s, bool start);
// The two counters below are kCounterShards device slots each (a workgroup
// adds to slot blockIdx.x % kCounterShards, so that one launch's workgroups
// do not all wait on one address); the report sums them.
constexpr int kCounterShards = 64;
// Device counter the descent kernels add their evaluated candidate rows to
// while timing is enabled (null otherwise).
unsigned long long* timing_row_counter();
// (query, row) pairs the leaf-batched data layer evaluates, or null
unsigned long long* timing_leaf_counter();
// Two device counters (points refined on 2-3 candidates, on the whole group)
// while timing is enabled, null otherwise.
unsigned long long* timing_refine_counter();
// rows not ruled out, rows read exactly and D^2 lowered by the k-means++
// updates of one level (three counters; levels at or above kSeedSlots - 1
// share the last slot)
constexpr int kSeedSlots = 16;
unsigned long long* timing_seed_counter(int slot);

struct ScopedTiming {
  const char* name;
  hipStream_t s;
  bool on;
  ScopedTiming(const char* n, hipStream_t st, bool want = true)
      : name(n), s(st), on(want && timing_enabled()) {
    if (on) timing_record(name, s, true);
  }
  ~ScopedTiming() {
    if (on) timing_record(name, s, false);
  }
};

// -------------------------------------------------------------- allocation

// Device memory owned by one object (an index or one build's scratch).  Every
// allocation goes through the caller's mask_allocator when one is given.
class Arena {
 public:
  Arena(const mask_allocator* a, hipStream_t s) : s_(s) {
    if (a) { a_ = *a; has_ = true; }
  }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena() { release(); }

  void* alloc_bytes(size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void* p = nullptr;
    if (has_) {
      p = a_.alloc(a_.ctx, bytes, (void*)s_);
      if (!p) throw Error{MASK_ERR_NOMEM, "allocator returned NULL"};
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        throw Error{MASK_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
      }
    }
    blocks_.push_back({p, bytes});
    bytes_ += bytes;
    return p;
  }
  template <class T>
  T* alloc(size_t count) {
    return static_cast<T*>(alloc_bytes(count * sizeof(T)));
  }
  // Frees one allocation early (scratch that is no longer needed).
  void free_one(void* p) {
    for (size_t i = 0; i < blocks_.size(); ++i) {
      if (blocks_[i].p == p) {
        do_free(blocks_[i]);
        bytes_ -= blocks_[i].bytes;
        blocks_.erase(blocks_.begin() + i);
        return;
      }
    }
  }
  void release() {
    for (auto& b : blocks_) do_free(b);
    blocks_.clear();
    bytes_ = 0;
  }
  size_t bytes() const { return bytes_; }
  hipStream_t stream() const { return s_; }
  void set_stream(hipStream_t s) { s_ = s; }

 private:
  struct Block { void* p; size_t bytes; };
  void do_free(const Block& b) {
    if (has_) a_.free(a_.ctx, b.p, b.bytes, (void*)s_);
    else (void)hipFree(b.p);
  }
  mask_allocator a_{};
  bool has_ = false;
  hipStream_t s_;
  std::vector<Block> blocks_;
  size_t bytes_ = 0;
};

// ------------------------------------------------------------- primitives
// (prims.hip)

// Workspace of the radix sort: ping-pong buffers, the per-wave digit
// histogram table and the scan's tile sums, sized for up to cap_n keys.
struct SortWork {
  void* keys2 = nullptr;
  uint32_t* vals2 = nullptr;
  uint32_t* hist = nullptr;
  uint32_t* sums = nullptr;
  int64_t cap_n = 0;
  bool wide = false;
};
void sort_work_alloc(SortWork& w, int64_t n, bool wide, Arena& a);
// The same buffers carved out of caller memory at base (256-byte aligned);
// returns the bytes they take (base may be null to size them only).
int64_t sort_work_carve(SortWork& w, void* base, int64_t n, bool wide);

// Stable LSD radix sort of (key, value) pairs on bits [0, key_bits), in place.
void radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int key_bits, SortWork& w,
                    hipStream_t s);
void radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int key_bits, SortWork& w,
                    hipStream_t s);

// Number of uint32 tile sums exclusive_scan_u32 needs for n elements.
int64_t scan_sums_needed(int64_t n);
// Exclusive scan of n uint32 values in place; the total goes to out_total
// (device) when it is not null.  sums: scratch of scan_sums_needed(n).
void exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* out_total, uint32_t* sums,
                        hipStream_t s);

// keys[i] = SplitMix64 output number i+1 from state seed; vals[i] = i.
void splitmix_keys(uint64_t seed, int64_t n, uint64_t* keys, uint32_t* vals, hipStream_t s);

// dst[i*ld_dst + c] = src[idx[i]*ld_src + c] for c < dim, zero for dim <= c < ld_dst.
void gather_rows(const float* src, int ld_src, const uint32_t* idx, int64_t n, int dim,
                 float* dst, int ld_dst, hipStream_t s);
// Same with int32 indices.
void gather_rows_i32(const float* src, int ld_src, const int32_t* idx, int64_t n, int dim,
                     float* dst, int ld_dst, hipStream_t s);
// dst[i*ld_dst + c] = src[i*ld_src + c] (c < dim), zero padding to ld_dst.
void copy_rows(const float* src, int ld_src, int64_t n, int dim, float* dst, int ld_dst,
               hipStream_t s);

// out[i] = sum_c x[i*ld + c]^2 in float32 (fixed order).
void row_norms(const float* x, int ld, int64_t n, float* out, hipStream_t s);

// Offsets of the runs of a sorted key array: off[p] = first i with keys[i] >= p,
// for p in [0, n_bins]; off[n_bins] = n.
void offsets_from_sorted(const uint32_t* keys, int64_t n, int64_t n_bins, uint32_t* off,
                         hipStream_t s);

// *count (device) := the number of i with a[i] != b[i]
void count_changed(const int32_t* a, const int32_t* b, int64_t n, uint32_t* count,
                   hipStream_t s);
// flag (device) := 1 when some a[i] lies outside [0, bound), else 0
void check_range_i32(const int32_t* a, int64_t n, int64_t bound, uint32_t* flag,
                     hipStream_t s);
// out[i] = map[in[i]]
void map_u32(const uint32_t* map, const uint32_t* in, int64_t n, uint32_t* out, hipStream_t s);
// out[idx[i]] = i
void scatter_iota(const uint32_t* idx, int64_t n, uint32_t* out, hipStream_t s);
// out[i] = src[idx[i]]
void gather_u32(const uint32_t* src, const uint32_t* idx, int64_t n, uint32_t* out,
                hipStream_t s);
void iota_u32(uint32_t* out, int64_t n, hipStream_t s);
void fill_u32(uint32_t* out, int64_t n, uint32_t v, hipStream_t s);

// ------------------------------------------------------------ k-means
// (kmeans.hip)

struct ChunkPlan {
  int n_chunks = 0;
  int k = 0;
  int64_t n_items = 0;
  int64_t max_chunk = 0;
  std::vector<int64_t> off;  // host copy, n_chunks + 1
  int64_t* d_off = nullptr;  // device copy
};

struct KmeansWork {
  // device scratch sized for one level
  uint32_t* sort_keys = nullptr;
  uint32_t* sort_vals = nullptr;
  SortWork sort;
  uint32_t* member_off = nullptr;  // n_protos + 1
  double* proto_inertia = nullptr; // n_protos
  uint32_t* refine_count = nullptr; // [0] points with 2-3 candidates, [1] whole group
  uint32_t* small_list = nullptr;   // n_items
  int32_t* small_cand = nullptr;    // 3 * n_items candidate ids, ascending, -1 padded
  uint32_t* full_cnt = nullptr;     // n_chunks: points of each group re-scored on the group
  uint32_t* full_list = nullptr;    // n_items, group c's entries start at the group offset
  uint2* tiles = nullptr;           // (group, 64-point tile) pairs
  uint32_t* tile_total = nullptr;
  double* partial_d = nullptr;      // n_items * full_splits
  int32_t* partial_j = nullptr;
  int full_splits = 1;
  int full_grid = 1;
  float* item_norms = nullptr;
  float* proto_norms = nullptr;
  double* proto_norms64 = nullptr;
  int32_t* slot_proto = nullptr;  // update work item slots (prototype or -1)
  double* upd_sum = nullptr;      // slots x ld FP64 partial sums
  double* upd_inert = nullptr;    // slots
  // BF16 form: rounded copies of the items and prototypes (row stride ldb)
  int precision = MASK_FP32;
  int ldb = 0;
  uint16_t* items_b = nullptr;
  uint16_t* protos_b = nullptr;
  float* proto_norms_b = nullptr;
  // FP8 form: quantised copies (row stride ldq bytes) and per-row scales
  int ldq = 0;
  uint8_t* items_q = nullptr;
  float* items_qs = nullptr;
  uint8_t* protos_q = nullptr;
  float* protos_qs = nullptr;
  float* proto_norms_q = nullptr;  // squared norms of the dequantised prototypes
};

// FP8 (OCP e4m3) rows with one FP32 scale per row: s = max|x| / 448 (1 for a
// zero row), q = e4m3(x / s) rounded to nearest; row stride ldq bytes (a
// multiple of 16), zero padded.  norms (may be null) = FP32 squared norm of
// the dequantised row s*q.  (fp8.hip)
int fp8_stride(int ld);
void quantize_fp8(const float* x, int ld, int64_t n, uint8_t* out, int ldq, float* scale,
                  float* norms, hipStream_t s);
// Assignment of the FP8 form: re-quantise the prototypes, then screen on
// v_mfma_f32_32x32x16_fp8_fp8 (no certification).
void kmeans_assign_fp8(int ld, const ChunkPlan& plan, const float* protos, int32_t* labels,
                       KmeansWork& w, hipStream_t s);

// out[i*ldb + c] = bf16(x[i*ld + c]) (round to nearest even), zero padding;
// norms[i] = FP32 squared norm of the rounded row when norms is not null.
void quantize_bf16(const float* x, int ld, int64_t n, uint16_t* out, int ldb, float* norms,
                   hipStream_t s);

void kmeans_alloc(KmeansWork& w, int64_t n_items, int n_chunks, int k, int ld,
                  Arena& scratch);

// One assignment of every item to its nearest prototype of its chunk
// (plain FP32 form: MFMA screening + direct-form certification).
void kmeans_assign(const float* items, int ld, int dim, const ChunkPlan& plan,
                   const float* protos, int32_t* labels, KmeansWork& w, int metric,
                   hipStream_t s);
// Update: new prototypes (mean of members; unchanged when empty), their
// norms, and the inertia of the assignment under the old prototypes
// (inertia_out[c] for chunk c, float64, may be null).
void kmeans_update(const float* items, int ld, int dim, const ChunkPlan& plan,
                   const int32_t* labels, float* protos, KmeansWork& w, int metric,
                   double* inertia_out, hipStream_t s);
// FP32 and FP64 squared norms of the prototypes (after init or import).
void kmeans_proto_norms(const float* protos, int ld, int64_t n_protos, KmeansWork& w,
                        hipStream_t s);
// Prototype c*k+j := item off[c] + j mod (size of group c).
void kmeans_init_first(const float* items, int ld, const ChunkPlan& plan, float* protos,
                       hipStream_t s);

// ------------------------------------------------------------ CSR rows
// (sparse.hip)

// Device CSR matrix: n rows over `cols` columns, int64 row pointers, column
// ids distinct within a row, FP32 values.
struct Csr {
  int64_t n = 0;
  int cols = 0;
  int64_t nnz = 0;
  int64_t* ptr = nullptr;
  int32_t* col = nullptr;
  float* val = nullptr;
};

// out = rows idx[0..n) of src, in that order (new arrays from `a`).
void csr_gather(const Csr& src, const uint32_t* idx, int64_t n, Csr& out, Arena& a,
                Arena& scratch, hipStream_t s);
// CSR of a dense row-major matrix (n x ld, the first `cols` columns), zeros dropped.
void csr_from_dense(const float* x, int ld, int64_t n, int cols, Csr& out, Arena& a,
                    Arena& scratch, hipStream_t s);
// FP64 squared norm of every CSR row / dense row.
void csr_norms64(const Csr& x, double* out, hipStream_t s);
void dense_norms64(const float* x, int ld, int64_t n, int cols, double* out, hipStream_t s);
// Checks that column ids are in range and strictly increasing within each
// row and that the row pointers are non-decreasing; flag (device) set to 1
// on a violation.
void csr_validate(const int64_t* ptr, const int32_t* col, int64_t n, int cols, int64_t nnz,
                  uint32_t* flag, hipStream_t s);

// Lloyd on CSR items (chunk-contiguous rows): prototypes dense row-major
// (n_chunks*k x ld, zero padded; init: device rows of the same shape or null
// for the first k items of every group), FP64 expanded-form distances, FP64
// means.  inertia_log: device [iters * n_chunks] or null.
void kmeans_sparse(const Csr& items, int ld, int n_chunks, int k, int iters, const float* init,
                   float* protos, int32_t* labels, double* inertia_log, Arena& scratch,
                   hipStream_t s,
                   const char* level_scope = nullptr);

// ------------------------------------------------------------ descent
// (query.hip)

struct LevelView {
  const float* protos;       // n x ld, position order (null for CSR data)
  const uint16_t* protos_b;  // n x ldb BF16 copy (BF16 form), position order
  const uint8_t* protos_q;   // n x ldq FP8 copy (FP8 form), position order
  const float* scale_q;      // FP32 scale of each FP8 row
  const int32_t* orig;       // position -> chunk-major id (data row id at level 0)
  const int32_t* inv;        // chunk-major id -> position (levels >= 1)
  const uint32_t* child_off; // n + 1 offsets into the level below (levels >= 1)
  // CSR index: level 0 rows in CSR (leaf order) and the FP64 squared norm of
  // every row of every level (position order)
  const int64_t* sp_ptr;
  const int32_t* sp_col;
  const float* sp_val;
  const double* norm64;
  int64_t n;
};

struct DescentArgs {
  LevelView lv[kMaxLevels + 1];  // lv[0] = data (leaf order), lv[l] = level l
  const int32_t* inv0;           // data row id -> leaf position (BF16 re-rank)
  int n_levels;
  int dim;
  int ld;
  int ldb;
  int ldq;  // FP8 row stride in bytes (FP8 form)
  int metric;
  int precision;
  int rerank_factor;
  int64_t max_leaf_children;  // largest child count of a level-1 prototype
  bool sparse;                // CSR index (dim = number of columns)
};

struct QueryArgs {
  const float* Q;
  int ldq;
  // CSR queries (sparse index): row pointers, column ids, values (device)
  const int64_t* q_ptr;
  const int32_t* q_col;
  const float* q_val;
  int64_t nq;
  int k, r;                 // uniform values, or the maxima when k_arr / r_arr are set
  int r_lev[kMaxLevels + 1];  // beam per level (index = level), 0 = use r
  // beam profile of a ragged batch (index = level): query i keeps
  // ceil(r_i * beam_e8[level] / 8) prototypes there; 0 = r_i
  int beam_e8[kMaxLevels + 1];
  const int32_t* k_arr;     // per-query k (device) or null
  const int32_t* r_arr;     // per-query r (device) or null
  const int64_t* out_off;   // per-query output offset (device) or null: qi * k
  int32_t* out_ids;
  float* out_dist;
  int32_t* sel;
  unsigned long long* rows;
  // range search: radius per query (device) or null, and the number of data
  // rows within it per query (device)
  const float* radius;
  int32_t* out_count;
  // point query: the level-1 prototype kept (chunk-major id, -1 if none),
  // with r = 1 (device) or null
  int32_t* out_leaf;
  // insertion descent: above level 1, prototypes without children are not
  // candidates
  bool skip_empty;
  // screened levels (precision form): squared distances of every query of
  // the launch to every prototype of the level, row-major (query, position)
  // with rows scr_ld[level] floats apart; null = rows are read and compared
  // in the descent
  const float* scr[kMaxLevels + 1];
  int64_t scr_ld[kMaxLevels + 1];
  // launch order (null = workgroup b takes query b): workgroup b takes query
  // order[(b % kXcds) * per_xcd + b / kXcds], so each XCD works through a
  // contiguous run of `order`
  const uint32_t* order;
  int64_t per_xcd;
  // Leaf-batched data layer (BF16 form, k-NN): leaf_mode 1 stops after the
  // level-1 selection and writes each query's kept leaves (leaf_cap slots
  // per query); leaf_mode 2 starts at the data layer from them and reads the
  // candidates' BF16 distances from cand (query i's list at cand_off[i], in
  // the order of its kept leaves) instead of evaluating the rows.
  int leaf_mode;
  int leaf_cap;
  uint32_t* leaf_b0;         // first data-row position (leaf order) of the leaf
  uint32_t* leaf_cnt;        // its rows
  uint32_t* leaf_off;        // its first candidate in the query's list
  uint32_t* leaf_key;        // its level-1 position (n_1 for an empty slot)
  uint32_t* leaf_val;        // query * leaf_cap + slot
  uint32_t* n_kept;          // leaves kept per query
  uint32_t* n_cand;          // candidates per query (mode 1)
  const uint32_t* cand_off;  // exclusive prefix of n_cand (mode 2)
  const float* cand;
};

// XCDs of an MI355X; workgroups are dispatched to them round-robin
constexpr int kXcds = 8;

// Launch order of a query batch for the descent: queries sorted by the end
// of their greedy path through the screened levels (top .. low, scores
// S[l] with rows ld[l] apart, children of level l + 1's position p at
// child_off[l + 1][p] ..), so queries in one subtree run together on one
// XCD.  keys, order: device uint32[nq]; n_low <= 16384.
struct ScreenPath {
  const float* S[kMaxLevels + 1];
  int64_t ld[kMaxLevels + 1];
  const uint32_t* child_off[kMaxLevels + 1];
  int top, low;
  int64_t n_top, n_low;
};
void order_queries(const ScreenPath& sp, int64_t nq, uint32_t* keys, uint32_t* order,
                   hipStream_t s);

void descent(const DescentArgs& a, const QueryArgs& qa, hipStream_t s);
// BF16 distances of every (query, kept leaf) pair: the n_pairs pairs sorted
// by leaf (pair_key: the leaf's position, n_1 for an empty slot; pair_val:
// query * cap + slot) in chunks of 32 per workgroup: the distance of row r
// of the leaf to query q goes to cand[cand_off[q] + leaf_off[q * cap + slot]
// + r], bit for bit the value the descent's data layer computes for it.
void leaf_scan(const DescentArgs& a, const uint32_t* pair_key, const uint32_t* pair_val,
               int64_t n_pairs, int cap, const uint32_t* leaf_off, const uint32_t* cand_off,
               const float* Q, int ldq, float* cand, hipStream_t s);
// Largest FP32 row stride of the leaf-batched data layer (its queries are
// staged in LDS).
constexpr int kMaxBatchedLd = 256;
// The data layer of the leaf-batched descent (leaf_mode 2 arguments) with
// one wave per query, for uniform k and re-rank sets of at most 192 and
// level-1 beams of at most 128 on an L2 BF16 index; false (nothing
// launched) otherwise.  Results equal descent()'s bit for bit.
bool leaf_select(const DescentArgs& a, const QueryArgs& qa, hipStream_t s);
// The prototype levels of the leaf-batched descent (leaf_mode 1 arguments)
// with one wave per query, for uniform beams of at most 192 per level and a
// level-1 beam (leaf_cap) of at most 128 on an L2 BF16 index; false (nothing
// launched) otherwise.  The kept sets equal descent()'s; their slot order may
// differ.
bool level_select(const DescentArgs& a, const QueryArgs& qa, hipStream_t s);

// Screening of one prototype level for a batch of queries on
// v_mfma_f32_32x32x16_bf16: S[i * n + p] = max(0, |q_i|^2 + |c~_p|^2 -
// 2 q_i . c~_p), c~ the BF16 rows (position order, stride ldb), pn their
// FP32 squared norms, q_i FP32 (split into two BF16 terms).
void level_scores(const float* Q, int ldq, int64_t nq, int dim, const uint16_t* protos_b,
                  int ldb, int64_t n, const float* pn, float* S, int64_t ldS, hipStream_t s);

// Exact-match scan of the point query: match[i] = lowest data row id under
// level-1 prototype leaf[i] whose coordinates equal query i's, else -1.
void point_match(const DescentArgs& a, const float* Q, int ldq, int64_t nq,
                 const int32_t* leaf, int32_t* match, hipStream_t s);

// ------------------------------------------------------------ seeding
// (seeding.hip)

// k-means++ seeds of every group of the plan (chunk-major prototypes, row
// stride ld <= 256); chosen (device int32[C * k], may be null) receives the
// item index of each seed.  Draw t of group c uses the SplitMix64 output at
// counter (level << 40) + c * k + t.
void kmeanspp_init(const float* items, int ld, int dim, const ChunkPlan& plan, uint64_t seed,
                   int level, float* protos, int32_t* chosen, Arena& scratch, hipStream_t s);

// ------------------------------------------------------------ insertion
// (relocate.hip)

// par1[orig0[q]] = orig1[p] for every leaf-order position q in the child
// range of level-1 position p (the level-1 parent of every data row).
void leaf_parents(const uint32_t* child_off1, int64_t n1, const int32_t* orig1,
                  const int32_t* orig0, int64_t n0, int32_t* par1, hipStream_t s);
// Keys of the level-0 order after an insertion: positions j < n of perm0
// get 2 * (their group), new rows i get 2 * (leaf[i] / k0) + 1 (value n + i).
void insert_group_keys(const int32_t* perm0, const int64_t* goff, int C, int64_t n,
                       const int32_t* leaf, int64_t m, int k0, uint32_t* keys, uint32_t* vals,
                       hipStream_t s);
// keys[j] = inv1[par1[ids[j]]] (leaf position of every id, in the given order)
void leaf_keys(const uint32_t* ids, int64_t n, const int32_t* par1, const int32_t* inv1,
               uint32_t* keys, hipStream_t s);
// Rows of ids from two sources: id < n0 reads rows0[pos0[id]], else
// rows1[id - n0] (row stride ld1); out is dense with stride ld.
void gather_two(const uint32_t* ids, int64_t n, const float* rows0, const int32_t* pos0,
                int64_t n0, const float* rows1, int ld1, int dim, int ld, float* out,
                hipStream_t s);
// dst[pos[t]] = src[t] for rows of stride ld
void scatter_rows(const float* src, const uint32_t* pos, int64_t n, int ld, float* dst,
                  hipStream_t s);
// par1[ids[i]] = group[labels[i] / k0] * k0 + labels[i] % k0
void relabel(const uint32_t* ids, const int32_t* labels, int64_t n, const int32_t* group, int k0,
             int32_t* par1, hipStream_t s);
// counts[par[i]] += 1
void count_labels(const int32_t* par, int64_t n, uint32_t* counts, int64_t n_bins,
                  hipStream_t s);

// ------------------------------------------------------------ relocation
// (relocate.hip)

// One relocation step: data rows with wrong[i] != 0 and leaf[i] >= 0 join
// level-0 group leaf[i] / k0; the rest stay.  perm0 / goff (device, C + 1
// entries) give the current level-0 order and groups.  Writes the stable
// order by (new group, joined) to perm_out and the run boundaries of the 2C
// keys to off2 (device, 2C + 1); *bad (device) becomes non-zero when a leaf
// lies outside [0, C * k0).
void relocate_order(const int32_t* perm0, const int64_t* goff, int C, int64_t n, int k0,
                    const int32_t* leaf, const int32_t* wrong, int32_t* perm_out,
                    uint32_t* off2, uint32_t* bad, Arena& scratch, hipStream_t s);

}  // namespace mask

// Host-visible structure behind the opaque mask_index handle.
struct mask_index {
  mask::Arena mem;
  int64_t n = 0;
  int dim = 0;
  int ld = 0;
  int metric = 0;
  int precision = 0;
  int n_levels = 0;
  std::vector<mask_level> levels;
  std::vector<int64_t> level_n;  // level_n[0] = n, level_n[l] = prototypes at level l
  // device arrays; index 0 = data in leaf order
  float* protos[mask::kMaxLevels + 1] = {};
  uint16_t* protos_b[mask::kMaxLevels + 1] = {};  // BF16 copies (BF16 form)
  float* norm_b[mask::kMaxLevels + 1] = {};       // their FP32 squared norms (levels >= 1)
  uint8_t* protos_q[mask::kMaxLevels + 1] = {};   // FP8 copies (FP8 form)
  float* scale_q[mask::kMaxLevels + 1] = {};
  int ldq = 0;
  int ldb = 0;
  int rerank_factor = 4;
  int32_t* inv0 = nullptr;  // data row id -> leaf position (BF16 form)
  int64_t max_children[mask::kMaxLevels + 1] = {};  // per level, largest child count
  // leaf_top[j]: data rows in the j largest level-1 leaves (j <= kMaxBeam),
  // the bound of one query's candidates at a level-1 beam of j
  std::vector<int64_t> leaf_top;
  int32_t* orig[mask::kMaxLevels + 1] = {};
  int32_t* inv[mask::kMaxLevels + 1] = {};
  uint32_t* child_off[mask::kMaxLevels + 1] = {};
  int64_t refined_last = 0;
  // CSR index: data rows in CSR, leaf order; FP64 squared norms per level
  bool sparse = false;
  int64_t* sp_ptr = nullptr;
  int32_t* sp_col = nullptr;
  float* sp_val = nullptr;
  int64_t sp_nnz = 0;
  double* norm64[mask::kMaxLevels + 1] = {};
  // level-0 order (data row ids) and group boundaries the index was built
  // with (dense builds; null / empty for imported indexes)
  int32_t* perm0 = nullptr;
  std::vector<int64_t> group_off0;
  int lloyd_iters = 0;  // of the build; used by the local rebuild after insertion
  explicit mask_index(const mask_allocator* a, hipStream_t s) : mem(a, s) {}
};

// Host runtime behind the C ABI of include/mask.h: argument checks, the
// level loop of Algorithm 1, the layout of the finished index, and the
// entry points.
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <cstring>
#include <memory>
#include <new>

#include "internal.hpp"

namespace mask {

namespace {
thread_local std::string g_last_error;

struct TimingState {
  std::mutex mu;
  bool on = false;
  struct Rec { std::string name; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<std::pair<std::string, hipEvent_t>> open;  // started, not yet ended
  // [1..2] refine counts; for level slot l of the k-means++ updates,
  // [4 + 3 l] rows not ruled out by the triangle inequality, [5 + 3 l] rows
  // read exactly (FP32), [6 + 3 l] D^2 lowered; then the shards of the
  // descent rows and of the (query, row) pairs of the leaf-batched data
  // layer ([0] and [3] unused)
  unsigned long long* rows = nullptr;
};
constexpr int kCounters = 4 + 3 * kSeedSlots;
constexpr int kRowShards0 = kCounters;                   // descent rows
constexpr int kLeafShards0 = kCounters + kCounterShards;  // leaf-scan pairs
constexpr int kCounterSlots = kCounters + 2 * kCounterShards;
TimingState& timing() {
  static TimingState t;
  return t;
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

bool timing_enabled() { return timing().on; }

void timing_record(const char* name, hipStream_t s, bool start) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  if (start) {
    t.open.push_back({name, e});
  } else {
    for (size_t i = t.open.size(); i-- > 0;) {
      if (t.open[i].first == name) {
        t.recs.push_back({name, t.open[i].second, e});
        t.open.erase(t.open.begin() + i);
        return;
      }
    }
    (void)hipEventDestroy(e);
  }
}

const char* level_scope_name(const char* prefix, int level) {
  static std::mutex mu;
  static std::map<std::string, std::vector<std::string>> names;
  std::lock_guard<std::mutex> g(mu);
  auto& v = names[prefix];
  if (v.empty())
    for (int l = 0; l <= kMaxLevels; ++l) v.push_back(std::string(prefix) + std::to_string(l));
  return v[std::min(std::max(level, 0), kMaxLevels)].c_str();
}

unsigned long long* timing_row_counter() {
  return timing().on && timing().rows ? timing().rows + kRowShards0 : nullptr;
}
unsigned long long* timing_refine_counter() {
  return timing().on && timing().rows ? timing().rows + 1 : nullptr;
}
unsigned long long* timing_seed_counter(int slot) {
  return timing().on && timing().rows ? timing().rows + 4 + 3 * slot : nullptr;
}
unsigned long long* timing_leaf_counter() {
  return timing().on && timing().rows ? timing().rows + kLeafShards0 : nullptr;
}

namespace {

int bits_for(int64_t n) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  return b;
}

int round_up4(int d) { return (d + 3) & ~3; }

// Prototype levels up to this size are screened by one BF16 GEMM per query
// batch in mask_query_screened.
constexpr int64_t kScreenMax = 16384;
// score rows of a screened level start on 128-byte lines
inline int64_t screen_ld(int64_t n) { return (n + 31) / 32 * 32; }
int bf16_stride(int ld) { return (ld + 7) & ~7; }

// split() of Algorithm 1: n_chunks contiguous groups whose sizes differ by at
// most one, the larger ones first.
std::vector<int64_t> split_offsets(int64_t n, int n_chunks) {
  std::vector<int64_t> off(n_chunks + 1);
  const int64_t base = n / n_chunks, extra = n % n_chunks;
  off[0] = 0;
  for (int c = 0; c < n_chunks; ++c) off[c + 1] = off[c] + base + (c < extra ? 1 : 0);
  return off;
}

// offs: explicit group boundaries (n_chunks + 1, rising from 0 to n_items)
// or null for split()
void make_plan(ChunkPlan& plan, int64_t n_items, int n_chunks, int k, Arena& a, hipStream_t s,
               const std::vector<int64_t>* offs = nullptr) {
  plan.n_chunks = n_chunks;
  plan.k = k;
  plan.n_items = n_items;
  plan.off = offs ? *offs : split_offsets(n_items, n_chunks);
  plan.max_chunk = 0;
  for (int c = 0; c < n_chunks; ++c)
    plan.max_chunk = std::max(plan.max_chunk, plan.off[c + 1] - plan.off[c]);
  plan.d_off = a.alloc<int64_t>(n_chunks + 1);
  MASK_HIP(hipMemcpyAsync(plan.d_off, plan.off.data(), (n_chunks + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
}

void check_dense(const mask_matrix* m, const char* what) {
  MASK_CHECK(m != nullptr, std::string(what) + " is NULL");
  MASK_CHECK(m->layout == MASK_DENSE, std::string(what) + ": only DENSE is supported here");
  MASK_CHECK(m->n >= 0 && m->dim >= 1, std::string(what) + ": bad shape");
  MASK_CHECK(m->ld == 0 || m->ld >= m->dim, std::string(what) + ": ld < dim");
  MASK_CHECK(m->n == 0 || m->x != nullptr, std::string(what) + ": x is NULL");
}

int ld_of(const mask_matrix* m) { return m->ld ? m->ld : m->dim; }

void check_csr(const mask_matrix* m, const char* what) {
  MASK_CHECK(m != nullptr, std::string(what) + " is NULL");
  MASK_CHECK(m->layout == MASK_CSR, std::string(what) + ": CSR expected");
  MASK_CHECK(m->n >= 0 && m->dim >= 1, std::string(what) + ": bad shape");
  MASK_CHECK(m->nnz >= 0 && m->nnz < ((int64_t)1 << 31), std::string(what) + ": nnz out of range");
  MASK_CHECK(m->n == 0 || m->indptr != nullptr, std::string(what) + ": indptr is NULL");
  MASK_CHECK(m->nnz == 0 || (m->indices && m->values), std::string(what) + ": arrays are NULL");
  if (m->dim > kMaxSparseDim)
    throw Error{MASK_ERR_UNSUPPORTED, std::string(what) + ": more than 16384 columns"};
}

Csr csr_view(const mask_matrix* m) {
  Csr c;
  c.n = m->n;
  c.cols = m->dim;
  c.nnz = m->nnz;
  c.ptr = const_cast<int64_t*>(m->indptr);
  c.col = const_cast<int32_t*>(m->indices);
  c.val = const_cast<float*>(m->values);
  return c;
}

// Device-side structure check of a CSR argument (synchronises the stream).
void validate_csr(const mask_matrix* m, const char* what, Arena& scratch, hipStream_t s) {
  uint32_t* flag = scratch.alloc<uint32_t>(1);
  csr_validate(m->indptr, m->indices, m->n, m->dim, m->nnz, flag, s);
  uint32_t h = 0;
  MASK_HIP(hipMemcpyAsync(&h, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  MASK_HIP(hipStreamSynchronize(s));
  MASK_CHECK(h == 0, std::string(what) +
                         ": indptr must rise from 0 to nnz and every row's column ids must "
                         "be strictly increasing and below dim");
}

// A caller's level-0 order must name data rows only (synchronises the
// stream); it is then used as a gather index.
void check_perm(const uint32_t* perm, int64_t n, Arena& scratch, hipStream_t s) {
  uint32_t* flag = scratch.alloc<uint32_t>(1);
  check_range_i32(reinterpret_cast<const int32_t*>(perm), n, n, flag, s);
  uint32_t h = 0;
  MASK_HIP(hipMemcpyAsync(&h, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  MASK_HIP(hipStreamSynchronize(s));
  MASK_CHECK(h == 0, "perm holds an id outside [0, n)");
}

void check_levels(int64_t n, int n_levels, const mask_level* levels, std::vector<int64_t>& sizes) {
  MASK_CHECK(n_levels >= 1 && n_levels <= kMaxLevels, "n_levels must be in [1, 16]");
  MASK_CHECK(levels != nullptr, "levels is NULL");
  sizes.assign(n_levels + 1, 0);
  sizes[0] = n;
  for (int l = 0; l < n_levels; ++l) {
    const int64_t items = sizes[l];
    const int C = levels[l].n_chunks, k = levels[l].k;
    MASK_CHECK(C >= 1 && k >= 1, "level with n_chunks < 1 or k < 1");
    MASK_CHECK(items >= C, "a level with more chunks than items");
    sizes[l + 1] = (int64_t)C * k;
    MASK_CHECK(sizes[l + 1] < ((int64_t)1 << 31), "level too large");
  }
}

mask_status fail(const Error& e) {
  set_error(e.msg);
  return e.status;
}

// Orders every level so that the children of each prototype are contiguous
// one level down, top-down: the top level keeps chunk-major order; the items
// of each level below are stably sorted by the position of their parent.
// labels[l] (l = 1..L) holds the chunk-major parent id of every item of level
// l-1 in that level's build order; items0_orig maps level-0 build order to
// data row ids; protos_cm[l] are the chunk-major prototypes.
// leaf_top from a host copy of the level-1 child offsets.
void set_leaf_top(mask_index& ix, const std::vector<uint32_t>& off) {
  const int64_t n1 = (int64_t)off.size() - 1;
  std::vector<int64_t> sz((size_t)std::max<int64_t>(n1, 0));
  for (int64_t p = 0; p < n1; ++p) sz[p] = (int64_t)off[p + 1] - off[p];
  const int64_t m = std::min<int64_t>(n1, kMaxBeamCsr);
  std::partial_sort(sz.begin(), sz.begin() + m, sz.end(), std::greater<int64_t>());
  ix.leaf_top.assign((size_t)m + 1, 0);
  for (int64_t j = 0; j < m; ++j) ix.leaf_top[j + 1] = ix.leaf_top[j] + sz[j];
}

void finalize_layout(mask_index& ix, const std::vector<int32_t*>& labels,
                     const std::vector<float*>& protos_cm, const float* items0,
                     const uint32_t* items0_orig, Arena& scratch, hipStream_t s,
                     const Csr* items0_csr = nullptr) {
  const int L = ix.n_levels;
  const int ld = ix.ld, dim = ix.dim;
  int64_t max_items = 0;
  for (int l = 0; l <= L; ++l) max_items = std::max(max_items, ix.level_n[l]);
  uint32_t* keys = scratch.alloc<uint32_t>(max_items);
  uint32_t* ord = scratch.alloc<uint32_t>(max_items);
  SortWork sw;
  sort_work_alloc(sw, max_items, false, scratch);

  // top level: chunk-major order
  const int64_t nL = ix.level_n[L];
  ix.protos[L] = ix.mem.alloc<float>(nL * ld);
  copy_rows(protos_cm[L], ld, nL, ld, ix.protos[L], ld, s);
  ix.orig[L] = ix.mem.alloc<int32_t>(nL);
  ix.inv[L] = ix.mem.alloc<int32_t>(nL);
  iota_u32(reinterpret_cast<uint32_t*>(ix.orig[L]), nL, s);
  iota_u32(reinterpret_cast<uint32_t*>(ix.inv[L]), nL, s);

  for (int l = L; l >= 1; --l) {
    const int64_t n_items = ix.level_n[l - 1];
    const int64_t n_par = ix.level_n[l];
    // key = position of the parent
    map_u32(reinterpret_cast<const uint32_t*>(ix.inv[l]),
            reinterpret_cast<const uint32_t*>(labels[l]), n_items, keys, s);
    iota_u32(ord, n_items, s);
    radix_sort_u32(keys, ord, n_items, bits_for(n_par), sw, s);
    ix.child_off[l] = ix.mem.alloc<uint32_t>(n_par + 1);
    offsets_from_sorted(keys, n_items, n_par, ix.child_off[l], s);
    {
      std::vector<uint32_t> off(n_par + 1);
      MASK_HIP(hipMemcpyAsync(off.data(), ix.child_off[l], (n_par + 1) * sizeof(uint32_t),
                              hipMemcpyDeviceToHost, s));
      MASK_HIP(hipStreamSynchronize(s));
      int64_t mx = 0;
      for (int64_t p = 0; p < n_par; ++p) mx = std::max<int64_t>(mx, off[p + 1] - off[p]);
      ix.max_children[l] = mx;
      if (l == 1) set_leaf_top(ix, off);
    }
    ix.orig[l - 1] = ix.mem.alloc<int32_t>(n_items);
    if (l - 1 >= 1 || !items0_csr) ix.protos[l - 1] = ix.mem.alloc<float>(n_items * ld);
    if (l - 1 == 0 && items0_csr) {
      // CSR data: rows in leaf order
      Csr leaf;
      csr_gather(*items0_csr, ord, n_items, leaf, ix.mem, scratch, s);
      ix.sp_ptr = leaf.ptr;
      ix.sp_col = leaf.col;
      ix.sp_val = leaf.val;
      ix.sp_nnz = leaf.nnz;
      gather_u32(items0_orig, ord, n_items, reinterpret_cast<uint32_t*>(ix.orig[0]), s);
    } else if (l - 1 >= 1) {
      gather_rows(protos_cm[l - 1], ld, ord, n_items, ld, ix.protos[l - 1], ld, s);
      MASK_HIP(hipMemcpyAsync(ix.orig[l - 1], ord, n_items * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s));
      ix.inv[l - 1] = ix.mem.alloc<int32_t>(n_items);
      scatter_iota(ord, n_items, reinterpret_cast<uint32_t*>(ix.inv[l - 1]), s);
    } else {
      gather_rows(items0, ld, ord, n_items, ld, ix.protos[0], ld, s);
      gather_u32(items0_orig, ord, n_items, reinterpret_cast<uint32_t*>(ix.orig[0]), s);
    }
  }
  (void)dim;
  if (ix.sparse) {
    // FP64 norms of the dense prototype rows (position order)
    for (int l = 1; l <= L; ++l) {
      ix.norm64[l] = ix.mem.alloc<double>(ix.level_n[l]);
      dense_norms64(ix.protos[l], ld, ix.level_n[l], ix.dim, ix.norm64[l], s);
    }
  }
  if (ix.precision == MASK_FP8_E4M3) {
    // FP8 copy and scales of the data layer (prototype levels are read in
    // FP32), and the data row -> leaf position map used by the FP32 re-rank
    ix.ldq = fp8_stride(ld);
    for (int l = 0; l <= 0; ++l) {
      ix.protos_q[l] = ix.mem.alloc<uint8_t>(ix.level_n[l] * ix.ldq);
      ix.scale_q[l] = ix.mem.alloc<float>(ix.level_n[l]);
      quantize_fp8(ix.protos[l], ld, ix.level_n[l], ix.protos_q[l], ix.ldq, ix.scale_q[l],
                   nullptr, s);
    }
    ix.inv0 = ix.mem.alloc<int32_t>(ix.level_n[0]);
    scatter_iota(reinterpret_cast<const uint32_t*>(ix.orig[0]), ix.level_n[0],
                 reinterpret_cast<uint32_t*>(ix.inv0), s);
  }
  if (ix.precision == MASK_BF16) {
    // BF16 copies of every level in position order, and the data row -> leaf
    // position map used by the FP32 re-rank
    ix.ldb = bf16_stride(ld);
    for (int l = 0; l <= L; ++l) {
      ix.protos_b[l] = ix.mem.alloc<uint16_t>(ix.level_n[l] * ix.ldb);
      if (l >= 1) ix.norm_b[l] = ix.mem.alloc<float>(ix.level_n[l]);
      quantize_bf16(ix.protos[l], ld, ix.level_n[l], ix.protos_b[l], ix.ldb, ix.norm_b[l], s);
    }
    ix.inv0 = ix.mem.alloc<int32_t>(ix.level_n[0]);
    scatter_iota(reinterpret_cast<const uint32_t*>(ix.orig[0]), ix.level_n[0],
                 reinterpret_cast<uint32_t*>(ix.inv0), s);
  }
}

struct BuildState {
  std::vector<int32_t*> labels;   // [L+1], index 0 unused
  std::vector<float*> protos_cm;  // [L+1], index 0 unused
};

// Lloyd at one level: `items` (n_items x ld, chunk-contiguous) -> prototypes
// (chunk-major) and the final labels.  inertia_log: device [iters * C] or null.
void run_level(const float* items, int64_t n_items, int ld, int dim, int C, int k, int iters,
               int metric, int precision, const float* init, float* protos, int32_t* labels,
               double* inertia_log, Arena& scratch, hipStream_t s, int64_t* refined,
               const std::vector<int64_t>* offs = nullptr, int init_method = MASK_INIT_FIRST,
               uint64_t seed = 0, int level = 0) {
  ChunkPlan plan;
  make_plan(plan, n_items, C, k, scratch, s, offs);
  KmeansWork w;
  kmeans_alloc(w, n_items, C, k, ld, scratch);
  if (precision == MASK_BF16 && metric == MASK_L2) {
    w.precision = MASK_BF16;
    w.ldb = bf16_stride(ld);
    w.items_b = scratch.alloc<uint16_t>(n_items * w.ldb);
    w.protos_b = scratch.alloc<uint16_t>((int64_t)C * k * w.ldb);
    w.proto_norms_b = scratch.alloc<float>((int64_t)C * k);
    quantize_bf16(items, ld, n_items, w.items_b, w.ldb, nullptr, s);
  }
  if (precision == MASK_FP8_E4M3 && metric == MASK_L2) {
    w.precision = MASK_FP8_E4M3;
    w.ldq = fp8_stride(ld);
    const int64_t np = (int64_t)C * k;
    w.items_q = scratch.alloc<uint8_t>(n_items * w.ldq);
    w.items_qs = scratch.alloc<float>(n_items);
    w.protos_q = scratch.alloc<uint8_t>(np * w.ldq);
    w.protos_qs = scratch.alloc<float>(np);
    w.proto_norms_q = scratch.alloc<float>(np);
    quantize_fp8(items, ld, n_items, w.items_q, w.ldq, w.items_qs, nullptr, s);
  }
  row_norms(items, ld, n_items, w.item_norms, s);
  if (init) copy_rows(init, ld, (int64_t)C * k, ld, protos, ld, s);
  else if (init_method == MASK_INIT_KMEANSPP)
    kmeanspp_init(items, ld, dim, plan, seed, level, protos, nullptr, scratch, s);
  else kmeans_init_first(items, ld, plan, protos, s);
  kmeans_proto_norms(protos, ld, (int64_t)C * k, w, s);
  auto assign = [&]() {
    // one timing scope per level: "assign_level<l>" counts this level's
    // assignment launches (the FP32 form's refinement included)
    ScopedTiming timing(level_scope_name("assign_level", level), s);
    if (w.precision == MASK_FP8_E4M3) kmeans_assign_fp8(ld, plan, protos, labels, w, s);
    else kmeans_assign(items, ld, dim, plan, protos, labels, w, metric, s);
  };
  // A fixed point ends the iterations early with the same result: when no
  // label changed since the previous iteration, the update reproduces the
  // prototypes, and so does every later iteration.  Checked every fourth
  // iteration (one host synchronisation each).
  const bool watch = iters >= 2;
  int32_t* prev = watch ? scratch.alloc<int32_t>(n_items) : nullptr;
  uint32_t* changed = watch ? scratch.alloc<uint32_t>(iters) : nullptr;
  for (int t = 0; t < iters; ++t) {
    assign();
    if (watch) {
      if (t > 0) count_changed(labels, prev, n_items, changed + t, s);
      MASK_HIP(hipMemcpyAsync(prev, labels, n_items * sizeof(int32_t), hipMemcpyDeviceToDevice,
                              s));
    }
    kmeans_update(items, ld, dim, plan, labels, protos, w, metric,
                  inertia_log ? inertia_log + (int64_t)t * C : nullptr, s);
    if (watch && t > 0 && t % 4 == 0 && t + 1 < iters) {
      uint32_t h = 1;
      MASK_HIP(hipMemcpyAsync(&h, changed + t, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      MASK_HIP(hipStreamSynchronize(s));
      if (h == 0) {
        // the inertia of every remaining iteration equals this one's
        if (inertia_log)
          for (int u = t + 1; u < iters; ++u)
            MASK_HIP(hipMemcpyAsync(inertia_log + (int64_t)u * C, inertia_log + (int64_t)t * C,
                                    C * sizeof(double), hipMemcpyDeviceToDevice, s));
        break;
      }
    }
  }
  assign();
  if (refined) {
    uint32_t cnt = 0;
    MASK_HIP(hipMemcpyAsync(&cnt, w.refine_count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    MASK_HIP(hipStreamSynchronize(s));
    *refined = cnt;
  }
}

// Algorithm 1 on CSR data: level 0 is the permuted CSR rows, every level's
// prototypes are dense rows, and the items of the next level are those
// prototypes as CSR (zeros dropped).
void build_sparse(mask_index& ix, const mask_matrix* data, const mask_build_params* p,
                  const mask_allocator* a, hipStream_t s) {
  const int L = p->n_levels;
  const int64_t n = data->n;
  const int ld = ix.ld;
  const std::vector<int64_t>& sizes = ix.level_n;
  Arena scratch(a, s);
  validate_csr(data, "data", scratch, s);
  uint32_t* perm = scratch.alloc<uint32_t>(n);
  if (p->perm) {
    MASK_HIP(hipMemcpyAsync(perm, p->perm, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    check_perm(perm, n, scratch, s);
  } else {
    uint64_t* keys = scratch.alloc<uint64_t>(n);
    SortWork sw;
    sort_work_alloc(sw, n, true, scratch);
    splitmix_keys(p->seed, n, keys, perm, s);
    radix_sort_u64(keys, perm, n, 64, sw, s);
  }
  Csr items0;
  csr_gather(csr_view(data), perm, n, items0, scratch, scratch, s);
  BuildState st;
  st.labels.assign(L + 1, nullptr);
  st.protos_cm.assign(L + 1, nullptr);
  Csr items = items0;
  for (int l = 1; l <= L; ++l) {
    const int C = p->levels[l - 1].n_chunks, k = p->levels[l - 1].k;
    st.protos_cm[l] = scratch.alloc<float>(sizes[l] * ld);
    st.labels[l] = scratch.alloc<int32_t>(sizes[l - 1]);
    {
      Arena level_scratch(a, s);
      kmeans_sparse(items, ld, C, k, p->lloyd_iters, nullptr, st.protos_cm[l], st.labels[l],
                    nullptr, level_scratch, s, level_scope_name("assign_level", l));
      MASK_HIP(hipStreamSynchronize(s));
    }
    if (l < L) csr_from_dense(st.protos_cm[l], ld, sizes[l], ix.dim, items, scratch, scratch, s);
  }
  finalize_layout(ix, st.labels, st.protos_cm, nullptr, perm, scratch, s, &items0);
  MASK_HIP(hipStreamSynchronize(s));
}

DescentArgs descent_args(const mask_index& ix) {
  DescentArgs a{};
  a.n_levels = ix.n_levels;
  a.dim = ix.dim;
  a.ld = ix.ld;
  a.ldb = ix.ldb;
  a.ldq = ix.ldq;
  a.metric = ix.metric;
  a.precision = ix.precision;
  a.rerank_factor = ix.rerank_factor;
  a.inv0 = ix.inv0;
  a.max_leaf_children = ix.max_children[1];
  a.sparse = ix.sparse;
  for (int l = 0; l <= ix.n_levels; ++l) {
    a.lv[l].norm64 = ix.norm64[l];
    a.lv[l].protos = ix.protos[l];
    a.lv[l].protos_b = ix.protos_b[l];
    a.lv[l].protos_q = ix.protos_q[l];
    a.lv[l].scale_q = ix.scale_q[l];
    a.lv[l].orig = ix.orig[l];
    a.lv[l].inv = ix.inv[l];
    a.lv[l].child_off = ix.child_off[l];
    a.lv[l].n = ix.level_n[l];
  }
  a.lv[0].sp_ptr = ix.sp_ptr;
  a.lv[0].sp_col = ix.sp_col;
  a.lv[0].sp_val = ix.sp_val;
  return a;
}

mask_status query_impl(const mask_index* ix, const mask_matrix* q, int32_t k, int32_t r,
                       const int32_t* k_arr, const int32_t* r_arr, const int64_t* out_off,
                       int32_t* out_ids, float* out_dist, int32_t* sel, void* hip_stream,
                       const int32_t* r_levels = nullptr, const float* radius = nullptr,
                       int32_t* out_count = nullptr, int32_t* out_leaf = nullptr,
                       const int32_t* beam_eighths = nullptr) {
  try {
    MASK_CHECK(ix != nullptr, "index is NULL");
    if (ix->sparse) check_csr(q, "queries (CSR index)");
    else check_dense(q, "queries");
    MASK_CHECK(q->dim == ix->dim, "query dim differs from the index dim");
    MASK_CHECK(k >= 1 && k <= kMaxBeam, "k must be in [1, 2048]");
    // beams above 2048: CSR indexes of at most 12,288 columns only
    const int max_beam = ix->sparse && ix->dim <= kMaxCsrWideDim ? kMaxBeamCsr : kMaxBeam;
    MASK_CHECK(r >= 1 && r <= max_beam,
               ix->sparse ? "r must be in [1, 3072] (in [1, 2048] above 12,288 columns)"
                          : "r must be in [1, 2048]");
    MASK_CHECK(q->n < ((int64_t)1 << 31), "too many queries in one call");
    if (q->n == 0) return MASK_OK;
    MASK_CHECK(out_ids && out_dist, "output pointer is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    QueryArgs qa{};
    if (ix->sparse) {
      qa.q_ptr = q->indptr;
      qa.q_col = q->indices;
      qa.q_val = q->values;
    } else {
      qa.Q = q->x;
      qa.ldq = ld_of(q);
    }
    qa.nq = q->n;
    qa.k = k;
    qa.r = r;
    qa.k_arr = k_arr;
    qa.r_arr = r_arr;
    qa.out_off = out_off;
    qa.out_ids = out_ids;
    qa.out_dist = out_dist;
    qa.sel = sel;
    qa.rows = timing_row_counter();
    qa.out_leaf = out_leaf;
    if (radius) {
      MASK_CHECK(out_count != nullptr, "out_count is NULL");
      if (ix->precision != MASK_FP32 || ix->metric != MASK_L2)
        throw Error{MASK_ERR_UNSUPPORTED, "range search: plain FP32 form, L2 metric"};
      qa.radius = radius;
      qa.out_count = out_count;
    }
    for (int l = 0; l <= kMaxLevels; ++l) qa.r_lev[l] = qa.beam_e8[l] = 0;
    if (beam_eighths) {
      MASK_CHECK(r_arr != nullptr, "a beam profile needs per-query r");
      for (int d = 0; d < ix->n_levels; ++d) {
        const int64_t e8 = beam_eighths[d];
        MASK_CHECK(e8 >= 0 && (r * e8 + 7) / 8 <= kMaxBeam,
                   "beam profile: every level's beam at r_max must be in [1, 2048]");
        qa.beam_e8[ix->n_levels - d] = (int)e8;
      }
    }
    if (r_levels) {
      for (int d = 0; d < ix->n_levels; ++d) {
        MASK_CHECK(r_levels[d] >= 1 && r_levels[d] <= max_beam,
                   ix->sparse ? "beam must be in [1, 3072] (in [1, 2048] above 12,288 columns)"
                              : "beam must be in [1, 2048]");
        qa.r_lev[ix->n_levels - d] = r_levels[d];
      }
    }
    descent(descent_args(*ix), qa, s);
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

}  // namespace
}  // namespace mask

using namespace mask;

extern "C" {

const char* mask_last_error(void) { return g_last_error.c_str(); }

mask_status mask_timing_enable(int32_t on) {
  try {
    TimingState& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    for (auto& r : t.recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto& o : t.open) (void)hipEventDestroy(o.second);
    t.recs.clear();
    t.open.clear();
    if (on && !t.rows) MASK_HIP(hipMalloc(&t.rows, kCounterSlots * sizeof(unsigned long long)));
    if (t.rows) MASK_HIP(hipMemset(t.rows, 0, kCounterSlots * sizeof(unsigned long long)));
    t.on = on != 0;
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

mask_status mask_timing_report(char* buf, int64_t cap, int64_t* needed) {
  try {
    TimingState& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    std::map<std::string, std::pair<int64_t, double>> agg;
    for (auto& r : t.recs) {
      MASK_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      MASK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      auto& a = agg[r.name];
      a.first += 1;
      a.second += ms;
    }
    unsigned long long cnt[kCounterSlots] = {};
    if (t.rows) MASK_HIP(hipMemcpy(cnt, t.rows, sizeof(cnt), hipMemcpyDeviceToHost));
    for (int i = 0; i < kCounterShards; ++i) {
      cnt[0] += cnt[kRowShards0 + i];
      cnt[3] += cnt[kLeafShards0 + i];
    }
    std::ostringstream os;
    for (auto& kv : agg) os << kv.first << " " << kv.second.first << " " << kv.second.second << "\n";
    os << "descent_rows " << cnt[0] << " 0\n";
    os << "refine_small_points " << cnt[1] << " 0\n";
    os << "refine_full_points " << cnt[2] << " 0\n";
    if (cnt[3]) os << "leaf_scan_pairs " << cnt[3] << " 0\n";
    for (int l = 0; l < kSeedSlots; ++l) {
      if (cnt[4 + 3 * l] == 0) continue;
      os << "seeding_rows_read_level" << l << " " << cnt[4 + 3 * l] << " 0\n";
      os << "seeding_rows_exact_level" << l << " " << cnt[5 + 3 * l] << " 0\n";
      os << "seeding_rows_lowered_level" << l << " " << cnt[6 + 3 * l] << " 0\n";
    }
    const std::string txt = os.str();
    if (needed) *needed = (int64_t)txt.size() + 1;
    if (buf && cap > 0) {
      const size_t n = std::min<size_t>(txt.size(), (size_t)cap - 1);
      std::memcpy(buf, txt.data(), n);
      buf[n] = 0;
    }
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

mask_status mask_plan_levels(int64_t n, int32_t length_group, int32_t n_centroids,
                             mask_level* out, int32_t cap, int32_t* n_levels) {
  try {
    MASK_CHECK(n >= 0 && length_group >= 1 && n_centroids >= 1, "bad arguments");
    MASK_CHECK(n_levels != nullptr, "n_levels is NULL");
    MASK_CHECK(n_centroids < length_group, "the schedule does not shrink");
    int count = 0;
    int64_t ngroups = n / length_group;
    while (ngroups >= 1) {
      MASK_CHECK(count < cap, "more levels than cap");
      MASK_CHECK(ngroups < ((int64_t)1 << 31), "too many groups");
      if (out) out[count] = mask_level{(int32_t)ngroups, n_centroids};
      ++count;
      ngroups = (ngroups * n_centroids) / length_group;
    }
    *n_levels = count;
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

mask_status mask_build(const mask_matrix* data, const mask_build_params* p,
                       const mask_allocator* a, void* hip_stream, mask_index** out) {
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    MASK_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    MASK_CHECK(data != nullptr, "data is NULL");
    const bool sparse = data->layout == MASK_CSR;
    if (sparse) check_csr(data, "data");
    else check_dense(data, "data");
    MASK_CHECK(p != nullptr, "params is NULL");
    MASK_CHECK(p->metric == MASK_L2 || p->metric == MASK_L1, "unknown metric");
    MASK_CHECK(p->precision >= MASK_FP32 && p->precision <= MASK_FP8_E4M3, "unknown precision");
    MASK_CHECK(p->lloyd_iters >= 0, "lloyd_iters < 0");
    MASK_CHECK(data->n >= 1 && data->n < ((int64_t)1 << 31), "n must be in [1, 2^31)");
    std::vector<int64_t> sizes;
    check_levels(data->n, p->n_levels, p->levels, sizes);
    if (sparse && (p->metric != MASK_L2 || p->precision != MASK_FP32))
      throw Error{MASK_ERR_UNSUPPORTED, "CSR data: L2 metric, FP32 form only"};
    if (!sparse && data->dim > kMaxDenseDim)
      throw Error{MASK_ERR_UNSUPPORTED, "dense dim above 256"};
    if (p->precision != MASK_FP32 && p->metric != MASK_L2)
      throw Error{MASK_ERR_UNSUPPORTED, "BF16 / FP8 form of L1"};
    MASK_CHECK(p->init == MASK_INIT_FIRST || p->init == MASK_INIT_KMEANSPP, "unknown init");
    if (p->init == MASK_INIT_KMEANSPP && (sparse || p->metric != MASK_L2))
      throw Error{MASK_ERR_UNSUPPORTED, "k-means++ seeding: dense data, L2 metric"};
    std::vector<int64_t> goff0;
    if (p->group_off) {
      if (sparse) throw Error{MASK_ERR_UNSUPPORTED, "CSR data: group_off"};
      const int C0 = p->levels[0].n_chunks;
      goff0.assign(p->group_off, p->group_off + C0 + 1);
      MASK_CHECK(goff0[0] == 0 && goff0[C0] == data->n,
                 "group_off must start at 0 and end at n");
      for (int c = 0; c < C0; ++c)
        MASK_CHECK(goff0[c + 1] > goff0[c], "group_off must rise strictly (no empty group)");
    }

    auto ix = std::make_unique<mask_index>(a, s);
    const int L = p->n_levels;
    ix->n = data->n;
    ix->dim = data->dim;
    ix->ld = round_up4(data->dim);
    ix->metric = p->metric;
    ix->precision = p->precision;
    ix->n_levels = L;
    ix->levels.assign(p->levels, p->levels + L);
    ix->level_n = sizes;
    ix->rerank_factor = p->rerank_factor != 0 ? p->rerank_factor
                                             : (p->precision == MASK_FP8_E4M3 ? 48 : 4);
    const int ld = ix->ld;
    const int64_t n = data->n;
    if (sparse) {
      ix->sparse = true;
      build_sparse(*ix, data, p, a, s);
      *out = ix.release();
      return MASK_OK;
    }

    Arena scratch(a, s);
    // level-0 order
    uint32_t* perm = scratch.alloc<uint32_t>(n);
    if (p->perm) {
      MASK_HIP(hipMemcpyAsync(perm, p->perm, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
      check_perm(perm, n, scratch, s);
    } else {
      uint64_t* keys = scratch.alloc<uint64_t>(n);
      SortWork sw;
      sort_work_alloc(sw, n, true, scratch);
      splitmix_keys(p->seed, n, keys, perm, s);
      radix_sort_u64(keys, perm, n, 64, sw, s);
    }
    float* items0 = scratch.alloc<float>(n * ld);
    gather_rows(data->x, ld_of(data), perm, n, data->dim, items0, ld, s);
    // kept for relocation: the level-0 order and groups of this build
    if (goff0.empty()) goff0 = split_offsets(n, p->levels[0].n_chunks);
    ix->group_off0 = goff0;
    ix->lloyd_iters = p->lloyd_iters;
    ix->perm0 = ix->mem.alloc<int32_t>(n);
    MASK_HIP(hipMemcpyAsync(ix->perm0, perm, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));

    BuildState st;
    st.labels.assign(L + 1, nullptr);
    st.protos_cm.assign(L + 1, nullptr);
    for (int l = 1; l <= L; ++l) {
      const int C = p->levels[l - 1].n_chunks, k = p->levels[l - 1].k;
      const int64_t n_items = sizes[l - 1];
      const float* items = (l == 1) ? items0 : st.protos_cm[l - 1];
      st.protos_cm[l] = scratch.alloc<float>(sizes[l] * ld);
      st.labels[l] = scratch.alloc<int32_t>(n_items);
      Arena level_scratch(a, s);
      run_level(items, n_items, ld, data->dim, C, k, p->lloyd_iters, p->metric, p->precision,
                nullptr, st.protos_cm[l], st.labels[l], nullptr, level_scratch, s,
                l == 1 ? &ix->refined_last : nullptr, l == 1 ? &goff0 : nullptr, p->init,
                p->seed, l);
      MASK_HIP(hipStreamSynchronize(s));
    }
    finalize_layout(*ix, st.labels, st.protos_cm, items0, perm, scratch, s);
    MASK_HIP(hipStreamSynchronize(s));
    *out = ix.release();
    return MASK_OK;
  } catch (const Error& e) {
    if (e.status != MASK_ERR_INVALID && e.status != MASK_ERR_UNSUPPORTED)
      (void)hipStreamSynchronize(s);
    return fail(e);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    return fail(Error{MASK_ERR_NOMEM, "host allocation failed"});
  }
}

mask_status mask_query(const mask_index* ix, const mask_matrix* q, int32_t k, int32_t r,
                       int32_t* out_ids, float* out_dist, void* hip_stream) {
  return query_impl(ix, q, k, r, nullptr, nullptr, nullptr, out_ids, out_dist, nullptr,
                    hip_stream);
}

mask_status mask_query_beams(const mask_index* ix, const mask_matrix* q, int32_t k,
                             const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                             void* hip_stream) {
  if (!r_levels) {
    set_error("r_levels is NULL");
    return MASK_ERR_INVALID;
  }
  int32_t rmax = 1;
  if (ix)
    for (int d = 0; d < ix->n_levels; ++d) rmax = r_levels[d] > rmax ? r_levels[d] : rmax;
  return query_impl(ix, q, k, rmax, nullptr, nullptr, nullptr, out_ids, out_dist, nullptr,
                    hip_stream, r_levels);
}

mask_status mask_screen_bytes(const mask_index* ix, int64_t* bytes_per_query) {
  if (!ix || !bytes_per_query) {
    set_error("NULL argument");
    return MASK_ERR_INVALID;
  }
  int64_t b = 0;
  if (ix->precision == MASK_BF16 && !ix->sparse)
    for (int l = 1; l <= ix->n_levels; ++l)
      if (ix->level_n[l] <= kScreenMax) b += screen_ld(ix->level_n[l]) * (int64_t)sizeof(float);
  if (b) b += 8;  // the launch order: a key and a slot per query
  *bytes_per_query = b;
  return MASK_OK;
}

}  // extern "C"

namespace mask {
namespace {

// Score rows of every screened level for the n queries at Qs (laid out as
// mask_screen_bytes counts them, from S), then the launch order: queries
// near each other in the tree (by their greedy path through the screened
// levels) run together on one XCD.  Sets qa.scr, qa.scr_ld, qa.order and
// qa.per_xcd.
void screen_batch(const mask_index& ix, const float* Qs, int ldq, int64_t n, float* S,
                  uint32_t* keys, uint32_t* order, QueryArgs& qa, hipStream_t s) {
  const int L = ix.n_levels;
  for (int l = 1; l <= L; ++l) {
    if (ix.level_n[l] > kScreenMax) continue;
    const int64_t ldS = screen_ld(ix.level_n[l]);
    level_scores(Qs, ldq, n, ix.dim, ix.protos_b[l], ix.ldb, ix.level_n[l], ix.norm_b[l], S,
                 ldS, s);
    qa.scr[l] = S;
    qa.scr_ld[l] = ldS;
    S += n * ldS;
  }
  if (qa.scr[L]) {  // the screened levels are the top ones
    ScreenPath sp{};
    sp.top = L;
    sp.low = L;
    while (sp.low > 1 && qa.scr[sp.low - 1]) --sp.low;
    for (int l = sp.low; l <= L; ++l) {
      sp.S[l] = qa.scr[l];
      sp.ld[l] = qa.scr_ld[l];
      sp.child_off[l] = ix.child_off[l];
    }
    sp.n_top = ix.level_n[L];
    sp.n_low = ix.level_n[sp.low];
    order_queries(sp, n, keys, order, s);
    qa.order = order;
    qa.per_xcd = (n + kXcds - 1) / kXcds;
  }
}

// mask_query_screened, with the per-level selections written to sel when it
// is not NULL (int32[q->n * n_levels * rmax], as mask_query_beams_debug).
mask_status screened_impl(const mask_index* ix, const mask_matrix* q, int32_t k,
                          const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                          int32_t* sel, void* workspace, int64_t workspace_bytes,
                          void* hip_stream) {
  try {
    MASK_CHECK(ix != nullptr, "index is NULL");
    if (ix->precision != MASK_BF16 || ix->sparse || ix->metric != MASK_L2)
      throw Error{MASK_ERR_UNSUPPORTED, "screened descent: BF16 form of dense L2 data"};
    check_dense(q, "queries");
    MASK_CHECK(q->dim == ix->dim, "query dim differs from the index dim");
    MASK_CHECK(r_levels != nullptr, "r_levels is NULL");
    MASK_CHECK(k >= 1 && k <= kMaxBeam, "k must be in [1, 2048]");
    MASK_CHECK(q->n < ((int64_t)1 << 31), "too many queries in one call");
    const int L = ix->n_levels;
    int rmax = 1;
    for (int d = 0; d < L; ++d) {
      MASK_CHECK(r_levels[d] >= 1 && r_levels[d] <= kMaxBeam, "beam must be in [1, 2048]");
      rmax = std::max(rmax, r_levels[d]);
    }
    if (q->n == 0) return MASK_OK;
    MASK_CHECK(out_ids && out_dist, "output pointer is NULL");
    int64_t per_query = 0;
    for (int l = 1; l <= L; ++l)
      if (ix->level_n[l] <= kScreenMax) per_query += screen_ld(ix->level_n[l]);
    MASK_CHECK(workspace != nullptr || per_query == 0, "workspace is NULL");
    MASK_CHECK(((uintptr_t)workspace & 255) == 0, "workspace must be 256-byte aligned");
    const int64_t query_bytes = per_query ? per_query * (int64_t)sizeof(float) + 8 : 0;
    const int64_t slice =
        per_query ? std::min<int64_t>(q->n, workspace_bytes / query_bytes) : q->n;
    MASK_CHECK(slice >= 1, "workspace smaller than one query's screened distances");
    const int64_t step = std::min<int64_t>(slice, (int64_t)1 << 20);  // grid-size bound
    hipStream_t s = (hipStream_t)hip_stream;
    const DescentArgs da = descent_args(*ix);
    const int ldq = ld_of(q);
    for (int64_t s0 = 0; s0 < q->n; s0 += step) {
      const int64_t len = std::min(step, q->n - s0);
      const float* Qs = q->x + s0 * ldq;
      QueryArgs qa{};
      qa.Q = Qs;
      qa.ldq = ldq;
      qa.nq = len;
      qa.k = k;
      qa.r = rmax;
      qa.out_ids = out_ids + s0 * k;
      qa.out_dist = out_dist + s0 * k;
      qa.sel = sel ? sel + s0 * (int64_t)L * rmax : nullptr;
      qa.rows = timing_row_counter();
      for (int d = 0; d < L; ++d) qa.r_lev[L - d] = r_levels[d];
      float* S = static_cast<float*>(workspace);
      uint32_t* keys = reinterpret_cast<uint32_t*>(S + len * per_query);
      screen_batch(*ix, Qs, ldq, len, S, keys, keys + len, qa, s);
      descent(da, qa, s);
    }
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

// Workspace of the leaf-batched descent for a slice of n queries at a
// level-1 beam of cap: the screened scores and launch order, the kept-leaf
// slots, the per-query counts and their scan, the pair sort and the
// candidates' distances (at most the rows of the cap largest leaves per
// query).  Every part 256-byte aligned.
struct BatchedLayout {
  float* S;
  uint32_t* keys;
  uint32_t* order;
  uint32_t* leaf[5];  // b0, cnt, off, key, val
  uint32_t* n_kept;
  uint32_t* n_cand;
  uint32_t* scan_sums;
  float* cand;
  SortWork sw;
  int64_t bytes;
};

int64_t batched_cand_bound(const mask_index& ix, int cap) {
  if (ix.leaf_top.empty()) return 0;
  return ix.leaf_top[(size_t)std::min<int64_t>(cap, (int64_t)ix.leaf_top.size() - 1)];
}

BatchedLayout batched_layout(const mask_index& ix, int cap, int64_t n, void* base) {
  BatchedLayout Lo{};
  char* b = static_cast<char*>(base);
  int64_t off = 0;
  auto take = [&](int64_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off += (bytes + 255) & ~int64_t(255);
    return p;
  };
  int64_t per_scores = 0;
  for (int l = 1; l <= ix.n_levels; ++l)
    if (ix.level_n[l] <= kScreenMax) per_scores += screen_ld(ix.level_n[l]);
  const int64_t slots = n * cap;
  Lo.S = static_cast<float*>(take(n * per_scores * 4));
  Lo.keys = static_cast<uint32_t*>(take(n * 4));
  Lo.order = static_cast<uint32_t*>(take(n * 4));
  for (int i = 0; i < 5; ++i) Lo.leaf[i] = static_cast<uint32_t*>(take(slots * 4));
  Lo.n_kept = static_cast<uint32_t*>(take(n * 4));
  Lo.n_cand = static_cast<uint32_t*>(take(n * 4));
  Lo.scan_sums = static_cast<uint32_t*>(take(scan_sums_needed(n) * 4));
  Lo.cand = static_cast<float*>(take(std::max<int64_t>(n * batched_cand_bound(ix, cap), 1) * 4));
  off += sort_work_carve(Lo.sw, b ? b + off : nullptr, slots, false);
  Lo.bytes = off;
  return Lo;
}

void check_batched(const mask_index* ix, const int32_t* r_levels) {
  MASK_CHECK(ix != nullptr, "index is NULL");
  if (ix->precision != MASK_BF16 || ix->sparse || ix->metric != MASK_L2)
    throw Error{MASK_ERR_UNSUPPORTED, "leaf-batched descent: BF16 form of dense L2 data"};
  if (ix->ld > kMaxBatchedLd)
    throw Error{MASK_ERR_UNSUPPORTED, "leaf-batched descent: dim above 256"};
  MASK_CHECK(r_levels != nullptr, "r_levels is NULL");
  for (int d = 0; d < ix->n_levels; ++d)
    MASK_CHECK(r_levels[d] >= 1 && r_levels[d] <= kMaxBeam, "beam must be in [1, 2048]");
}

// The screened descent with the data layer evaluated leaf by leaf: a first
// descent stops after level 1 and lists each query's kept leaves; the
// (leaf, query) pairs are sorted by leaf; one workgroup per leaf computes
// the BF16 distance of each of its rows to each query that kept it (the
// descent's own arithmetic); a second descent runs the data layer (the
// re-rank set, the FP32 re-rank, the k nearest) on those distances.
// Results equal mask_query_screened's bit for bit.
mask_status batched_impl(const mask_index* ix, const mask_matrix* q, int32_t k,
                         const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                         int32_t* sel, void* workspace, int64_t workspace_bytes,
                         void* hip_stream) {
  try {
    check_batched(ix, r_levels);
    check_dense(q, "queries");
    MASK_CHECK(q->dim == ix->dim, "query dim differs from the index dim");
    MASK_CHECK(k >= 1 && k <= kMaxBeam, "k must be in [1, 2048]");
    MASK_CHECK(q->n < ((int64_t)1 << 31), "too many queries in one call");
    const int L = ix->n_levels;
    int rmax = 1;
    for (int d = 0; d < L; ++d) rmax = std::max(rmax, r_levels[d]);
    if (q->n == 0) return MASK_OK;
    MASK_CHECK(out_ids && out_dist, "output pointer is NULL");
    MASK_CHECK(workspace != nullptr, "workspace is NULL");
    MASK_CHECK(((uintptr_t)workspace & 255) == 0, "workspace must be 256-byte aligned");
    const int cap = r_levels[L - 1];  // the level-1 beam
    const int64_t cb = std::max<int64_t>(batched_cand_bound(*ix, cap), 1);
    // the largest slice that fits the workspace, with 32-bit (unsigned)
    // candidate offsets and pair indexes
    int64_t hi = std::min<int64_t>({q->n, (int64_t)1 << 20, (int64_t)UINT32_MAX / cb,
                                    (int64_t)UINT32_MAX / std::max(cap, 1)});
    int64_t lo = 1;
    MASK_CHECK(hi >= 1 && batched_layout(*ix, cap, 1, nullptr).bytes <= workspace_bytes,
               "workspace smaller than one query's leaf-batched descent (mask_batched_bytes)");
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (batched_layout(*ix, cap, mid, nullptr).bytes <= workspace_bytes) lo = mid;
      else hi = mid - 1;
    }
    const int64_t step = lo;
    hipStream_t s = (hipStream_t)hip_stream;
    const DescentArgs da = descent_args(*ix);
    const int ldq = ld_of(q);
    const int64_t n1 = ix->level_n[1];
    for (int64_t s0 = 0; s0 < q->n; s0 += step) {
      const int64_t len = std::min(step, q->n - s0);
      const float* Qs = q->x + s0 * ldq;
      BatchedLayout W = batched_layout(*ix, cap, len, workspace);
      QueryArgs qa{};
      qa.Q = Qs;
      qa.ldq = ldq;
      qa.nq = len;
      qa.k = k;
      qa.r = rmax;
      qa.out_ids = out_ids + s0 * k;
      qa.out_dist = out_dist + s0 * k;
      qa.sel = sel ? sel + s0 * (int64_t)L * rmax : nullptr;
      qa.rows = timing_row_counter();
      for (int d = 0; d < L; ++d) qa.r_lev[L - d] = r_levels[d];
      screen_batch(*ix, Qs, ldq, len, W.S, W.keys, W.order, qa, s);
      // 1. the prototype levels: each query's kept leaves
      qa.leaf_mode = 1;
      qa.leaf_cap = cap;
      qa.leaf_b0 = W.leaf[0];
      qa.leaf_cnt = W.leaf[1];
      qa.leaf_off = W.leaf[2];
      qa.leaf_key = W.leaf[3];
      qa.leaf_val = W.leaf[4];
      qa.n_kept = W.n_kept;
      qa.n_cand = W.n_cand;
      if (!level_select(da, qa, s)) descent(da, qa, s);
      // 2. candidate offsets; the pairs grouped by leaf
      exclusive_scan_u32(W.n_cand, len, nullptr, W.scan_sums, s);
      radix_sort_u32(qa.leaf_key, qa.leaf_val, len * cap, bits_for(n1 + 1), W.sw, s);
      // 3. the BF16 distances, leaf by leaf
      leaf_scan(da, qa.leaf_key, qa.leaf_val, len * cap, cap, qa.leaf_off, W.n_cand, Qs, ldq,
                W.cand, s);
      // 4. the data layer on them
      qa.leaf_mode = 2;
      qa.sel = nullptr;
      qa.cand_off = W.n_cand;
      qa.cand = W.cand;
      if (!leaf_select(da, qa, s)) descent(da, qa, s);
    }
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

}  // namespace
}  // namespace mask

extern "C" {

mask_status mask_query_screened(const mask_index* ix, const mask_matrix* q, int32_t k,
                                const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                                void* workspace, int64_t workspace_bytes, void* hip_stream) {
  return screened_impl(ix, q, k, r_levels, out_ids, out_dist, nullptr, workspace,
                       workspace_bytes, hip_stream);
}

mask_status mask_query_batched(const mask_index* ix, const mask_matrix* q, int32_t k,
                               const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                               void* workspace, int64_t workspace_bytes, void* hip_stream) {
  return mask::batched_impl(ix, q, k, r_levels, out_ids, out_dist, nullptr, workspace,
                            workspace_bytes, hip_stream);
}

mask_status mask_query_batched_debug(const mask_index* ix, const mask_matrix* q, int32_t k,
                                     const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                                     int32_t* sel, void* workspace, int64_t workspace_bytes,
                                     void* hip_stream) {
  if (!sel) {
    mask::set_error("sel is NULL");
    return MASK_ERR_INVALID;
  }
  return mask::batched_impl(ix, q, k, r_levels, out_ids, out_dist, sel, workspace,
                            workspace_bytes, hip_stream);
}

mask_status mask_batched_bytes(const mask_index* ix, const int32_t* r_levels, int64_t n_queries,
                               int64_t* bytes) {
  try {
    mask::check_batched(ix, r_levels);
    MASK_CHECK(bytes != nullptr, "bytes is NULL");
    MASK_CHECK(n_queries >= 1 && n_queries <= ((int64_t)1 << 20),
               "n_queries must be in [1, 2^20]");
    const int cap = r_levels[ix->n_levels - 1];
    *bytes = mask::batched_layout(*ix, cap, n_queries, nullptr).bytes;
    return MASK_OK;
  } catch (const mask::Error& e) {
    return mask::fail(e);
  }
}

mask_status mask_query_screened_debug(const mask_index* ix, const mask_matrix* q, int32_t k,
                                      const int32_t* r_levels, int32_t* out_ids,
                                      float* out_dist, int32_t* sel, void* workspace,
                                      int64_t workspace_bytes, void* hip_stream) {
  if (!sel) {
    set_error("sel is NULL");
    return MASK_ERR_INVALID;
  }
  return screened_impl(ix, q, k, r_levels, out_ids, out_dist, sel, workspace, workspace_bytes,
                       hip_stream);
}

}  // extern "C"

// Scratch of mask_query_screened_noalloc: score rows and launch order of one
// slice of queries.  Host code uses only the per-device address that
// hipGetSymbolAddress returns (the array's name is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[MASK_NOALLOC_SCRATCH_BYTES];

namespace mask {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices] = {};

// The current device's copy of the scratch array, looked up on its first use
// on that device.
void* device_scratch() {
  int dev = -1;
  MASK_HIP(hipGetDevice(&dev));
  MASK_CHECK(dev >= 0 && dev < kMaxDevices, "device ordinal beyond the supported range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{MASK_ERR_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_at[dev] = p;
  }
  return g_scratch_at[dev];
}

}  // namespace
}  // namespace mask

extern "C" {

mask_status mask_query_screened_noalloc(const mask_index* ix, const mask_matrix* q, int32_t k,
                                        const int32_t* r_levels, int32_t* out_ids,
                                        float* out_dist, void* hip_stream) {
  try {
    if (ix) {
      int64_t per_query = 0;
      const mask_status st = mask_screen_bytes(ix, &per_query);
      if (st != MASK_OK) return st;
      if (per_query > MASK_NOALLOC_SCRATCH_BYTES) {
        std::ostringstream m;
        m << "one query's screened scores take " << per_query << " bytes, more than the "
          << MASK_NOALLOC_SCRATCH_BYTES << "-byte static scratch";
        throw Error{MASK_ERR_INVALID, m.str()};
      }
    }
    void* ws = device_scratch();
    return screened_impl(ix, q, k, r_levels, out_ids, out_dist, nullptr, ws,
                         MASK_NOALLOC_SCRATCH_BYTES, hip_stream);
  } catch (const Error& e) {
    return fail(e);
  }
}

mask_status mask_query_ragged(const mask_index* ix, const mask_matrix* q, const int32_t* k_i,
                              const int32_t* r_i, const int64_t* out_off, int32_t k_max,
                              int32_t r_max, const int32_t* beam_eighths, int32_t* out_ids,
                              float* out_dist, void* hip_stream) {
  if (!k_i || !r_i || !out_off) {
    set_error("k_i, r_i and out_off are required");
    return MASK_ERR_INVALID;
  }
  return query_impl(ix, q, k_max, r_max, k_i, r_i, out_off, out_ids, out_dist, nullptr,
                    hip_stream, nullptr, nullptr, nullptr, nullptr, beam_eighths);
}

mask_status mask_query_range(const mask_index* ix, const mask_matrix* q, const float* radius,
                             int32_t max_out, int32_t level_cap, int32_t* out_ids,
                             float* out_dist, int32_t* out_count, void* hip_stream) {
  if (!radius) {
    set_error("radius is NULL");
    return MASK_ERR_INVALID;
  }
  return query_impl(ix, q, max_out, level_cap, nullptr, nullptr, nullptr, out_ids, out_dist,
                    nullptr, hip_stream, nullptr, radius, out_count);
}

mask_status mask_point_query(const mask_index* ix, const mask_matrix* q, int32_t* out_ids,
                             float* out_dist, int32_t* out_leaf, int32_t* out_match,
                             void* hip_stream) {
  try {
    MASK_CHECK(ix != nullptr, "index is NULL");
    if (ix->sparse) throw Error{MASK_ERR_UNSUPPORTED, "point query on a CSR index"};
    MASK_CHECK(q != nullptr, "queries is NULL");
    MASK_CHECK(q->n == 0 || (out_leaf && out_match), "output pointer is NULL");
  } catch (const Error& e) {
    return fail(e);
  }
  const mask_status st = query_impl(ix, q, 1, 1, nullptr, nullptr, nullptr, out_ids, out_dist,
                                    nullptr, hip_stream, nullptr, nullptr, nullptr, out_leaf);
  if (st != MASK_OK || q->n == 0) return st;
  try {
    point_match(descent_args(*ix), q->x, ld_of(q), q->n, out_leaf, out_match,
                (hipStream_t)hip_stream);
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

mask_status mask_insert(mask_index* ix, const mask_matrix* points, int32_t max_leaf,
                        int32_t* out_leaf, int32_t* n_rebuilt, const mask_allocator* a,
                        void* hip_stream) {
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    MASK_CHECK(ix != nullptr, "index is NULL");
    if (ix->sparse || !ix->perm0)
      throw Error{MASK_ERR_UNSUPPORTED, "insertion needs a dense index built by mask_build"};
    check_dense(points, "points");
    MASK_CHECK(points->dim == ix->dim, "points dim differs from the index dim");
    MASK_CHECK(n_rebuilt != nullptr, "n_rebuilt is NULL");
    *n_rebuilt = 0;
    const int64_t n = ix->n, m = points->n;
    if (m == 0) return MASK_OK;
    MASK_CHECK(out_leaf != nullptr, "out_leaf is NULL");
    MASK_CHECK(n + m < ((int64_t)1 << 31), "the index would exceed 2^31 rows");
    const int ld = ix->ld, dim = ix->dim, ldp = ld_of(points);
    const int C = (int)ix->group_off0.size() - 1, k0 = ix->levels[0].k;
    const int64_t n1 = ix->level_n[1], n2 = n + m;
    Arena scratch(a, s);

    // 1. every new point descends to a leaf (prototypes without children
    //    above level 1 are skipped, so a leaf is always reached)
    {
      QueryArgs qa{};
      qa.Q = points->x;
      qa.ldq = ldp;
      qa.nq = m;
      qa.k = 1;
      qa.r = 1;
      qa.out_ids = scratch.alloc<int32_t>(m);
      qa.out_dist = scratch.alloc<float>(m);
      qa.out_leaf = out_leaf;
      qa.skip_empty = true;
      descent(descent_args(*ix), qa, s);
      uint32_t* flag = scratch.alloc<uint32_t>(1);
      check_range_i32(out_leaf, m, n1, flag, s);
      uint32_t h = 0;
      MASK_HIP(hipMemcpyAsync(&h, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      MASK_HIP(hipStreamSynchronize(s));
      if (h != 0) throw Error{MASK_ERR_DEVICE, "insertion descent reached no leaf"};
    }
    // 2. level-1 parent of every row, the new ones last
    int32_t* par1 = scratch.alloc<int32_t>(n2);
    leaf_parents(ix->child_off[1], n1, ix->orig[1], ix->orig[0], n, par1, s);
    MASK_HIP(hipMemcpyAsync(par1 + n, out_leaf, m * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    // 3. level-0 groups: a new row joins the group of its leaf, after its members
    int64_t* goff = scratch.alloc<int64_t>(C + 1);
    MASK_HIP(hipMemcpyAsync(goff, ix->group_off0.data(), (C + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
    uint32_t* keys = scratch.alloc<uint32_t>(n2);
    uint32_t* perm = scratch.alloc<uint32_t>(n2);
    SortWork sw;
    sort_work_alloc(sw, n2, false, scratch);
    insert_group_keys(ix->perm0, goff, C, n, out_leaf, m, k0, keys, perm, s);
    radix_sort_u32(keys, perm, n2, bits_for(2 * (int64_t)C), sw, s);
    uint32_t* off2 = scratch.alloc<uint32_t>(2 * (int64_t)C + 1);
    offsets_from_sorted(keys, n2, 2 * (int64_t)C, off2, s);
    std::vector<uint32_t> h2(2 * (size_t)C + 1);
    MASK_HIP(hipMemcpyAsync(h2.data(), off2, h2.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                            s));
    int32_t* pos0 = scratch.alloc<int32_t>(n);  // data row id -> old leaf-order position
    scatter_iota(reinterpret_cast<const uint32_t*>(ix->orig[0]), n,
                 reinterpret_cast<uint32_t*>(pos0), s);
    MASK_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> goff_new(C + 1);
    for (int g = 0; g < C; ++g) goff_new[g] = h2[2 * (size_t)g];
    goff_new[C] = n2;

    // 4. local rebuild of every group holding a leaf above max_leaf: its
    //    Lloyd iterations over its current members, from its current
    //    prototypes; the levels above keep their structure
    std::vector<int32_t> groups;
    if (max_leaf > 0) {
      uint32_t* cnt = scratch.alloc<uint32_t>(n1);
      count_labels(par1, n2, cnt, n1, s);
      std::vector<uint32_t> hc(n1);
      MASK_HIP(hipMemcpyAsync(hc.data(), cnt, n1 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      MASK_HIP(hipStreamSynchronize(s));
      for (int g = 0; g < C; ++g) {
        uint32_t mx = 0;
        for (int j = 0; j < k0; ++j) mx = std::max(mx, hc[(size_t)g * k0 + j]);
        if (mx > (uint32_t)max_leaf) groups.push_back(g);
      }
    }
    if (!groups.empty()) {
      const int Cf = (int)groups.size();
      std::vector<int64_t> offs(Cf + 1, 0);
      for (int c = 0; c < Cf; ++c)
        offs[c + 1] = offs[c] + (goff_new[groups[c] + 1] - goff_new[groups[c]]);
      const int64_t M = offs[Cf];
      uint32_t* mem_ids = scratch.alloc<uint32_t>(M);
      for (int c = 0; c < Cf; ++c)
        MASK_HIP(hipMemcpyAsync(mem_ids + offs[c], perm + goff_new[groups[c]],
                                (offs[c + 1] - offs[c]) * sizeof(uint32_t),
                                hipMemcpyDeviceToDevice, s));
      float* items = scratch.alloc<float>(M * ld);
      gather_two(mem_ids, M, ix->protos[0], pos0, n, points->x, ldp, dim, ld, items, s);
      std::vector<uint32_t> slots((size_t)Cf * k0);
      for (int c = 0; c < Cf; ++c)
        for (int j = 0; j < k0; ++j) slots[(size_t)c * k0 + j] = (uint32_t)(groups[c] * k0 + j);
      uint32_t* d_slots = scratch.alloc<uint32_t>(slots.size());
      uint32_t* d_pos = scratch.alloc<uint32_t>(slots.size());
      int32_t* d_groups = scratch.alloc<int32_t>(Cf);
      MASK_HIP(hipMemcpyAsync(d_slots, slots.data(), slots.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, s));
      MASK_HIP(hipMemcpyAsync(d_groups, groups.data(), Cf * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
      map_u32(reinterpret_cast<const uint32_t*>(ix->inv[1]), d_slots, slots.size(), d_pos, s);
      float* init = scratch.alloc<float>(slots.size() * ld);
      gather_rows(ix->protos[1], ld, d_pos, slots.size(), ld, init, ld, s);
      float* protos_new = scratch.alloc<float>(slots.size() * ld);
      int32_t* labels = scratch.alloc<int32_t>(M);
      {
        Arena level_scratch(a, s);
        run_level(items, M, ld, dim, Cf, k0, ix->lloyd_iters, ix->metric, ix->precision, init,
                  protos_new, labels, nullptr, level_scratch, s, nullptr, &offs);
        MASK_HIP(hipStreamSynchronize(s));
      }
      scatter_rows(protos_new, d_pos, slots.size(), ld, ix->protos[1], s);
      relabel(mem_ids, labels, M, d_groups, k0, par1, s);
      if (ix->precision == MASK_BF16)
        quantize_bf16(ix->protos[1], ld, n1, ix->protos_b[1], ix->ldb, ix->norm_b[1], s);
      *n_rebuilt = Cf;
    }

    // 5. leaf order of the data: the new group order, stably sorted by the
    //    position of each row's leaf
    uint32_t* order = scratch.alloc<uint32_t>(n2);
    MASK_HIP(hipMemcpyAsync(order, perm, n2 * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    leaf_keys(order, n2, par1, ix->inv[1], keys, s);
    radix_sort_u32(keys, order, n2, bits_for(n1), sw, s);
    uint32_t* child_off1 = ix->mem.alloc<uint32_t>(n1 + 1);
    offsets_from_sorted(keys, n2, n1, child_off1, s);
    int32_t* orig0 = ix->mem.alloc<int32_t>(n2);
    MASK_HIP(hipMemcpyAsync(orig0, order, n2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    float* rows0 = ix->mem.alloc<float>(n2 * ld);
    gather_two(order, n2, ix->protos[0], pos0, n, points->x, ldp, dim, ld, rows0, s);
    int32_t* perm0 = ix->mem.alloc<int32_t>(n2);
    MASK_HIP(hipMemcpyAsync(perm0, perm, n2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    uint16_t* rows_b = nullptr;
    uint8_t* rows_q = nullptr;
    float* scale_q = nullptr;
    int32_t* inv0 = nullptr;
    if (ix->precision == MASK_BF16) {
      rows_b = ix->mem.alloc<uint16_t>(n2 * ix->ldb);
      quantize_bf16(rows0, ld, n2, rows_b, ix->ldb, nullptr, s);
    }
    if (ix->precision == MASK_FP8_E4M3) {
      rows_q = ix->mem.alloc<uint8_t>(n2 * ix->ldq);
      scale_q = ix->mem.alloc<float>(n2);
      quantize_fp8(rows0, ld, n2, rows_q, ix->ldq, scale_q, nullptr, s);
    }
    if (ix->inv0) {
      inv0 = ix->mem.alloc<int32_t>(n2);
      scatter_iota(reinterpret_cast<const uint32_t*>(orig0), n2,
                   reinterpret_cast<uint32_t*>(inv0), s);
    }
    std::vector<uint32_t> hoff(n1 + 1);
    MASK_HIP(hipMemcpyAsync(hoff.data(), child_off1, (n1 + 1) * sizeof(uint32_t),
                            hipMemcpyDeviceToHost, s));
    MASK_HIP(hipStreamSynchronize(s));
    int64_t mx = 0;
    for (int64_t p = 0; p < n1; ++p) mx = std::max<int64_t>(mx, hoff[p + 1] - hoff[p]);

    // 6. swap the level-0 arrays of the index
    ix->mem.free_one(ix->child_off[1]);
    ix->mem.free_one(ix->orig[0]);
    ix->mem.free_one(ix->protos[0]);
    ix->mem.free_one(ix->perm0);
    ix->child_off[1] = child_off1;
    ix->orig[0] = orig0;
    ix->protos[0] = rows0;
    ix->perm0 = perm0;
    if (rows_b) { ix->mem.free_one(ix->protos_b[0]); ix->protos_b[0] = rows_b; }
    if (rows_q) {
      ix->mem.free_one(ix->protos_q[0]);
      ix->mem.free_one(ix->scale_q[0]);
      ix->protos_q[0] = rows_q;
      ix->scale_q[0] = scale_q;
    }
    if (inv0) { ix->mem.free_one(ix->inv0); ix->inv0 = inv0; }
    ix->max_children[1] = mx;
    set_leaf_top(*ix, hoff);
    ix->n = n2;
    ix->level_n[0] = n2;
    ix->group_off0 = goff_new;
    return MASK_OK;
  } catch (const Error& e) {
    if (e.status != MASK_ERR_INVALID && e.status != MASK_ERR_UNSUPPORTED)
      (void)hipStreamSynchronize(s);
    return fail(e);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    return fail(Error{MASK_ERR_NOMEM, "host allocation failed"});
  }
}

mask_status mask_relocate(const mask_index* ix, const int32_t* leaf, const int32_t* wrong,
                          int32_t* perm_out, int64_t* group_off_out, int32_t cap,
                          int32_t* n_groups, const mask_allocator* a, void* hip_stream) {
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    MASK_CHECK(ix != nullptr, "index is NULL");
    if (!ix->perm0)
      throw Error{MASK_ERR_UNSUPPORTED, "index without a level-0 order (imported or CSR)"};
    MASK_CHECK(leaf && wrong && perm_out && group_off_out && n_groups, "NULL argument");
    const int C = ix->levels[0].n_chunks, k0 = ix->levels[0].k;
    MASK_CHECK(cap >= C + 1, "group_off_out holds fewer than n_chunks + 1 entries");
    const int64_t n = ix->n;
    Arena scratch(a, s);
    int64_t* goff = scratch.alloc<int64_t>(C + 1);
    MASK_HIP(hipMemcpyAsync(goff, ix->group_off0.data(), (C + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
    uint32_t* off2 = scratch.alloc<uint32_t>(2 * (int64_t)C + 2);
    uint32_t* bad = off2 + 2 * (int64_t)C + 1;
    relocate_order(ix->perm0, goff, C, n, k0, leaf, wrong, perm_out, off2, bad, scratch, s);
    std::vector<uint32_t> h(2 * (size_t)C + 2);
    MASK_HIP(hipMemcpyAsync(h.data(), off2, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                            s));
    MASK_HIP(hipStreamSynchronize(s));
    MASK_CHECK(h[2 * (size_t)C + 1] == 0, "a leaf lies outside level 1");
    int count = 0;
    group_off_out[0] = 0;
    for (int g = 0; g < C; ++g) {
      const uint32_t end = h[2 * (size_t)g + 2];
      if (end > h[2 * (size_t)g]) group_off_out[++count] = end;
    }
    *n_groups = count;
    return MASK_OK;
  } catch (const Error& e) {
    if (e.status != MASK_ERR_INVALID && e.status != MASK_ERR_UNSUPPORTED)
      (void)hipStreamSynchronize(s);
    return fail(e);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    return fail(Error{MASK_ERR_NOMEM, "host allocation failed"});
  }
}

mask_status mask_query_beams_debug(const mask_index* ix, const mask_matrix* q, int32_t k,
                                   const int32_t* r_levels, int32_t* out_ids, float* out_dist,
                                   int32_t* sel, void* hip_stream) {
  if (!r_levels || !sel) {
    set_error("r_levels and sel are required");
    return MASK_ERR_INVALID;
  }
  int32_t rmax = 1;
  if (ix)
    for (int d = 0; d < ix->n_levels; ++d) rmax = r_levels[d] > rmax ? r_levels[d] : rmax;
  return query_impl(ix, q, k, rmax, nullptr, nullptr, nullptr, out_ids, out_dist, sel,
                    hip_stream, r_levels);
}

mask_status mask_query_debug(const mask_index* ix, const mask_matrix* q, int32_t k, int32_t r,
                             int32_t* out_ids, float* out_dist, int32_t* sel,
                             void* hip_stream) {
  if (!sel) {
    set_error("sel is NULL");
    return MASK_ERR_INVALID;
  }
  return query_impl(ix, q, k, r, nullptr, nullptr, nullptr, out_ids, out_dist, sel, hip_stream);
}

mask_status mask_free(mask_index* ix) {
  if (!ix) return MASK_OK;
  (void)hipStreamSynchronize(ix->mem.stream());
  delete ix;
  return MASK_OK;
}

mask_status mask_index_info(const mask_index* ix, mask_info* out) {
  if (!ix || !out) {
    set_error("NULL argument");
    return MASK_ERR_INVALID;
  }
  std::memset(out, 0, sizeof(*out));
  out->n = ix->n;
  out->dim = ix->dim;
  out->n_levels = ix->n_levels;
  out->metric = ix->metric;
  out->precision = ix->precision;
  for (int l = 1; l <= ix->n_levels; ++l) out->level_size[l - 1] = ix->level_n[l];
  out->device_bytes = (int64_t)ix->mem.bytes();
  out->refined_last_level = ix->refined_last;
  out->layout = ix->sparse ? MASK_CSR : MASK_DENSE;
  out->nnz = ix->sp_nnz;
  return MASK_OK;
}

mask_status mask_export_level(const mask_index* ix, int32_t level, float* protos_host,
                              int32_t* parent_host) {
  try {
    MASK_CHECK(ix != nullptr, "index is NULL");
    MASK_CHECK(level >= 1 && level <= ix->n_levels, "level out of range");
    MASK_CHECK(protos_host != nullptr, "protos_host is NULL");
    const int64_t nl = ix->level_n[level], nb = ix->level_n[level - 1];
    const int ld = ix->ld, dim = ix->dim;
    std::vector<float> P(nl * ld);
    std::vector<int32_t> orig(nl);
    MASK_HIP(hipMemcpy(P.data(), ix->protos[level], nl * ld * sizeof(float), hipMemcpyDeviceToHost));
    MASK_HIP(hipMemcpy(orig.data(), ix->orig[level], nl * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t pos = 0; pos < nl; ++pos)
      std::memcpy(protos_host + (int64_t)orig[pos] * dim, P.data() + pos * ld, dim * sizeof(float));
    if (parent_host) {
      std::vector<uint32_t> off(nl + 1);
      std::vector<int32_t> orig_below(nb);
      MASK_HIP(hipMemcpy(off.data(), ix->child_off[level], (nl + 1) * sizeof(uint32_t),
                         hipMemcpyDeviceToHost));
      MASK_HIP(hipMemcpy(orig_below.data(), ix->orig[level - 1], nb * sizeof(int32_t),
                         hipMemcpyDeviceToHost));
      for (int64_t p = 0; p < nl; ++p)
        for (uint32_t q = off[p]; q < off[p + 1]; ++q) parent_host[orig_below[q]] = orig[p];
    }
    return MASK_OK;
  } catch (const Error& e) {
    return fail(e);
  }
}

mask_status mask_import(const mask_matrix* data, int32_t n_levels, const mask_level* levels,
                        const float* const* protos_host, const int32_t* const* parents_host,
                        const mask_build_params* p, const mask_allocator* a, void* hip_stream,
                        mask_index** out) {
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    MASK_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    MASK_CHECK(data != nullptr, "data is NULL");
    const bool sparse = data->layout == MASK_CSR;
    if (sparse) check_csr(data, "data");
    else check_dense(data, "data");
    MASK_CHECK(data->n >= 1 && data->n < ((int64_t)1 << 31), "n must be in [1, 2^31)");
    MASK_CHECK(protos_host && parents_host, "host arrays are NULL");
    std::vector<int64_t> sizes;
    check_levels(data->n, n_levels, levels, sizes);
    const int metric = p ? p->metric : MASK_L2;
    MASK_CHECK(metric == MASK_L2 || metric == MASK_L1, "unknown metric");
    if (!sparse && data->dim > kMaxQueryDim) throw Error{MASK_ERR_UNSUPPORTED, "dim above 4096"};
    for (int l = 0; l < n_levels; ++l) {
      MASK_CHECK(protos_host[l] && parents_host[l], "a level's host array is NULL");
      for (int64_t i = 0; i < sizes[l]; ++i)
        MASK_CHECK(parents_host[l][i] >= 0 && parents_host[l][i] < sizes[l + 1],
                   "parent id out of range");
    }
    auto ix = std::make_unique<mask_index>(a, s);
    const int L = n_levels;
    ix->n = data->n;
    ix->dim = data->dim;
    ix->ld = round_up4(data->dim);
    ix->metric = metric;
    ix->precision = p ? p->precision : MASK_FP32;
    MASK_CHECK(ix->precision >= MASK_FP32 && ix->precision <= MASK_FP8_E4M3,
               "unsupported precision");
    if (ix->precision != MASK_FP32 && metric != MASK_L2)
      throw Error{MASK_ERR_UNSUPPORTED, "BF16 / FP8 form of L1"};
    if (sparse && (ix->precision != MASK_FP32 || metric != MASK_L2))
      throw Error{MASK_ERR_UNSUPPORTED, "CSR data: L2 metric, FP32 form only"};
    ix->sparse = sparse;
    ix->rerank_factor = (p && p->rerank_factor != 0) ? p->rerank_factor
                        : (ix->precision == MASK_FP8_E4M3 ? 48 : 4);
    ix->n_levels = L;
    ix->levels.assign(levels, levels + L);
    ix->level_n = sizes;
    const int ld = ix->ld, dim = ix->dim;
    Arena scratch(a, s);
    float* items0 = nullptr;
    Csr view;
    if (sparse) {
      validate_csr(data, "data", scratch, s);
      view = csr_view(data);
    } else {
      items0 = scratch.alloc<float>(data->n * ld);
      copy_rows(data->x, ld_of(data), data->n, dim, items0, ld, s);
    }
    uint32_t* ident = scratch.alloc<uint32_t>(data->n);
    iota_u32(ident, data->n, s);
    BuildState st;
    st.labels.assign(L + 1, nullptr);
    st.protos_cm.assign(L + 1, nullptr);
    std::vector<float> padded;
    for (int l = 1; l <= L; ++l) {
      const int64_t nl = sizes[l];
      padded.assign(nl * ld, 0.f);
      for (int64_t i = 0; i < nl; ++i)
        std::memcpy(padded.data() + i * ld, protos_host[l - 1] + i * dim, dim * sizeof(float));
      st.protos_cm[l] = scratch.alloc<float>(nl * ld);
      MASK_HIP(hipMemcpy(st.protos_cm[l], padded.data(), nl * ld * sizeof(float),
                         hipMemcpyHostToDevice));
      st.labels[l] = scratch.alloc<int32_t>(sizes[l - 1]);
      MASK_HIP(hipMemcpy(st.labels[l], parents_host[l - 1], sizes[l - 1] * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    }
    finalize_layout(*ix, st.labels, st.protos_cm, items0, ident, scratch, s,
                    sparse ? &view : nullptr);
    MASK_HIP(hipStreamSynchronize(s));
    *out = ix.release();
    return MASK_OK;
  } catch (const Error& e) {
    if (e.status != MASK_ERR_INVALID && e.status != MASK_ERR_UNSUPPORTED)
      (void)hipStreamSynchronize(s);
    return fail(e);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    return fail(Error{MASK_ERR_NOMEM, "host allocation failed"});
  }
}

mask_status mask_kmeanspp(const mask_matrix* items, int32_t n_chunks, int32_t k, uint64_t seed,
                          int32_t level, float* centroids, int32_t* chosen,
                          const mask_allocator* a, void* hip_stream) {
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    MASK_CHECK(items != nullptr, "items is NULL");
    if (items->layout == MASK_CSR)
      throw Error{MASK_ERR_UNSUPPORTED, "k-means++ seeding: dense items only"};
    check_dense(items, "items");
    MASK_CHECK(items->n >= 1 && items->n < ((int64_t)1 << 31), "n must be in [1, 2^31)");
    MASK_CHECK(n_chunks >= 1 && k >= 1, "bad n_chunks or k");
    MASK_CHECK(items->n >= n_chunks, "more chunks than items");
    MASK_CHECK((int64_t)n_chunks * k < ((int64_t)1 << 31), "too many prototypes");
    MASK_CHECK(level >= 0 && level < (1 << 23), "level must be in [0, 2^23)");
    MASK_CHECK(centroids != nullptr, "centroids is NULL");
    if (items->dim > kMaxDenseDim) throw Error{MASK_ERR_UNSUPPORTED, "dense dim above 256"};
    const int dim = items->dim, ld = round_up4(dim);
    const int64_t n = items->n, np = (int64_t)n_chunks * k;
    Arena scratch(a, s);
    float* x = scratch.alloc<float>(n * ld);
    copy_rows(items->x, ld_of(items), n, dim, x, ld, s);
    ChunkPlan plan;
    make_plan(plan, n, n_chunks, k, scratch, s);
    float* P = scratch.alloc<float>(np * ld);
    kmeanspp_init(x, ld, dim, plan, seed, level, P, chosen, scratch, s);
    copy_rows(P, ld, np, dim, centroids, dim, s);
    MASK_HIP(hipStreamSynchronize(s));
    return MASK_OK;
  } catch (const Error& e) {
    if (e.status != MASK_ERR_INVALID && e.status != MASK_ERR_UNSUPPORTED)
      (void)hipStreamSynchronize(s);
    return fail(e);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    return fail(Error{MASK_ERR_NOMEM, "host allocation failed"});
  }
}

mask_status mask_kmeans(const mask_matrix* items, int32_t n_chunks, int32_t k, int32_t iters,
                        int32_t metric, const float* init, float* centroids, int32_t* labels,
                        double* inertia, const mask_allocator* a, void* hip_stream) {
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    MASK_CHECK(items != nullptr, "items is NULL");
    if (items->layout == MASK_CSR) {
      check_csr(items, "items");
      MASK_CHECK(items->n >= 1 && items->n < ((int64_t)1 << 31), "n must be in [1, 2^31)");
      MASK_CHECK(n_chunks >= 1 && k >= 1 && iters >= 0, "bad n_chunks, k or iters");
      MASK_CHECK(items->n >= n_chunks, "more chunks than items");
      MASK_CHECK(centroids && labels, "output pointer is NULL");
      if (metric != MASK_L2) throw Error{MASK_ERR_UNSUPPORTED, "CSR items: L2 metric only"};
      const int dim = items->dim, ld = round_up4(dim);
      const int64_t np = (int64_t)n_chunks * k;
      Arena scratch(a, s);
      validate_csr(items, "items", scratch, s);
      float* P = scratch.alloc<float>(np * ld);
      float* init_p = nullptr;
      if (init) {
        init_p = scratch.alloc<float>(np * ld);
        copy_rows(init, dim, np, dim, init_p, ld, s);
      }
      kmeans_sparse(csr_view(items), ld, n_chunks, k, iters, init_p, P, labels, inertia, scratch,
                    s);
      copy_rows(P, ld, np, dim, centroids, dim, s);
      MASK_HIP(hipStreamSynchronize(s));
      return MASK_OK;
    }
    check_dense(items, "items");
    MASK_CHECK(items->n >= 1 && items->n < ((int64_t)1 << 31), "n must be in [1, 2^31)");
    MASK_CHECK(n_chunks >= 1 && k >= 1 && iters >= 0, "bad n_chunks, k or iters");
    MASK_CHECK(items->n >= n_chunks, "more chunks than items");
    MASK_CHECK(centroids && labels, "output pointer is NULL");
    MASK_CHECK(metric == MASK_L2 || metric == MASK_L1, "unknown metric");
    if (items->dim > kMaxDenseDim) throw Error{MASK_ERR_UNSUPPORTED, "dense dim above 256"};
    const int dim = items->dim, ld = round_up4(dim);
    const int64_t n = items->n, np = (int64_t)n_chunks * k;
    Arena scratch(a, s);
    float* x = scratch.alloc<float>(n * ld);
    copy_rows(items->x, ld_of(items), n, dim, x, ld, s);
    float* P = scratch.alloc<float>(np * ld);
    float* init_p = nullptr;
    if (init) {
      init_p = scratch.alloc<float>(np * ld);
      copy_rows(init, dim, np, dim, init_p, ld, s);
    }
    run_level(x, n, ld, dim, n_chunks, k, iters, metric, MASK_FP32, init_p, P, labels, inertia,
              scratch, s, nullptr);
    copy_rows(P, ld, np, dim, centroids, dim, s);
    MASK_HIP(hipStreamSynchronize(s));
    return MASK_OK;
  } catch (const Error& e) {
    if (e.status != MASK_ERR_INVALID && e.status != MASK_ERR_UNSUPPORTED)
      (void)hipStreamSynchronize(s);
    return fail(e);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    return fail(Error{MASK_ERR_NOMEM, "host allocation failed"});
  }
}

}  // extern "C"

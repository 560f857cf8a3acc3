// Level-0 reorganisation: the relocation step of the point-query evaluation
// (Sections 4.1-4.2 and the relocation table), where data rows that their own
// point query did not find correctly join the level-0 group whose prototypes
// hold the leaf the query reached before the index is built again; and the
// bookkeeping of dynamic insertion (Section 3.3), where new rows join the
// leaf their descent reaches and the leaf order of the data is rebuilt.
//
// The new order is a stable radix sort of the old level-0 order by the key
// 2 * (new group) + (joined), so every group keeps the rows that stay in
// their old order, followed by the rows that join it in their old order.
#include "internal.hpp"

namespace mask {
namespace {

constexpr int kBlock = 256;

// key and value of position j of the old order; the group of j comes from a
// binary search of the group boundaries
__global__ __launch_bounds__(kBlock) void k_relocate_keys(
    const int32_t* __restrict__ perm0, const int64_t* __restrict__ goff, int C, int64_t n,
    int k0, const int32_t* __restrict__ leaf, const int32_t* __restrict__ wrong,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ bad) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  int lo = 0, hi = C - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (goff[mid] <= j) lo = mid;
    else hi = mid - 1;
  }
  const int g = lo;
  const int32_t i = perm0[j];
  int t = g;
  if (wrong[i] != 0) {
    const int32_t p = leaf[i];
    if (p >= (int64_t)C * k0) atomicOr(bad, 1u);
    else if (p >= 0) t = p / k0;
  }
  keys[j] = 2u * (uint32_t)t + (t != g ? 1u : 0u);
  vals[j] = (uint32_t)i;
}

// one thread per leaf-order position: binary search of its level-1 range
__global__ __launch_bounds__(kBlock) void k_leaf_parents(
    const uint32_t* __restrict__ child_off1, int64_t n1, const int32_t* __restrict__ orig1,
    const int32_t* __restrict__ orig0, int64_t n0, int32_t* __restrict__ par1) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n0) return;
  int64_t lo = 0, hi = n1 - 1;  // last p with child_off1[p] <= q
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (child_off1[mid] <= (uint32_t)q) lo = mid;
    else hi = mid - 1;
  }
  par1[orig0[q]] = orig1[lo];
}

__global__ __launch_bounds__(kBlock) void k_insert_group_keys(
    const int32_t* __restrict__ perm0, const int64_t* __restrict__ goff, int C, int64_t n,
    const int32_t* __restrict__ leaf, int64_t m, int k0, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ vals) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n + m) return;
  if (j < n) {
    int lo = 0, hi = C - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (goff[mid] <= j) lo = mid;
      else hi = mid - 1;
    }
    keys[j] = 2u * (uint32_t)lo;
    vals[j] = (uint32_t)perm0[j];
  } else {
    keys[j] = 2u * (uint32_t)(leaf[j - n] / k0) + 1u;
    vals[j] = (uint32_t)j;
  }
}

__global__ __launch_bounds__(kBlock) void k_leaf_keys(const uint32_t* __restrict__ ids,
                                                      int64_t n, const int32_t* __restrict__ par1,
                                                      const int32_t* __restrict__ inv1,
                                                      uint32_t* __restrict__ keys) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < n) keys[j] = (uint32_t)inv1[par1[ids[j]]];
}

// one lane per float of the output row
__global__ __launch_bounds__(kBlock) void k_gather_two(
    const uint32_t* __restrict__ ids, int64_t n, const float* __restrict__ rows0,
    const int32_t* __restrict__ pos0, int64_t n0, const float* __restrict__ rows1, int ld1,
    int dim, int ld, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * ld) return;
  const int64_t j = t / ld;
  const int c = (int)(t % ld);
  const int64_t id = ids[j];
  float v = 0.f;
  if (c < dim) v = id < n0 ? rows0[(int64_t)pos0[id] * ld + c] : rows1[(id - n0) * ld1 + c];
  out[t] = v;
}

__global__ __launch_bounds__(kBlock) void k_count_labels(const int32_t* __restrict__ par,
                                                         int64_t n, uint32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) atomicAdd(&counts[par[i]], 1u);
}

// dst[pos[t]] = src[t] row by row (stride ld)
__global__ __launch_bounds__(kBlock) void k_scatter_rows(const float* __restrict__ src,
                                                         const uint32_t* __restrict__ pos,
                                                         int64_t n, int ld,
                                                         float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * ld) return;
  const int64_t j = t / ld;
  dst[(int64_t)pos[j] * ld + t % ld] = src[t];
}

// par1[ids[i]] = group[c] * k0 + j for the batch label c * k0 + j
__global__ __launch_bounds__(kBlock) void k_relabel(const uint32_t* __restrict__ ids,
                                                    const int32_t* __restrict__ labels,
                                                    int64_t n, const int32_t* __restrict__ group,
                                                    int k0, int32_t* __restrict__ par1) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t l = labels[i];
  par1[ids[i]] = group[l / k0] * k0 + l % k0;
}

inline unsigned blocks_for(int64_t work) {
  const int64_t g = (work + kBlock - 1) / kBlock;
  return (unsigned)(g < 1 ? 1 : g);
}

int bits_for(int64_t n) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  return b;
}

}  // namespace

void leaf_parents(const uint32_t* child_off1, int64_t n1, const int32_t* orig1,
                  const int32_t* orig0, int64_t n0, int32_t* par1, hipStream_t s) {
  if (n0 <= 0) return;
  k_leaf_parents<<<blocks_for(n0), kBlock, 0, s>>>(child_off1, n1, orig1, orig0, n0, par1);
  check_launch("leaf_parents");
}

void insert_group_keys(const int32_t* perm0, const int64_t* goff, int C, int64_t n,
                       const int32_t* leaf, int64_t m, int k0, uint32_t* keys, uint32_t* vals,
                       hipStream_t s) {
  k_insert_group_keys<<<blocks_for(n + m), kBlock, 0, s>>>(perm0, goff, C, n, leaf, m, k0, keys,
                                                          vals);
  check_launch("insert_group_keys");
}

void leaf_keys(const uint32_t* ids, int64_t n, const int32_t* par1, const int32_t* inv1,
               uint32_t* keys, hipStream_t s) {
  if (n <= 0) return;
  k_leaf_keys<<<blocks_for(n), kBlock, 0, s>>>(ids, n, par1, inv1, keys);
  check_launch("leaf_keys");
}

void gather_two(const uint32_t* ids, int64_t n, const float* rows0, const int32_t* pos0,
                int64_t n0, const float* rows1, int ld1, int dim, int ld, float* out,
                hipStream_t s) {
  if (n <= 0) return;
  k_gather_two<<<blocks_for(n * ld), kBlock, 0, s>>>(ids, n, rows0, pos0, n0, rows1, ld1, dim,
                                                     ld, out);
  check_launch("gather_two");
}

void count_labels(const int32_t* par, int64_t n, uint32_t* counts, int64_t n_bins,
                  hipStream_t s) {
  MASK_HIP(hipMemsetAsync(counts, 0, n_bins * sizeof(uint32_t), s));
  if (n <= 0) return;
  k_count_labels<<<blocks_for(n), kBlock, 0, s>>>(par, n, counts);
  check_launch("count_labels");
}

void scatter_rows(const float* src, const uint32_t* pos, int64_t n, int ld, float* dst,
                  hipStream_t s) {
  if (n <= 0) return;
  k_scatter_rows<<<blocks_for(n * ld), kBlock, 0, s>>>(src, pos, n, ld, dst);
  check_launch("scatter_rows");
}

void relabel(const uint32_t* ids, const int32_t* labels, int64_t n, const int32_t* group, int k0,
             int32_t* par1, hipStream_t s) {
  if (n <= 0) return;
  k_relabel<<<blocks_for(n), kBlock, 0, s>>>(ids, labels, n, group, k0, par1);
  check_launch("relabel");
}

void relocate_order(const int32_t* perm0, const int64_t* goff, int C, int64_t n, int k0,
                    const int32_t* leaf, const int32_t* wrong, int32_t* perm_out,
                    uint32_t* off2, uint32_t* bad, Arena& scratch, hipStream_t s) {
  uint32_t* keys = scratch.alloc<uint32_t>(n);
  uint32_t* vals = scratch.alloc<uint32_t>(n);
  SortWork sw;
  sort_work_alloc(sw, n, false, scratch);
  MASK_HIP(hipMemsetAsync(bad, 0, sizeof(uint32_t), s));
  {
    ScopedTiming timing("relocate", s);
    k_relocate_keys<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        perm0, goff, C, n, k0, leaf, wrong, keys, vals, bad);
    check_launch("relocate_keys");
    radix_sort_u32(keys, vals, n, bits_for(2 * (int64_t)C), sw, s);
    offsets_from_sorted(keys, n, 2 * (int64_t)C, off2, s);
  }
  MASK_HIP(hipMemcpyAsync(perm_out, vals, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
}

}  // namespace mask

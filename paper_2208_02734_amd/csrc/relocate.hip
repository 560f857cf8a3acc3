// Relocation step of the point-query evaluation (Sections 4.1-4.2 and the
// relocation table): data rows that their own point query did not find
// correctly join the level-0 group whose prototypes hold the leaf the query
// reached, and the index is then built again on the new groups.
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

int bits_for(int64_t n) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  return b;
}

}  // namespace

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

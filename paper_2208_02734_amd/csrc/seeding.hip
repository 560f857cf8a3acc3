// k-means++ seeding (Arthur and Vassilvitskii 2007; Section 3.1 names it as
// the remedy for initial prototypes placed badly) for every group of a level
// at once: one workgroup per group walks the k sequential draws.
//
// Draw t of group c uses u = the top 53 bits of the SplitMix64 output at
// counter tag + c * k + t.  Draw 0 picks member floor(u * m); draw t > 0 picks
// the first member whose running sum of D^2 (in group order) exceeds
// u * sum D^2, where D^2 is the squared distance (FP64, direct form) to the
// nearest prototype chosen so far.  With sum D^2 = 0 the pick is uniform as
// for draw 0; if rounding leaves no member above the target, the last member
// with D^2 > 0 is taken.
#include "internal.hpp"

namespace mask {
namespace {

constexpr int kBlock = 256;

__device__ inline double uniform01(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

// Each thread owns a contiguous run of members for the running sums (its
// partial sum, then the owner of the target scans its run); the D^2 update is
// strided so that neighbouring threads read neighbouring rows.
__global__ __launch_bounds__(kBlock) void k_kmeanspp(
    const float* __restrict__ items, int ld, int dim, const int64_t* __restrict__ chunk_off,
    int k, uint64_t seed, uint64_t tag, double* __restrict__ d2, float* __restrict__ protos,
    int32_t* __restrict__ chosen) {
  __shared__ double s_part[kBlock];
  __shared__ float s_c[kMaxDenseDim];
  __shared__ int64_t s_pick;
  const int c = blockIdx.x, tid = threadIdx.x;
  const int64_t c0 = chunk_off[c], c1 = chunk_off[c + 1], m = c1 - c0;
  const int64_t per = (m + kBlock - 1) / kBlock;
  const int64_t r0 = c0 + min(m, (int64_t)tid * per), r1 = c0 + min(m, (int64_t)(tid + 1) * per);
  for (int t = 0; t < k; ++t) {
    const double u = uniform01(seed, tag + (uint64_t)c * (uint64_t)k + (uint64_t)t);
    if (t > 0) {
      double ps = 0.0;
      for (int64_t i = r0; i < r1; ++i) ps += d2[i];
      s_part[tid] = ps;
    }
    __syncthreads();
    if (tid == 0) {
      int64_t pick = -1;
      if (t > 0) {
        double total = 0.0;
        for (int j = 0; j < kBlock; ++j) total += s_part[j];
        if (total > 0.0) {
          const double target = u * total;
          double run = 0.0;
          int j = 0;
          while (j < kBlock && !(run + s_part[j] > target)) run += s_part[j++];
          if (j < kBlock) {
            const int64_t a0 = c0 + min(m, (int64_t)j * per);
            const int64_t a1 = c0 + min(m, (int64_t)(j + 1) * per);
            for (int64_t i = a0; i < a1; ++i) {
              run += d2[i];
              if (run > target) { pick = i - c0; break; }
            }
          }
          if (pick < 0)
            for (int64_t i = m - 1; i >= 0; --i)
              if (d2[c0 + i] > 0.0) { pick = i; break; }
        }
      }
      if (pick < 0) {
        pick = (int64_t)(u * (double)m);
        if (pick >= m) pick = m - 1;
      }
      s_pick = pick;
    }
    __syncthreads();
    const int64_t pi = c0 + s_pick;
    const int64_t slot = (int64_t)c * k + t;
    for (int q = tid; q < ld; q += kBlock) {
      const float v = items[pi * ld + q];
      protos[slot * ld + q] = v;
      s_c[q] = v;
    }
    if (tid == 0 && chosen) chosen[slot] = (int32_t)pi;
    __syncthreads();
    for (int64_t i = c0 + tid; i < c1; i += kBlock) {
      const float* x = items + i * ld;
      double acc = 0.0;
      for (int q = 0; q < dim; ++q) {
        const double df = (double)x[q] - (double)s_c[q];
        acc = fma(df, df, acc);
      }
      d2[i] = (t == 0) ? acc : fmin(d2[i], acc);
    }
    __syncthreads();
  }
}

}  // namespace

void kmeanspp_init(const float* items, int ld, int dim, const ChunkPlan& plan, uint64_t seed,
                   int level, float* protos, int32_t* chosen, Arena& scratch, hipStream_t s) {
  MASK_CHECK(ld <= kMaxDenseDim, "k-means++ seeding: dim above 256");
  double* d2 = scratch.alloc<double>(plan.n_items);
  ScopedTiming timing("kmeanspp", s);
  const uint64_t tag = ((uint64_t)level << 40);
  k_kmeanspp<<<(unsigned)plan.n_chunks, kBlock, 0, s>>>(items, ld, dim, plan.d_off, plan.k, seed,
                                                       tag, d2, protos, chosen);
  check_launch("kmeanspp");
}

}  // namespace mask

// CSR rows (the sparse, high-dimensional setting of Section 4.3): row
// movement, conversion of dense prototypes to CSR, FP64 norms, and the
// batched per-group Lloyd of Algorithm 1 on CSR items.
//
// Distances are the expanded form |x|^2 + |c|^2 - 2 x.c evaluated in FP64:
// products of FP32 values are exact in FP64 and the sums run in a fixed order,
// so labels agree with an FP64 direct-form evaluation except where two
// prototypes are within about 1e-15 relative.  There is no MFMA form: an
// item touches only its own non-zero columns.
//
// Prototypes are dense FP32 rows (row-major, ld >= cols, zero padded).  The
// assignment reads them transposed per group (column-major: for column c,
// the k prototypes of the group are contiguous), so that a wave walking one
// item's non-zeros loads k consecutive values per non-zero.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace mask {
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t work, int per_block) {
  return (unsigned)((work + per_block - 1) / per_block);
}

// ---------------------------------------------------------------- movement

__global__ void k_row_len(const int64_t* __restrict__ ptr, const uint32_t* __restrict__ idx,
                          int64_t n, uint32_t* __restrict__ len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = idx ? idx[i] : i;
  len[i] = (uint32_t)(ptr[r + 1] - ptr[r]);
}

__global__ void k_widen_ptr(const uint32_t* __restrict__ off, int64_t n,
                            const uint32_t* __restrict__ total, int64_t* __restrict__ ptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ptr[i] = off[i];
  if (i == n) ptr[n] = *total;
}

// One wave per destination row.
__global__ __launch_bounds__(kBlock) void k_copy_rows(
    const int64_t* __restrict__ sp, const int32_t* __restrict__ sc, const float* __restrict__ sv,
    const uint32_t* __restrict__ idx, int64_t n, const int64_t* __restrict__ dp,
    int32_t* __restrict__ dc, float* __restrict__ dv) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n) return;
  const int64_t r = idx[i];
  const int64_t b = sp[r], len = sp[r + 1] - b, o = dp[i];
  for (int64_t e = lane; e < len; e += kWave) {
    dc[o + e] = sc[b + e];
    dv[o + e] = sv[b + e];
  }
}

// Non-zero count of every dense row (one wave per row).
__global__ __launch_bounds__(kBlock) void k_count_nz(const float* __restrict__ x, int ld,
                                                     int64_t n, int cols,
                                                     uint32_t* __restrict__ cnt) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n) return;
  uint32_t c = 0;
  for (int j = lane; j < cols; j += kWave) c += x[i * ld + j] != 0.f;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
  if (lane == 0) cnt[i] = c;
}

// Compaction of every dense row's non-zeros in column order (one wave per row).
__global__ __launch_bounds__(kBlock) void k_fill_nz(const float* __restrict__ x, int ld,
                                                    int64_t n, int cols,
                                                    const int64_t* __restrict__ ptr,
                                                    int32_t* __restrict__ col,
                                                    float* __restrict__ val) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n) return;
  int64_t o = ptr[i];
  for (int j0 = 0; j0 < cols; j0 += kWave) {
    const int j = j0 + lane;
    const float v = j < cols ? x[i * ld + j] : 0.f;
    const bool nz = v != 0.f;
    const uint64_t m = __ballot(nz);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (nz) {
      col[o + rank] = j;
      val[o + rank] = v;
    }
    o += __popcll(m);
  }
}

// FP64 squared norms, one wave per row: lane partials in entry order, then a
// butterfly (a fixed order).
__global__ __launch_bounds__(kBlock) void k_csr_norms64(const int64_t* __restrict__ ptr,
                                                        const float* __restrict__ val,
                                                        int64_t n, double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n) return;
  double a = 0.0;
  for (int64_t e = ptr[i] + lane; e < ptr[i + 1]; e += kWave) {
    const double v = val[e];
    a = fma(v, v, a);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) out[i] = a;
}

__global__ __launch_bounds__(kBlock) void k_dense_norms64(const float* __restrict__ x, int ld,
                                                          int64_t n, int cols,
                                                          double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n) return;
  double a = 0.0;
  for (int j = lane; j < cols; j += kWave) {
    const double v = x[i * ld + j];
    a = fma(v, v, a);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) out[i] = a;
}

__global__ void k_csr_validate(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                               int64_t n, int cols, int64_t nnz, uint32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool bad = false;
  const int64_t b = ptr[i], e = ptr[i + 1];
  if (i == 0 && b != 0) bad = true;
  if (i == n - 1 && e != nnz) bad = true;
  if (b > e || b < 0 || e > nnz) {
    bad = true;
  } else {
    int32_t prev = -1;
    for (int64_t t = b; t < e; ++t) {
      const int32_t c = col[t];
      if (c <= prev || c >= cols) { bad = true; break; }
      prev = c;
    }
  }
  if (bad) atomicOr(flag, 1u);
}

// ---------------------------------------------------------------- k-means

__global__ void k_zero_f32(float* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

// Prototype c*k+j := item off[c]+j, scattered into a zeroed dense row.
__global__ __launch_bounds__(kBlock) void k_init_first_csr(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, const int64_t* __restrict__ chunk_off, int n_chunks, int k,
    float* __restrict__ P, int ld) {
  const int lane = threadIdx.x % kWave;
  const int64_t p = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (p >= (int64_t)n_chunks * k) return;
  const int64_t item = chunk_off[p / k] + p % k;
  for (int64_t e = ptr[item] + lane; e < ptr[item + 1]; e += kWave) P[p * ld + col[e]] = val[e];
}

// PT[(c*cols + d)*k + j] = P[(c*k + j)*ld + d], 32 x 32 tiles through LDS.
__global__ __launch_bounds__(kBlock) void k_transpose_groups(const float* __restrict__ P,
                                                             int ld, int k, int cols,
                                                             int tiles_d, int tiles_j,
                                                             float* __restrict__ PT) {
  __shared__ float t[32][33];
  const int64_t b = blockIdx.x;
  const int c = (int)(b / ((int64_t)tiles_d * tiles_j));
  const int rem = (int)(b % ((int64_t)tiles_d * tiles_j));
  const int d0 = (rem / tiles_j) * 32, j0 = (rem % tiles_j) * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int j = j0 + y, d = d0 + tx;
    t[y][tx] = (j < k && d < cols) ? P[((int64_t)c * k + j) * ld + d] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int d = d0 + y, j = j0 + tx;
    if (d < cols && j < k) PT[((int64_t)c * cols + d) * k + j] = t[tx][y];
  }
}

__device__ inline int group_of(const int64_t* __restrict__ off, int n_chunks, int64_t i) {
  int lo = 0, hi = n_chunks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One wave per item.  Lanes take prototypes j = j0 + lane + 64 t (T per
// lane per pass); the item's non-zeros are walked in order, U at a time,
// each broadcast to the wave, and every lane adds value * PT[column][j] to
// its FP64 dot products.  Then d = |x|^2 + |c_j|^2 - 2 x.c_j and the wave's
// argmin by (d, j).
template <int T, int U>
__global__ __launch_bounds__(kBlock) void k_assign_csr(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, const double* __restrict__ xnorm,
    const float* __restrict__ PT, const double* __restrict__ pnorm,
    const int64_t* __restrict__ chunk_off, int n_chunks, int k, int cols, int64_t n_items,
    int32_t* __restrict__ labels, double* __restrict__ best_d) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n_items) return;
  const int c = group_of(chunk_off, n_chunks, i);
  const double xn = xnorm[i];
  const int64_t b = ptr[i], e = ptr[i + 1];
  const float* pt = PT + (int64_t)c * cols * k;
  const double* pn = pnorm + (int64_t)c * k;
  double bd = INFINITY;
  int bj = k;
  for (int j0 = 0; j0 < k; j0 += kWave * T) {
    double acc[T];
    int jj[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      acc[t] = 0.0;
      const int j = j0 + lane + kWave * t;
      jj[t] = j < k ? j : k - 1;  // clamped: loads stay in bounds, results unused
    }
    for (int64_t e0 = b; e0 < e; e0 += kWave) {
      const int m = (int)min<int64_t>(kWave, e - e0);
      const int my_c = lane < m ? col[e0 + lane] : 0;
      const float my_v = lane < m ? val[e0 + lane] : 0.f;
      for (int q = 0; q < m; q += U) {
        float x[U][T];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int src = q + u < m ? q + u : q;
          const int cc = __shfl(my_c, src);
          v[u] = q + u < m ? (double)__shfl(my_v, src) : 0.0;
          const float* row = pt + (int64_t)cc * k;
#pragma unroll
          for (int t = 0; t < T; ++t) x[u][t] = row[jj[t]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int t = 0; t < T; ++t) acc[t] = fma(v[u], (double)x[u][t], acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int j = j0 + lane + kWave * t;
      if (j < k) {
        const double d = xn + pn[j] - 2.0 * acc[t];
        if (d < bd) { bd = d; bj = j; }
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double od = __shfl_xor(bd, o);
    const int oj = __shfl_xor(bj, o);
    if (od < bd || (od == bd && oj < bj)) { bd = od; bj = oj; }
  }
  if (lane == 0) {
    labels[i] = c * k + bj;
    best_d[i] = bd > 0.0 ? bd : 0.0;
  }
}

__global__ void k_labels_keys(const int32_t* __restrict__ labels, int64_t n,
                              uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = (uint32_t)labels[i];
  vals[i] = (uint32_t)i;
}

// One wave per prototype: the FP64 sum of its members over a window of
// kSumWin columns at a time in LDS (members in item order; a member's
// columns are distinct, so its lanes never collide, and one wave's LDS
// accesses complete in program order), then the FP32 mean and the FP64
// squared norm of the rounded mean.  A prototype with no member keeps its
// row and norm.
constexpr int kSumWin = 4096;

__global__ __launch_bounds__(kWave) void k_update_csr(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, const uint32_t* __restrict__ members,
    const uint32_t* __restrict__ member_off, int cols, float* __restrict__ P, int ld,
    double* __restrict__ pnorm) {
  __shared__ double acc[kSumWin];
  const int lane = threadIdx.x;
  const int64_t p = blockIdx.x;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  if (m1 == m0) return;
  const double inv_n = 1.0 / (double)(m1 - m0);
  double nrm = 0.0;
  for (int d0 = 0; d0 < cols; d0 += kSumWin) {
    const int w = min(kSumWin, cols - d0);
    for (int j = lane; j < w; j += kWave) acc[j] = 0.0;
    for (uint32_t m = m0; m < m1; ++m) {
      const int64_t it = members[m];
      for (int64_t e = ptr[it] + lane; e < ptr[it + 1]; e += kWave) {
        const int cc = col[e] - d0;
        if (cc >= 0 && cc < w) acc[cc] += (double)val[e];
      }
    }
    for (int j = lane; j < w; j += kWave) {
      const float v = (float)(acc[j] * inv_n);
      P[p * ld + d0 + j] = v;
      nrm = fma((double)v, (double)v, nrm);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) nrm += __shfl_xor(nrm, o);
  if (lane == 0) pnorm[p] = nrm;
}

// Inertia of every group: the sum of its items' distances in item order
// (lane partials, then a butterfly).
__global__ __launch_bounds__(kBlock) void k_group_sum(const double* __restrict__ d,
                                                      const int64_t* __restrict__ off,
                                                      int n_chunks, double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int64_t c = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (c >= n_chunks) return;
  double a = 0.0;
  for (int64_t i = off[c] + lane; i < off[c + 1]; i += kWave) a += d[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) out[c] = a;
}

void check_launch_sp(const char* what) { check_launch(what); }

}  // namespace

void csr_gather(const Csr& src, const uint32_t* idx, int64_t n, Csr& out, Arena& a,
                Arena& scratch, hipStream_t s) {
  out.n = n;
  out.cols = src.cols;
  uint32_t* len = scratch.alloc<uint32_t>(n + 1);
  uint32_t* total = scratch.alloc<uint32_t>(1);
  uint32_t* sums = scratch.alloc<uint32_t>(scan_sums_needed(n));
  if (n > 0) {
    k_row_len<<<grid_for(n, kBlock), kBlock, 0, s>>>(src.ptr, idx, n, len);
    check_launch_sp("row_len");
  }
  exclusive_scan_u32(len, n, total, sums, s);
  out.ptr = a.alloc<int64_t>(n + 1);
  k_widen_ptr<<<grid_for(n + 1, kBlock), kBlock, 0, s>>>(len, n, total, out.ptr);
  check_launch_sp("widen_ptr");
  uint32_t h_total = 0;
  MASK_HIP(hipMemcpyAsync(&h_total, total, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  MASK_HIP(hipStreamSynchronize(s));
  out.nnz = h_total;
  out.col = a.alloc<int32_t>(std::max<int64_t>(out.nnz, 1));
  out.val = a.alloc<float>(std::max<int64_t>(out.nnz, 1));
  if (n > 0) {
    k_copy_rows<<<grid_for(n * kWave, kBlock), kBlock, 0, s>>>(src.ptr, src.col, src.val, idx, n,
                                                              out.ptr, out.col, out.val);
    check_launch_sp("copy_rows");
  }
}

void csr_from_dense(const float* x, int ld, int64_t n, int cols, Csr& out, Arena& a,
                    Arena& scratch, hipStream_t s) {
  out.n = n;
  out.cols = cols;
  uint32_t* cnt = scratch.alloc<uint32_t>(n + 1);
  uint32_t* total = scratch.alloc<uint32_t>(1);
  uint32_t* sums = scratch.alloc<uint32_t>(scan_sums_needed(n));
  k_count_nz<<<grid_for(n * kWave, kBlock), kBlock, 0, s>>>(x, ld, n, cols, cnt);
  check_launch_sp("count_nz");
  exclusive_scan_u32(cnt, n, total, sums, s);
  out.ptr = a.alloc<int64_t>(n + 1);
  k_widen_ptr<<<grid_for(n + 1, kBlock), kBlock, 0, s>>>(cnt, n, total, out.ptr);
  check_launch_sp("widen_ptr");
  uint32_t h_total = 0;
  MASK_HIP(hipMemcpyAsync(&h_total, total, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  MASK_HIP(hipStreamSynchronize(s));
  out.nnz = h_total;
  out.col = a.alloc<int32_t>(std::max<int64_t>(out.nnz, 1));
  out.val = a.alloc<float>(std::max<int64_t>(out.nnz, 1));
  k_fill_nz<<<grid_for(n * kWave, kBlock), kBlock, 0, s>>>(x, ld, n, cols, out.ptr, out.col,
                                                          out.val);
  check_launch_sp("fill_nz");
}

void csr_norms64(const Csr& x, double* out, hipStream_t s) {
  if (x.n <= 0) return;
  k_csr_norms64<<<grid_for(x.n * kWave, kBlock), kBlock, 0, s>>>(x.ptr, x.val, x.n, out);
  check_launch_sp("csr_norms64");
}

void dense_norms64(const float* x, int ld, int64_t n, int cols, double* out, hipStream_t s) {
  if (n <= 0) return;
  k_dense_norms64<<<grid_for(n * kWave, kBlock), kBlock, 0, s>>>(x, ld, n, cols, out);
  check_launch_sp("dense_norms64");
}

void csr_validate(const int64_t* ptr, const int32_t* col, int64_t n, int cols, int64_t nnz,
                  uint32_t* flag, hipStream_t s) {
  fill_u32(flag, 1, 0u, s);
  if (n <= 0) return;
  k_csr_validate<<<grid_for(n, kBlock), kBlock, 0, s>>>(ptr, col, n, cols, nnz, flag);
  check_launch_sp("csr_validate");
}

void kmeans_sparse(const Csr& items, int ld, int n_chunks, int k, int iters, const float* init,
                   float* protos, int32_t* labels, double* inertia_log, Arena& scratch,
                   hipStream_t s) {
  const int64_t n = items.n, np = (int64_t)n_chunks * k;
  const int cols = items.cols;
  // group offsets: split() of Algorithm 1
  std::vector<int64_t> off(n_chunks + 1);
  {
    const int64_t base = n / n_chunks, extra = n % n_chunks;
    off[0] = 0;
    for (int c = 0; c < n_chunks; ++c) off[c + 1] = off[c] + base + (c < extra ? 1 : 0);
  }
  int64_t* d_off = scratch.alloc<int64_t>(n_chunks + 1);
  MASK_HIP(hipMemcpyAsync(d_off, off.data(), (n_chunks + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  double* xnorm = scratch.alloc<double>(n);
  double* pnorm = scratch.alloc<double>(np);
  double* best = scratch.alloc<double>(n);
  float* PT = scratch.alloc<float>(np * cols);
  uint32_t* keys = scratch.alloc<uint32_t>(n);
  uint32_t* vals = scratch.alloc<uint32_t>(n);
  uint32_t* member_off = scratch.alloc<uint32_t>(np + 1);
  SortWork sw;
  sort_work_alloc(sw, n, false, scratch);
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < np) ++bits;

  csr_norms64(items, xnorm, s);
  if (init) {
    MASK_HIP(hipMemcpyAsync(protos, init, np * ld * sizeof(float), hipMemcpyDeviceToDevice, s));
  } else {
    k_zero_f32<<<grid_for(np * ld, kBlock), kBlock, 0, s>>>(protos, np * ld);
    check_launch_sp("zero");
    k_init_first_csr<<<grid_for(np * kWave, kBlock), kBlock, 0, s>>>(
        items.ptr, items.col, items.val, d_off, n_chunks, k, protos, ld);
    check_launch_sp("init_first_csr");
  }
  dense_norms64(protos, ld, np, cols, pnorm, s);

  const int tiles_d = (cols + 31) / 32, tiles_j = (k + 31) / 32;
  auto transpose = [&]() {
    k_transpose_groups<<<(unsigned)((int64_t)n_chunks * tiles_d * tiles_j), kBlock, 0, s>>>(
        protos, ld, k, cols, tiles_d, tiles_j, PT);
    check_launch_sp("transpose_groups");
  };
  auto assign = [&]() {
    ScopedTiming timing("assign_csr", s);
    const unsigned g = grid_for(n * kWave, kBlock);
    if (k <= 256)
      k_assign_csr<4, 4><<<g, kBlock, 0, s>>>(items.ptr, items.col, items.val, xnorm, PT, pnorm,
                                              d_off, n_chunks, k, cols, n, labels, best);
    else
      k_assign_csr<8, 4><<<g, kBlock, 0, s>>>(items.ptr, items.col, items.val, xnorm, PT, pnorm,
                                              d_off, n_chunks, k, cols, n, labels, best);
    check_launch_sp("assign_csr");
  };
  transpose();
  for (int t = 0; t < iters; ++t) {
    assign();
    if (inertia_log) {
      k_group_sum<<<grid_for((int64_t)n_chunks * kWave, kBlock), kBlock, 0, s>>>(
          best, d_off, n_chunks, inertia_log + (int64_t)t * n_chunks);
      check_launch_sp("group_sum");
    }
    {
      ScopedTiming timing("member_sort", s);
      k_labels_keys<<<grid_for(n, kBlock), kBlock, 0, s>>>(labels, n, keys, vals);
      check_launch_sp("labels_keys");
      radix_sort_u32(keys, vals, n, bits, sw, s);
      offsets_from_sorted(keys, n, np, member_off, s);
    }
    {
      ScopedTiming timing("update_csr", s);
      k_update_csr<<<(unsigned)np, kWave, 0, s>>>(items.ptr, items.col, items.val, vals,
                                                  member_off, cols, protos, ld, pnorm);
      check_launch_sp("update_csr");
    }
    transpose();
  }
  assign();
}

}  // namespace mask

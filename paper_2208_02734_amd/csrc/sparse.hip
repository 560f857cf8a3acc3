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

// Prototype c*k+j := item off[c] + j mod (group size), scattered into a
// zeroed dense row.
__global__ __launch_bounds__(kBlock) void k_init_first_csr(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, const int64_t* __restrict__ chunk_off, int n_chunks, int k,
    float* __restrict__ P, int ld) {
  const int lane = threadIdx.x % kWave;
  const int64_t p = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (p >= (int64_t)n_chunks * k) return;
  const int64_t c = p / k, m = chunk_off[c + 1] - chunk_off[c];
  const int64_t item = chunk_off[c] + (p % k) % m;
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

// Update: FP64 sums of each prototype's members, split into work items of at
// most S members (S chosen per level from the rows' density), one wave per
// item.  Item slots are laid out as in the dense update: prototype p owns
// [p + m0 / S, p + 1 + m1 / S), which holds at least max(1, ceil(cnt / S))
// slots.  A prototype with one item is finished by it; the items of a larger
// one write dense FP64 partial sums (rows of a compact buffer numbered by an
// exclusive scan over the prototypes) that k_update_csr_finish adds in item
// order.  Sums run over a window of kSumWin columns at a time in LDS; a
// member's columns are distinct, so its lanes never collide, and one wave's
// LDS accesses complete in program order, so members add in item order.
constexpr int kSumWin = 4096;

__global__ void k_sp_slots(const uint32_t* __restrict__ member_off, int64_t n_protos, int S,
                           int32_t* __restrict__ slot_proto, uint32_t* __restrict__ pcount) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_protos) return;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  const uint32_t cnt = m1 - m0;
  const int64_t b0 = p + m0 / S, b1 = p + 1 + m1 / S;
  const int64_t nch = cnt == 0 ? 1 : (cnt + S - 1) / S;
  for (int64_t t = b0; t < b1; ++t) slot_proto[t] = (t - b0 < nch) ? (int32_t)p : -1;
  pcount[p] = cnt > (uint32_t)S ? (uint32_t)nch : 0u;
}

// The item's member entries are staged in LDS first when they fit (all
// their loads in flight at once), so the per-window passes read LDS only.
constexpr int kStage = 1024;

__global__ __launch_bounds__(kWave) void k_update_csr_items(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, const uint32_t* __restrict__ members,
    const uint32_t* __restrict__ member_off, const int32_t* __restrict__ slot_proto,
    const uint32_t* __restrict__ pbase, int S, int cols, float* __restrict__ P, int ld,
    double* __restrict__ pnorm, double* __restrict__ part) {
  __shared__ double acc[kSumWin];
  __shared__ int32_t s_col[kStage];
  __shared__ float s_val[kStage];
  __shared__ uint32_t s_moff[kWave + 1];  // staged entry offset of each member
  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  const int32_t p = slot_proto[t];
  if (p < 0) return;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  const uint32_t cnt = m1 - m0;
  if (cnt == 0) return;  // keeps its row and norm
  const int64_t j = t - ((int64_t)p + m0 / S);
  const uint32_t a = m0 + (uint32_t)j * S;
  const uint32_t b = min(m1, a + (uint32_t)S);
  const bool single = cnt <= (uint32_t)S;
  const double inv_n = 1.0 / (double)cnt;
  double* prow = single ? nullptr : part + (int64_t)(pbase[p] + j) * cols;

  // stage when the item has at most 64 members and kStage entries
  bool staged = false;
  if (b - a <= (uint32_t)kWave) {
    const uint32_t mi = a + lane;
    int64_t beg = 0;
    uint32_t len = 0;
    if (mi < b) {
      const int64_t it = members[mi];
      beg = ptr[it];
      len = (uint32_t)(ptr[it + 1] - beg);
    }
    uint32_t x = len;  // inclusive scan over the lanes
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    const uint32_t total = __shfl(x, kWave - 1);
    if (total <= (uint32_t)kStage) {
      staged = true;
      s_moff[lane + 1] = x;
      if (lane == 0) s_moff[0] = 0;
      const uint32_t nm = b - a;
      for (uint32_t f = 0; f < nm; ++f) {
        const int64_t fb = __shfl(beg, (int)f);
        const uint32_t fl = __shfl(len, (int)f);
        const uint32_t fo = __shfl(x - len, (int)f);
        for (uint32_t e = lane; e < fl; e += kWave) {
          s_col[fo + e] = col[fb + e];
          s_val[fo + e] = val[fb + e];
        }
      }
    }
  }

  double nrm = 0.0;
  for (int d0 = 0; d0 < cols; d0 += kSumWin) {
    const int w = min(kSumWin, cols - d0);
    for (int c = lane; c < w; c += kWave) acc[c] = 0.0;
    if (staged) {
      for (uint32_t f = 0; f < b - a; ++f) {
        const uint32_t e0 = s_moff[f], e1 = s_moff[f + 1];
        for (uint32_t e = e0 + lane; e < e1; e += kWave) {
          const int cc = s_col[e] - d0;
          if (cc >= 0 && cc < w) acc[cc] += (double)s_val[e];
        }
      }
    } else {
      // a member's columns are distinct, so its adds commute: load 4 entries
      // per lane before adding them
      for (uint32_t m = a; m < b; ++m) {
        const int64_t it = members[m];
        const int64_t eb = ptr[it], ee = ptr[it + 1];
        for (int64_t e0 = eb; e0 < ee; e0 += 4 * kWave) {
          int cc[4];
          float vv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + lane + u * kWave;
            cc[u] = e < ee ? col[e] - d0 : -1;
            vv[u] = e < ee ? val[e] : 0.f;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (cc[u] >= 0 && cc[u] < w) acc[cc[u]] += (double)vv[u];
        }
      }
    }
    if (single) {
      for (int c = lane; c < w; c += kWave) {
        const float v = (float)(acc[c] * inv_n);
        P[(int64_t)p * ld + d0 + c] = v;
        nrm = fma((double)v, (double)v, nrm);
      }
    } else {
      for (int c = lane; c < w; c += kWave) prow[d0 + c] = acc[c];
    }
  }
  if (single) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nrm += __shfl_xor(nrm, o);
    if (lane == 0) pnorm[p] = nrm;
  }
}

// Prototypes with more than one item: one wave per (prototype, block of
// kFinCols columns) adds the item sums in item order (8 loads in flight, adds
// in sequence), writes the FP32 mean and the block's FP64 squared norm;
// k_update_csr_norm adds the blocks in order.
constexpr int kFinCols = 512;

__global__ __launch_bounds__(kBlock) void k_update_csr_finish(
    const uint32_t* __restrict__ member_off, int64_t n_protos, int S,
    const uint32_t* __restrict__ pbase, const double* __restrict__ part, int cols, int nblk,
    float* __restrict__ P, int ld, double* __restrict__ bnorm) {
  const int lane = threadIdx.x % kWave;
  const int64_t wv = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t p = wv / nblk;
  const int blk = (int)(wv % nblk);
  if (p >= n_protos) return;
  const uint32_t cnt = member_off[p + 1] - member_off[p];
  if (cnt <= (uint32_t)S) return;
  const int nch = (int)((cnt + S - 1) / S);
  const double* base = part + (int64_t)pbase[p] * cols;
  const double inv_n = 1.0 / (double)cnt;
  double nrm = 0.0;
  const int c1 = min(cols, (blk + 1) * kFinCols);
  for (int c = blk * kFinCols + lane; c < c1; c += kWave) {
    double sum = 0.0;
    int i = 0;
    for (; i + 8 <= nch; i += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = base[(int64_t)(i + u) * cols + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += v[u];
    }
    for (; i < nch; ++i) sum += base[(int64_t)i * cols + c];
    const float v = (float)(sum * inv_n);
    P[p * ld + c] = v;
    nrm = fma((double)v, (double)v, nrm);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) nrm += __shfl_xor(nrm, o);
  if (lane == 0) bnorm[p * nblk + blk] = nrm;
}

__global__ void k_update_csr_norm(const uint32_t* __restrict__ member_off, int64_t n_protos,
                                  int S, const double* __restrict__ bnorm, int nblk,
                                  double* __restrict__ pnorm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_protos) return;
  if (member_off[p + 1] - member_off[p] <= (uint32_t)S) return;
  double a = 0.0;
  for (int b = 0; b < nblk; ++b) a += bnorm[p * nblk + b];
  pnorm[p] = a;
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
                   hipStream_t s, const char* level_scope) {
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
  // update work items: about 6400 non-zeros each, and at most 256 MB of
  // partial sums (2n / S item rows of cols doubles bound them)
  const double avg_nnz = n > 0 ? (double)items.nnz / (double)n : 1.0;
  int64_t S = std::max<int64_t>(1, (int64_t)(6400.0 / std::max(avg_nnz, 1.0)));
  const int64_t part_budget = (int64_t)256 << 20;
  S = std::max<int64_t>(S, (2 * n * (int64_t)cols * 8 + part_budget - 1) / part_budget);
  S = std::min<int64_t>(S, (int64_t)1 << 20);
  const int64_t n_slots = np + n / S;
  const int64_t part_rows = 2 * (n / S) + 2;
  int32_t* slot_proto = scratch.alloc<int32_t>(n_slots);
  uint32_t* pbase = scratch.alloc<uint32_t>(np + 1);
  uint32_t* scan_sums = scratch.alloc<uint32_t>(scan_sums_needed(np));
  double* part = scratch.alloc<double>(part_rows * cols);
  const int nblk = (cols + kFinCols - 1) / kFinCols;
  double* bnorm = scratch.alloc<double>(np * nblk);
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
    ScopedTiming level_timing(level_scope, s, level_scope != nullptr);
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
      k_sp_slots<<<grid_for(np, kBlock), kBlock, 0, s>>>(member_off, np, (int)S, slot_proto,
                                                        pbase);
      check_launch_sp("sp_slots");
      exclusive_scan_u32(pbase, np, nullptr, scan_sums, s);
      k_update_csr_items<<<(unsigned)n_slots, kWave, 0, s>>>(
          items.ptr, items.col, items.val, vals, member_off, slot_proto, pbase, (int)S, cols,
          protos, ld, pnorm, part);
      check_launch_sp("update_csr_items");
      k_update_csr_finish<<<grid_for(np * nblk * kWave, kBlock), kBlock, 0, s>>>(
          member_off, np, (int)S, pbase, part, cols, nblk, protos, ld, bnorm);
      check_launch_sp("update_csr_finish");
      k_update_csr_norm<<<grid_for(np, kBlock), kBlock, 0, s>>>(member_off, np, (int)S, bnorm,
                                                               nblk, pnorm);
      check_launch_sp("update_csr_norm");
    }
    transpose();
  }
  assign();
}

}  // namespace mask

// Batched per-group k-means (the kmeans(nCentroids, points) step of
// Algorithm 1, run for every group of a level in one launch).
//
// Assignment (plain FP32 form):
//   s_ij = x_i . c_j - |c_j|^2 / 2 on MFMA (v_mfma_f32_32x32x2_f32), so the
//   nearest prototype maximises s_ij.  Prototypes are the MFMA rows and points
//   the columns: each lane owns one point and sixteen prototypes of every
//   32x32 tile, so the running best is kept in-lane.  The four best screened
//   values certify the result: when the gap to the runner-up exceeds twice a
//   rounding bound of s, the screened winner is the exact one; otherwise the
//   point is re-scored in direct form (sum of squared differences, FP32) on
//   the two or three prototypes inside the uncertainty window, or on every
//   prototype of its group when the fourth is inside it too.
//
// Update: members of each prototype are listed in item order (stable radix
// sort of the labels), summed in FP64 in that fixed order, and divided by the
// count; an empty prototype keeps its value.  The inertia of the assignment
// under the old prototypes is accumulated in FP64 on the same pass.
#include <cfloat>

#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace mask {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8),
// each with its own L2.  Give every XCD a contiguous range of logical tiles,
// so tiles of one group, which read the same prototypes, share an L2.
__device__ inline unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, i = b >> 3;
  const unsigned q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + i;
}

template <int DP>
struct LdsWidth {
  // Row stride of a prototype tile in LDS: DP + padding with stride = 4
  // (mod 32) floats, so that the 16-byte reads of 8 consecutive lanes (8
  // different rows, same column) land in different bank groups.
  static constexpr int value = DP + ((((4 - DP) % 32) + 32) % 32);
};

__device__ inline void top4_insert(float v, int j, float& b1, int& i1, float& b2, int& i2,
                                   float& b3, int& i3, float& b4) {
  if (v > b4) {
    if (v > b3) {
      b4 = b3;
      if (v > b2) {
        b3 = b2; i3 = i2;
        if (v > b1) {
          b2 = b1; i2 = i1; b1 = v; i1 = j;
        } else {
          b2 = v; i2 = j;
        }
      } else {
        b3 = v; i3 = j;
      }
    } else {
      b4 = v;
    }
  }
}

// DP: padded dimension (multiple of 8) held in registers; PB: 32-point blocks
// per wave; TN: prototypes per LDS stage; MINB: blocks per CU the register
// budget is sized for (1 = a full 512-entry register file per wave).
template <int DP, int PB, int TN, int MINB>
__global__ __launch_bounds__(kBlock, MINB) void k_assign_l2_mfma(
    const float* __restrict__ items, int ld, const float* __restrict__ protos,
    const float* __restrict__ pnorm, const float* __restrict__ inorm,
    const int64_t* __restrict__ chunk_off, int k, int tiles_per_chunk,
    int32_t* __restrict__ labels, uint32_t* __restrict__ refine_count,
    uint32_t* __restrict__ small_list, int32_t* __restrict__ small_cand,
    uint32_t* __restrict__ full_cnt, uint32_t* __restrict__ full_list, float err_coef) {
  constexpr int KS = DP / 2;
  constexpr int LDW = LdsWidth<DP>::value;
  constexpr int BM = 4 * 32 * PB;
  constexpr int F4_PER_ROW = DP / 4;
  constexpr int LOADS = TN * F4_PER_ROW / kBlock;
  static_assert(LOADS * kBlock == TN * F4_PER_ROW, "tile must split evenly over the block");
  static_assert(TN % 32 == 0 && TN <= kBlock, "TN");

  __shared__ float s_c[2][TN * LDW];
  __shared__ float s_hn[2][TN];

  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = (int)(lb / (unsigned)tiles_per_chunk);
  const int tile = (int)(lb % (unsigned)tiles_per_chunk);
  const int64_t c0 = chunk_off[chunk], c1 = chunk_off[chunk + 1];
  const int64_t pbase = c0 + (int64_t)tile * BM;
  if (pbase >= c1) return;  // uniform for the whole block, before any barrier

  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int h = lane >> 5, col = lane & 31;

  // Point fragments: MFMA k-slot (s, h) is dimension h*KS + s.
  float bf[PB][KS];
  float xn[PB];
  int64_t pidx[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t p = pbase + (wave * PB + pb) * 32 + col;
    pidx[pb] = p;
    const bool ok = p < c1;
    xn[pb] = ok ? inorm[p] : 0.f;
    const float* row = items + (ok ? p : c0) * (int64_t)ld;
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      const int c = h * KS + s;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (ok && c < ld) v = *reinterpret_cast<const float4*>(row + c);
      bf[pb][s] = v.x; bf[pb][s + 1] = v.y; bf[pb][s + 2] = v.z; bf[pb][s + 3] = v.w;
    }
  }

  const float* cbase = protos + (int64_t)chunk * k * ld;
  const float* nbase = pnorm + (int64_t)chunk * k;
  const int ntiles = (k + TN - 1) / TN;

  float4 stage[LOADS];
  float hstage = INFINITY;
  auto load_tile = [&](int t) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int idx = threadIdx.x + i * kBlock;
      const int row = idx / F4_PER_ROW, c4 = idx % F4_PER_ROW;
      const int j = t * TN + row;
      stage[i] = (j < k && c4 * 4 < ld)
                     ? *reinterpret_cast<const float4*>(cbase + (int64_t)j * ld + c4 * 4)
                     : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (threadIdx.x < TN) {
      const int j = t * TN + threadIdx.x;
      hstage = (j < k) ? 0.5f * nbase[j] : INFINITY;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int idx = threadIdx.x + i * kBlock;
      const int row = idx / F4_PER_ROW, c4 = idx % F4_PER_ROW;
      *reinterpret_cast<float4*>(&s_c[buf][row * LDW + c4 * 4]) = stage[i];
    }
    if (threadIdx.x < TN) s_hn[buf][threadIdx.x] = hstage;
  };

  load_tile(0);
  store_tile(0);
  __syncthreads();

  float b1[PB], b2[PB], b3[PB], b4[PB];
  int i1[PB], i2[PB], i3[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    b1[pb] = b2[pb] = b3[pb] = b4[pb] = -INFINITY;
    i1[pb] = i2[pb] = i3[pb] = 0;
  }
  float hmax = 0.f;

  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    if (t + 1 < ntiles) load_tile(t + 1);
#pragma unroll
    for (int cb = 0; cb < TN / 32; ++cb) {
      floatx16 acc[PB];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float hv = s_hn[buf][cb * 32 + 8 * (i >> 2) + 4 * h + (i & 3)];
        if (hv < INFINITY) hmax = fmaxf(hmax, hv);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) acc[pb][i] = -hv;
      }
      const float* arow = &s_c[buf][(cb * 32 + col) * LDW + h * KS];
#pragma unroll
      for (int s = 0; s < KS; s += 4) {
        const float4 a4 = *reinterpret_cast<const float4*>(arow + s);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          acc[pb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bf[pb][s + 0], acc[pb], 0, 0, 0);
          acc[pb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bf[pb][s + 1], acc[pb], 0, 0, 0);
          acc[pb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bf[pb][s + 2], acc[pb], 0, 0, 0);
          acc[pb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bf[pb][s + 3], acc[pb], 0, 0, 0);
        }
      }
      const int jbase = t * TN + cb * 32 + 4 * h;
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int j = jbase + 8 * (i >> 2) + (i & 3);
          top4_insert(acc[pb][i], j, b1[pb], i1[pb], b2[pb], i2[pb], b3[pb], i3[pb], b4[pb]);
        }
      }
    }
    if (t + 1 < ntiles) store_tile(buf ^ 1);
    __syncthreads();
  }

  // Lanes l and l^32 hold the same point and disjoint halves of the rows.
  hmax = fmaxf(hmax, __shfl_xor(hmax, 32));
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const float o1 = __shfl_xor(b1[pb], 32), o2 = __shfl_xor(b2[pb], 32),
                o3 = __shfl_xor(b3[pb], 32), o4 = __shfl_xor(b4[pb], 32);
    const int oi1 = __shfl_xor(i1[pb], 32), oi2 = __shfl_xor(i2[pb], 32),
              oi3 = __shfl_xor(i3[pb], 32);
    if (h == 0) {
      top4_insert(o1, oi1, b1[pb], i1[pb], b2[pb], i2[pb], b3[pb], i3[pb], b4[pb]);
      top4_insert(o2, oi2, b1[pb], i1[pb], b2[pb], i2[pb], b3[pb], i3[pb], b4[pb]);
      top4_insert(o3, oi3, b1[pb], i1[pb], b2[pb], i2[pb], b3[pb], i3[pb], b4[pb]);
      top4_insert(o4, -1, b1[pb], i1[pb], b2[pb], i2[pb], b3[pb], i3[pb], b4[pb]);
      const int64_t p = pidx[pb];
      if (p < c1) {
        labels[p] = chunk * k + i1[pb];
        // |error of a screened value| <= err_coef * (|x|^2 + 3 max|c|^2); the
        // exact winner lies in {j : s_j >= b1 - 2e}.
        const float w = 2.0f * err_coef * (xn[pb] + 6.0f * hmax);
        if (k > 1 && !(b1[pb] - b2[pb] > w)) {
          if (b1[pb] - b4[pb] > w) {
            int c0 = i1[pb], c1i = i2[pb], c2 = (b1[pb] - b3[pb] > w) ? -1 : i3[pb];
            // ascending order, -1 last
            if (c1i < c0) { const int t = c0; c0 = c1i; c1i = t; }
            if (c2 >= 0) {
              if (c2 < c0) { const int t = c2; c2 = c1i; c1i = c0; c0 = t; }
              else if (c2 < c1i) { const int t = c2; c2 = c1i; c1i = t; }
            }
            const uint32_t slot = atomicAdd(&refine_count[0], 1u);
            small_list[slot] = (uint32_t)p;
            small_cand[3 * slot] = c0;
            small_cand[3 * slot + 1] = c1i;
            small_cand[3 * slot + 2] = c2;
          } else {
            // per-group list: slots c0 .. c0 + group size - 1 belong to this group
            const uint32_t slot = atomicAdd(&full_cnt[chunk], 1u);
            full_list[c0 + slot] = (uint32_t)p;
          }
        }
      }
    }
  }
}

// Direct-form distance in a fixed order, accumulated in FP64: the difference
// of two FP32 values is exact in FP64, so the result carries only the FP64
// rounding of the squares and sums.  Four partial sums over the float4 lanes
// of the row, combined as (p0+p1)+(p2+p3).  ld is a multiple of 4 and the
// padding is zero in both rows.
template <int METRIC>
__device__ inline double direct_dist64(const float* __restrict__ x, const float* __restrict__ c,
                                       int ld) {
  const float4* x4 = reinterpret_cast<const float4*>(x);
  const float4* c4 = reinterpret_cast<const float4*>(c);
  double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
  for (int i = 0; i < ld / 4; ++i) {
    const float4 a = x4[i], b = c4[i];
    const double dx = (double)a.x - (double)b.x, dy = (double)a.y - (double)b.y,
                 dz = (double)a.z - (double)b.z, dw = (double)a.w - (double)b.w;
    if (METRIC == 0) {
      p0 = fma(dx, dx, p0); p1 = fma(dy, dy, p1); p2 = fma(dz, dz, p2); p3 = fma(dw, dw, p3);
    } else {
      p0 += fabs(dx); p1 += fabs(dy); p2 += fabs(dz); p3 += fabs(dw);
    }
  }
  return (p0 + p1) + (p2 + p3);
}

__device__ inline int find_chunk(const int64_t* __restrict__ off, int n_chunks, int64_t p) {
  int lo = 0, hi = n_chunks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Points with two or three candidates: four lanes per point, one candidate
// per lane, then the nearest (lowest index on exact ties) over the four.
template <int METRIC>
__global__ __launch_bounds__(kBlock) void k_refine_small(
    const float* __restrict__ items, int ld, const float* __restrict__ protos,
    const int64_t* __restrict__ chunk_off, int n_chunks, int k,
    const uint32_t* __restrict__ refine_count, const uint32_t* __restrict__ small_list,
    const int32_t* __restrict__ small_cand, int32_t* __restrict__ labels,
    unsigned long long* __restrict__ stats) {
  const uint32_t count = refine_count[0];
  const int64_t stride = (int64_t)gridDim.x * kBlock / 4;
  const int slot = threadIdx.x & 3;
  for (int64_t e = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 4;; e += stride) {
    // uniform trip count per wave: a wave covers 16 consecutive entries
    const int64_t wave_first = e - (threadIdx.x % kWave) / 4;
    if (wave_first >= (int64_t)count) break;
    const bool valid = e < (int64_t)count;
    double dist = INFINITY;
    int cand = 0x7fffffff;
    int64_t p = 0;
    int chunk = 0;
    if (valid) {
      p = small_list[e];
      chunk = find_chunk(chunk_off, n_chunks, p);
      const int c = slot < 3 ? small_cand[3 * e + slot] : -1;
      if (c >= 0) {
        cand = c;
        dist = direct_dist64<METRIC>(items + p * ld, protos + ((int64_t)chunk * k + c) * ld, ld);
      }
    }
#pragma unroll
    for (int o = 1; o <= 2; o <<= 1) {
      const double od = __shfl_xor(dist, o);
      const int oc = __shfl_xor(cand, o);
      if (od < dist || (od == dist && oc < cand)) { dist = od; cand = oc; }
    }
    if (valid && slot == 0) labels[p] = chunk * k + cand;
    if (stats) {
      const uint64_t b = __ballot(valid && slot == 0);
      if ((threadIdx.x % kWave) == 0 && b) atomicAdd(&stats[0], (unsigned long long)__popcll(b));
    }
  }
}

// Points whose uncertainty window holds four or more prototypes are listed
// per group (full_list[off_c + i], i < full_cnt[c]).  One block builds the
// list of 64-point tiles over all groups.
__global__ __launch_bounds__(kBlock) void k_full_tiles(const uint32_t* __restrict__ full_cnt,
                                                      int n_chunks, uint2* __restrict__ tiles,
                                                      uint32_t* __restrict__ tile_total) {
  __shared__ uint32_t s_wave[kBlock / kWave];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  uint32_t carry = 0;
  for (int base = 0; base < n_chunks; base += kBlock) {
    const int c = base + threadIdx.x;
    const uint32_t nt = c < n_chunks ? (full_cnt[c] + 63u) / 64u : 0u;
    uint32_t x = nt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_wave[wave] = x;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      if (w < wave) wbase += s_wave[w];
      tot += s_wave[w];
    }
    __syncthreads();
    const uint32_t ex = carry + wbase + x - nt;
    for (uint32_t t = 0; t < nt; ++t) tiles[ex + t] = make_uint2((uint32_t)c, t);
    carry += tot;
  }
  if (threadIdx.x == 0) *tile_total = carry;
}

// One wave per (tile of up to 64 listed points of one group, range of that
// group's prototypes).  Lane i owns point i of the tile, whose row is staged
// in LDS (row stride ld + 4 floats, so 16-byte reads of different rows spread
// over the banks); every lane walks the same prototypes, read with
// wave-uniform loads, and keeps its nearest (FP64 direct form, lowest index
// on exact ties).  Partial results per range go to
// partial_d/partial_j[list slot * S + s].
template <int METRIC>
__global__ __launch_bounds__(kWave) void k_refine_full(
    const float* __restrict__ items, int ld, const float* __restrict__ protos,
    const int64_t* __restrict__ chunk_off, int k, const uint32_t* __restrict__ full_cnt,
    const uint32_t* __restrict__ full_list, const uint2* __restrict__ tiles,
    const uint32_t* __restrict__ tile_total, int S, double* __restrict__ partial_d,
    int32_t* __restrict__ partial_j) {
  extern __shared__ float4 s_x[];  // 64 rows x (ld4 + 1) float4
  const int lane = threadIdx.x;
  const int ld4 = ld / 4, xs = ld4 + 1;
  const int s = blockIdx.y;
  const int R = (k + S - 1) / S;
  const int jlo = s * R, jhi = min(k, jlo + R);
  const uint32_t total = *tile_total;
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    const uint2 tc = tiles[t];
    const int c = (int)tc.x;
    const uint32_t cnt = full_cnt[c];
    const int np = (int)min(64u, cnt - tc.y * 64u);
    const int64_t qbase = chunk_off[c] + (int64_t)tc.y * 64;
    __syncthreads();  // the previous tile's rows are no longer read
    for (int i = lane; i < np * ld4; i += kWave) {
      const int row = i / ld4, c4 = i % ld4;
      const int64_t p = full_list[qbase + row];
      s_x[row * xs + c4] = reinterpret_cast<const float4*>(items + p * ld)[c4];
    }
    __syncthreads();
    const float4* xr = s_x + (lane < np ? lane : 0) * xs;
    double best_d = INFINITY;
    int best_j = 0x7fffffff;
    const float* cbase = protos + (int64_t)c * k * ld;
    for (int j = jlo; j < jhi; ++j) {
      const float4* crow = reinterpret_cast<const float4*>(cbase + (int64_t)j * ld);
      double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
      for (int i = 0; i < ld4; ++i) {
        const float4 a = xr[i], b = crow[i];
        const double dx = (double)a.x - (double)b.x, dy = (double)a.y - (double)b.y,
                     dz = (double)a.z - (double)b.z, dw = (double)a.w - (double)b.w;
        if (METRIC == 0) {
          p0 = fma(dx, dx, p0); p1 = fma(dy, dy, p1); p2 = fma(dz, dz, p2); p3 = fma(dw, dw, p3);
        } else {
          p0 += fabs(dx); p1 += fabs(dy); p2 += fabs(dz); p3 += fabs(dw);
        }
      }
      const double dd = (p0 + p1) + (p2 + p3);
      if (dd < best_d) { best_d = dd; best_j = j; }  // j ascends: ties keep the lower
    }
    if (lane < np) {
      partial_d[(qbase + lane) * S + s] = best_d;
      partial_j[(qbase + lane) * S + s] = best_j;
    }
  }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// Squared-Euclidean variant of the whole-group re-scoring on FP64 MFMA
// (v_mfma_f64_16x16x4f64): s_ij = x_i . c_j - |c_j|^2 / 2 in FP64 from the
// FP32 coordinates, whose rounding (~1e-10 absolute at these norms) is far
// below any gap that matters.  Block = 4 waves; one (tile of up to 64 listed
// points of one group, range of that group's prototypes) per iteration; wave
// w owns points 16w..16w+15 (MFMA columns), prototypes are the rows and are
// staged through LDS 64 at a time.  MFMA k-slot (s, g) is dimension g*KS+s.
// Operand lanes: A[i][k] from lane 16k+i, B[k][j] from lane 16k+j; result
// register r of lane l holds row 4r + l/16, column l%16.
// Each point keeps the largest s (lowest index on exact ties); the negated
// value goes to partial_d so the merge takes the smallest.
template <int DP>
__global__ __launch_bounds__(kBlock) void k_refine_f64(
    const float* __restrict__ items, int ld, const float* __restrict__ protos,
    const double* __restrict__ pnorm64, const int64_t* __restrict__ chunk_off, int k,
    const uint32_t* __restrict__ full_cnt, const uint32_t* __restrict__ full_list,
    const uint2* __restrict__ tiles, const uint32_t* __restrict__ tile_total, int S,
    double* __restrict__ partial_d, int32_t* __restrict__ partial_j) {
  constexpr int KS = DP / 4;
  constexpr int TP = 64;
  constexpr int LDW = DP + 4;
  constexpr int F4_PER_ROW = DP / 4;
  __shared__ float s_c[TP * LDW];
  __shared__ double s_hn[TP];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int col = lane & 15, g = lane >> 4;
  const int s = blockIdx.y;
  const int R = (k + S - 1) / S;
  const int jlo = s * R, jhi = min(k, jlo + R);
  const uint32_t total = *tile_total;
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    const uint2 tc = tiles[t];
    const int c = (int)tc.x;
    const uint32_t cnt = full_cnt[c];
    const int np = (int)min(64u, cnt - tc.y * 64u);
    const int64_t qbase = chunk_off[c] + (int64_t)tc.y * 64;
    const int pt = wave * 16 + col;  // this lane's point within the tile
    double b[KS];
    {
      const int64_t p = pt < np ? (int64_t)full_list[qbase + pt] : 0;
      const float* row = items + p * ld;
#pragma unroll
      for (int i = 0; i < KS; i += 4) {
        const int cc = g * KS + i;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (pt < np && cc < ld) v = *reinterpret_cast<const float4*>(row + cc);
        b[i] = v.x; b[i + 1] = v.y; b[i + 2] = v.z; b[i + 3] = v.w;
      }
    }
    double best = -INFINITY;
    int bj = 0x7fffffff;
    const float* cbase = protos + (int64_t)c * k * ld;
    const double* nbase = pnorm64 + (int64_t)c * k;
    for (int j0 = jlo; j0 < jhi; j0 += TP) {
      __syncthreads();  // the previous prototype tile is no longer read
      for (int idx = threadIdx.x; idx < TP * F4_PER_ROW; idx += kBlock) {
        const int row = idx / F4_PER_ROW, c4 = idx % F4_PER_ROW;
        const int j = j0 + row;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < jhi && c4 * 4 < ld) v = *reinterpret_cast<const float4*>(cbase + (int64_t)j * ld + c4 * 4);
        *reinterpret_cast<float4*>(&s_c[row * LDW + c4 * 4]) = v;
      }
      if (threadIdx.x < TP) {
        const int j = j0 + threadIdx.x;
        s_hn[threadIdx.x] = (j < jhi) ? 0.5 * nbase[j] : INFINITY;
      }
      __syncthreads();
#pragma unroll
      for (int pb = 0; pb < TP / 16; ++pb) {
        doublex4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = -s_hn[pb * 16 + 4 * r + g];  // row 4r + lane/16
        const float* arow = &s_c[(pb * 16 + col) * LDW + g * KS];
#pragma unroll
        for (int i = 0; i < KS; i += 4) {
          const float4 a4 = *reinterpret_cast<const float4*>(arow + i);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a4.x, b[i], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a4.y, b[i + 1], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a4.z, b[i + 2], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a4.w, b[i + 3], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = j0 + pb * 16 + 4 * r + g;
          if (acc[r] > best) { best = acc[r]; bj = j; }  // padded rows hold -inf
        }
      }
    }
    // lanes col, col+16, col+32, col+48 hold the same point
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
      const double ov = __shfl_xor(best, o);
      const int oj = __shfl_xor(bj, o);
      if (ov > best || (ov == best && oj < bj)) { best = ov; bj = oj; }
    }
    if (g == 0 && pt < np) {
      partial_d[(qbase + pt) * S + s] = -best;
      partial_j[(qbase + pt) * S + s] = bj;
    }
  }
}

// Final label of every listed point: the nearest over the S ranges.
__global__ __launch_bounds__(kBlock) void k_refine_merge(
    const int64_t* __restrict__ chunk_off, int k, const uint32_t* __restrict__ full_cnt,
    const uint32_t* __restrict__ full_list, const uint2* __restrict__ tiles,
    const uint32_t* __restrict__ tile_total, int S, const double* __restrict__ partial_d,
    const int32_t* __restrict__ partial_j, int32_t* __restrict__ labels,
    unsigned long long* __restrict__ stats) {
  const int lane = threadIdx.x % kWave;
  const uint32_t total = *tile_total;
  const uint32_t n_waves = gridDim.x * (kBlock / kWave);
  for (uint32_t t = (blockIdx.x * kBlock + threadIdx.x) / kWave; t < total; t += n_waves) {
    const uint2 tc = tiles[t];
    const int c = (int)tc.x;
    const uint32_t i = tc.y * 64u + lane;
    if (i >= full_cnt[c]) continue;
    const int64_t q = chunk_off[c] + i;
    double bd = INFINITY;
    int bj = 0x7fffffff;
    for (int s = 0; s < S; ++s) {
      const double d = partial_d[q * S + s];
      const int j = partial_j[q * S + s];
      if (d < bd || (d == bd && j < bj)) { bd = d; bj = j; }
    }
    labels[full_list[q]] = c * k + bj;
    if (stats) atomicAdd(&stats[1], 1ull);
  }
}

// Update of the L2 form: FP64 sums of each prototype's members, split into
// work items of at most kUpdChunk members so that a large cluster is spread
// over many waves.  Prototype p owns the item slots [p + m0 / S, p + 1 + m1 / S)
// (S = kUpdChunk, [m0, m1) its member range): at least max(1, ceil(cnt / S))
// of them, since floor(m1 / S) - floor(m0 / S) >= floor(cnt / S).  The first
// max(1, ceil(cnt / S)) slots hold its items and the rest stay empty.  A
// prototype with one item is finished by that item; the partial sums of a
// larger one are combined in item order by k_update_finish.  Every sum has a
// fixed order, so the result does not depend on scheduling.
constexpr int kUpdChunk = 64;

__global__ void k_update_slots(const uint32_t* __restrict__ member_off, int64_t n_protos,
                               int32_t* __restrict__ slot_proto) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_protos) return;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  const uint32_t cnt = m1 - m0;
  const int64_t b0 = p + m0 / kUpdChunk, b1 = p + 1 + m1 / kUpdChunk;
  const int64_t nch = cnt == 0 ? 1 : (cnt + kUpdChunk - 1) / kUpdChunk;
  for (int64_t t = b0; t < b1; ++t) slot_proto[t] = (t - b0 < nch) ? (int32_t)p : -1;
}

// Mean (unchanged when empty) written to the prototype row with its FP32 and
// FP64 squared norms; the FP64 sum of the 4-dim slice owned by one lane.
__device__ inline void finish_slice(double t0, double t1, double t2, double t3, uint32_t cnt,
                                    float4 c_old, float4* prow, bool own, float& nrm,
                                    double& nrm64) {
  float4 v = c_old;
  if (cnt > 0) {
    const double n = (double)cnt;
    v = make_float4((float)(t0 / n), (float)(t1 / n), (float)(t2 / n), (float)(t3 / n));
  }
  nrm = 0.f;
  nrm64 = 0.0;
  if (own) {
    *prow = v;
    nrm = fmaf(v.x, v.x, fmaf(v.y, v.y, fmaf(v.z, v.z, v.w * v.w)));
    nrm64 = fma((double)v.x, (double)v.x,
                fma((double)v.y, (double)v.y, fma((double)v.z, (double)v.z, (double)v.w * v.w)));
  }
}

// One wave per item slot.  LPR lanes per row (each one float4 of the row),
// 64 / LPR rows per step, U steps in flight.  Row r of the item goes to lane
// group (r % (64 / LPR)) and partial u = (r / (64 / LPR)) % U.
template <int LPR, int U>
__global__ __launch_bounds__(kBlock) void k_update_items(
    const float* __restrict__ items, int ld, const uint32_t* __restrict__ members,
    const uint32_t* __restrict__ member_off, const int32_t* __restrict__ slot_proto,
    int64_t n_slots, float* __restrict__ protos, float* __restrict__ pnorm,
    double* __restrict__ pnorm64, double* __restrict__ proto_inertia,
    double* __restrict__ part_sum, double* __restrict__ part_inert) {
  constexpr int RPW = kWave / LPR;
  const int lane = threadIdx.x % kWave;
  const int64_t t = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (t >= n_slots) return;
  const int32_t p = slot_proto[t];
  if (p < 0) return;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  const uint32_t cnt = m1 - m0;
  const int64_t j = t - ((int64_t)p + m0 / kUpdChunk);
  const uint32_t a = m0 + (uint32_t)j * kUpdChunk;
  const uint32_t b = min(m1, a + (uint32_t)kUpdChunk);
  const int f4 = ld / 4;
  const int gl = lane % LPR, h = lane / LPR;
  const bool act = gl < f4;
  const float4* prow = reinterpret_cast<const float4*>(protos + (int64_t)p * ld) + gl;
  const float4 c_old = act ? *prow : make_float4(0.f, 0.f, 0.f, 0.f);
  // the item's member ids, one per lane
  static_assert(kUpdChunk == kWave, "one member id per lane");
  const uint32_t my_id = (a + lane < b) ? members[a + lane] : 0u;
  double ps[U][4];
#pragma unroll
  for (int u = 0; u < U; ++u) ps[u][0] = ps[u][1] = ps[u][2] = ps[u][3] = 0.0;
  double inert = 0.0;
  for (uint32_t base = 0; base < b - a; base += RPW * U) {
    float4 x[U];
    bool val[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t r = base + u * RPW + h;
      val[u] = r < b - a;
      const uint32_t id = __shfl(my_id, (int)(val[u] ? r : 0));
      const float4* row = reinterpret_cast<const float4*>(items + (int64_t)id * ld);
      const float4 v = row[act ? gl : 0];
      x[u] = (val[u] && act) ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!val[u] || !act) continue;
      ps[u][0] += (double)x[u].x;
      ps[u][1] += (double)x[u].y;
      ps[u][2] += (double)x[u].z;
      ps[u][3] += (double)x[u].w;
      const double d0 = (double)x[u].x - (double)c_old.x, d1 = (double)x[u].y - (double)c_old.y;
      const double d2 = (double)x[u].z - (double)c_old.z, d3 = (double)x[u].w - (double)c_old.w;
      inert = fma(d0, d0, inert);
      inert = fma(d1, d1, inert);
      inert = fma(d2, d2, inert);
      inert = fma(d3, d3, inert);
    }
  }
  double tot[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double acc = ps[0][e];
#pragma unroll
    for (int u = 1; u < U; ++u) acc += ps[u][e];
    tot[e] = acc;
  }
  // lane groups hold disjoint rows: combine them (the same sum on every group)
#pragma unroll
  for (int o = LPR; o < kWave; o <<= 1)
#pragma unroll
    for (int e = 0; e < 4; ++e) tot[e] += __shfl_xor(tot[e], o);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) inert += __shfl_xor(inert, o);
  if (cnt <= (uint32_t)kUpdChunk) {
    float nrm;
    double nrm64;
    finish_slice(tot[0], tot[1], tot[2], tot[3], cnt, c_old,
                 reinterpret_cast<float4*>(protos + (int64_t)p * ld) + gl, act && h == 0, nrm,
                 nrm64);
#pragma unroll
    for (int o = LPR / 2; o >= 1; o >>= 1) {
      nrm += __shfl_xor(nrm, o);
      nrm64 += __shfl_xor(nrm64, o);
    }
    if (lane == 0) {
      pnorm[p] = nrm;
      pnorm64[p] = nrm64;
      proto_inertia[p] = inert;
    }
  } else {
    if (act && h == 0) {
      double* dst = part_sum + t * ld + 4 * gl;
      dst[0] = tot[0];
      dst[1] = tot[1];
      dst[2] = tot[2];
      dst[3] = tot[3];
    }
    if (lane == 0) part_inert[t] = inert;
  }
}

// One wave per prototype with more than one item: item sums added in item
// order, then the mean, norms and inertia as above.
template <int LPR>
__global__ __launch_bounds__(kBlock) void k_update_finish(
    int ld, const uint32_t* __restrict__ member_off, int64_t n_protos,
    float* __restrict__ protos, float* __restrict__ pnorm, double* __restrict__ pnorm64,
    double* __restrict__ proto_inertia, const double* __restrict__ part_sum,
    const double* __restrict__ part_inert) {
  const int lane = threadIdx.x % kWave;
  const int64_t p = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (p >= n_protos) return;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  const uint32_t cnt = m1 - m0;
  if (cnt <= (uint32_t)kUpdChunk) return;
  const int64_t t0 = p + m0 / kUpdChunk;
  const int nch = (int)((cnt + kUpdChunk - 1) / kUpdChunk);
  const int f4 = ld / 4;
  const int gl = lane % LPR, h = lane / LPR;
  const bool act = gl < f4 && h == 0;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  double inert = 0.0;
  for (int i = 0; i < nch; ++i) {
    if (act) {
      const double* src = part_sum + (t0 + i) * ld + 4 * gl;
      tot[0] += src[0];
      tot[1] += src[1];
      tot[2] += src[2];
      tot[3] += src[3];
    }
    inert += part_inert[t0 + i];
  }
  float4* prow = reinterpret_cast<float4*>(protos + (int64_t)p * ld) + gl;
  const float4 c_old = act ? *prow : make_float4(0.f, 0.f, 0.f, 0.f);
  float nrm;
  double nrm64;
  finish_slice(tot[0], tot[1], tot[2], tot[3], cnt, c_old, prow, act, nrm, nrm64);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    nrm += __shfl_xor(nrm, o);
    nrm64 += __shfl_xor(nrm64, o);
  }
  if (lane == 0) {
    pnorm[p] = nrm;
    pnorm64[p] = nrm64;
    proto_inertia[p] = inert;
  }
}

// One wave per group: sum of the per-prototype inertia in a fixed order.
__global__ __launch_bounds__(kBlock) void k_chunk_inertia(const double* __restrict__ proto_inertia,
                                                         int n_chunks, int k,
                                                         double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int64_t c = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (c >= n_chunks) return;
  double acc = 0.0;
  for (int j = lane; j < k; j += kWave) acc += proto_inertia[c * k + j];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) out[c] = acc;
}

// ------------------------------------------------------------- BF16 form
// Round-to-nearest-even of FP32 to BF16 bits (inputs are finite).
__device__ inline uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// out[i*ldb + c] = bf16(x[i*ld + c]) for c < ld, zero up to ldb; norms[i] =
// squared norm of the rounded row (FP32, fixed order) when norms != null.
// G lanes per row (G a power of two); each lane rounds 8 consecutive values
// per step (two float4 loads, one 16-byte store) and the group adds the
// squares of the rounded values.
template <int G>
__global__ __launch_bounds__(kBlock) void k_quantize_bf16(const float* __restrict__ x, int ld,
                                                          int64_t n, uint16_t* __restrict__ out,
                                                          int ldb, float* __restrict__ norms) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = t / G;
  const int gl = (int)(t % G);
  const bool live = i < n;  // every lane stays for the group sum
  float acc = 0.f;
  if (live) {
    for (int c = 8 * gl; c < ldb; c += 8 * G) {
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 lo = c < ld ? *reinterpret_cast<const float4*>(x + i * ld + c) : z;
      const float4 hi = c + 4 < ld ? *reinterpret_cast<const float4*>(x + i * ld + c + 4) : z;
      const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint16_t b0 = bf16_rne(v[2 * e]), b1 = bf16_rne(v[2 * e + 1]);
        w[e] = (uint32_t)b0 | ((uint32_t)b1 << 16);
        const float r0 = bf16_to_f32(b0), r1 = bf16_to_f32(b1);
        acc = fmaf(r0, r0, acc);
        acc = fmaf(r1, r1, acc);
      }
      *reinterpret_cast<uint4*>(out + i * ldb + c) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if (live && gl == 0 && norms) norms[i] = acc;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ inline bf16x8_t as_bf16x8(uint4 v) {
  bf16x8_t r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

// BF16 screening on v_mfma_f32_32x32x16_bf16 (FP32 accumulate): s_ij =
// x~_i . c~_j - |c~_j|^2 / 2 on the BF16-rounded rows, no certification.
// Layout as the FP32 kernel (prototypes = rows, points = columns); MFMA
// k-slot (s, h, e) is dimension 16s + 8h + e, so every lane feeds 8
// consecutive BF16 of a row (one 16-byte load).  The running best per lane
// is updated from the tile maximum (max3 chains), so the epilogue stays
// short next to the MFMA work at small d.
template <int DP, int PB, int TN, int MINB>
__global__ __launch_bounds__(kBlock, MINB) void k_assign_bf16(
    const uint16_t* __restrict__ items, int ldb, const uint16_t* __restrict__ protos,
    const float* __restrict__ pnorm, const int64_t* __restrict__ chunk_off, int k,
    int tiles_per_chunk, int32_t* __restrict__ labels) {
  constexpr int KS = DP / 16;
  constexpr int LDW = DP + 8;  // BF16 elements per LDS row (16-byte pad)
  constexpr int BM = 4 * 32 * PB;
  constexpr int V_PER_ROW = DP / 8;  // 16-byte vectors per row
  constexpr int LOADS = TN * V_PER_ROW / kBlock;
  static_assert(LOADS * kBlock == TN * V_PER_ROW, "tile must split evenly over the block");
  __shared__ uint4 s_c4[2][TN * LDW / 8];
  __shared__ float s_hn[2][TN];

  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = (int)(lb / (unsigned)tiles_per_chunk);
  const int tile = (int)(lb % (unsigned)tiles_per_chunk);
  const int64_t c0 = chunk_off[chunk], c1 = chunk_off[chunk + 1];
  const int64_t pbase = c0 + (int64_t)tile * BM;
  if (pbase >= c1) return;

  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int h = lane >> 5, col = lane & 31;
  bf16x8_t bf[PB][KS];
  int64_t pidx[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t p = pbase + (wave * PB + pb) * 32 + col;
    pidx[pb] = p;
    const bool ok = p < c1;
    const uint16_t* row = items + (ok ? p : c0) * (int64_t)ldb;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int c = 16 * s + 8 * h;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (ok && c < ldb) v = *reinterpret_cast<const uint4*>(row + c);
      bf[pb][s] = as_bf16x8(v);
    }
  }
  const uint16_t* cbase = protos + (int64_t)chunk * k * ldb;
  const float* nbase = pnorm + (int64_t)chunk * k;
  const int ntiles = (k + TN - 1) / TN;
  // The next tile's loads are issued before the current tile's MFMA work
  // and consumed only after it: indexes are clamped instead of branched on
  // and nothing is computed on a loaded value before the store to LDS, so no
  // wait for them sits inside the loop.  s_hn holds -|c|^2 / 2 (-inf past k).
  uint4 stage[LOADS];
  float hstage = 0.f;
  int tile_base = 0;
  auto load_tile = [&](int t) {
    tile_base = t * TN;
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int idx = threadIdx.x + i * kBlock;
      const int row = idx / V_PER_ROW, v8 = idx % V_PER_ROW;
      const int j = min(t * TN + row, k - 1);
      const bool in_row = v8 * 8 < ldb;  // rows are ldb wide, the tile DP
      const uint4 v =
          *reinterpret_cast<const uint4*>(cbase + (int64_t)j * ldb + (in_row ? v8 * 8 : 0));
      stage[i] = in_row ? v : make_uint4(0, 0, 0, 0);
    }
    if (threadIdx.x < TN) hstage = nbase[min(t * TN + (int)threadIdx.x, k - 1)];
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int idx = threadIdx.x + i * kBlock;
      const int row = idx / V_PER_ROW, v8 = idx % V_PER_ROW;
      s_c4[buf][(row * LDW) / 8 + v8] = stage[i];
    }
    if (threadIdx.x < TN)
      // past k: the most negative finite value (the index bits below must
      // not turn the score into a NaN)
      s_hn[buf][threadIdx.x] = (tile_base + (int)threadIdx.x < k) ? -0.5f * hstage : -FLT_MAX;
  };
  load_tile(0);
  store_tile(0);
  __syncthreads();

  // Running best per lane: the score with the accumulator register's index
  // in its 4 low mantissa bits (a change of at most 2^-19 relative), and the
  // first prototype of the 32-row block it came from.
  float b1[PB];
  int blk[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) { b1[pb] = -INFINITY; blk[pb] = 0; }

  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    if (t + 1 < ntiles) load_tile(t + 1);
#pragma unroll
    for (int cb = 0; cb < TN / 32; ++cb) {
      floatx16 acc[PB];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float hv = s_hn[buf][cb * 32 + 8 * (i >> 2) + 4 * h + (i & 3)];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) acc[pb][i] = hv;
      }
      const uint4* arow = &s_c4[buf][((cb * 32 + col) * LDW + 8 * h) / 8];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const bf16x8_t a = as_bf16x8(arow[2 * s]);  // dims 16s + 8h .. +7
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
          acc[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bf[pb][s], acc[pb], 0, 0, 0);
      }
      const int jbase = t * TN + cb * 32;
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          acc[pb][i] = __uint_as_float((__float_as_uint(acc[pb][i]) & ~15u) | (uint32_t)i);
        float m = fmaxf(fmaxf(acc[pb][0], acc[pb][1]), acc[pb][2]);
#pragma unroll
        for (int i = 3; i < 15; i += 2) m = fmaxf(fmaxf(m, acc[pb][i]), acc[pb][i + 1]);
        m = fmaxf(m, acc[pb][15]);
        const bool better = m > b1[pb];
        b1[pb] = better ? m : b1[pb];
        blk[pb] = better ? jbase : blk[pb];
      }
    }
    if (t + 1 < ntiles) store_tile(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const uint32_t ii = __float_as_uint(b1[pb]) & 15u;
    int i1 = blk[pb] + 8 * (int)(ii >> 2) + 4 * h + (int)(ii & 3u);
    const float o = __shfl_xor(b1[pb], 32);
    const int oi = __shfl_xor(i1, 32);
    if (o > b1[pb] || (o == b1[pb] && oi < i1)) { b1[pb] = o; i1 = oi; }
    if (h == 0 && pidx[pb] < c1) labels[pidx[pb]] = chunk * k + i1;
  }
}

// Direct-form assignment on the vector units, for metrics without an MFMA
// form (L1) and for wide rows: one wave per 64 items of one group, item rows
// staged in LDS with an odd row stride (conflict-free per-lane reads), every
// lane walks all k prototypes of the group with wave-uniform loads.  The
// per-element difference is exact in FP64 and accumulated in FP64, so the
// labels agree with an FP64 evaluation except for gaps of about 1e-15.
template <int METRIC>
__global__ __launch_bounds__(kWave) void k_assign_direct(
    const float* __restrict__ items, int ld, const float* __restrict__ protos,
    const int64_t* __restrict__ chunk_off, int k, int tiles_per_chunk,
    int32_t* __restrict__ labels) {
  extern __shared__ float s_xr[];  // 64 rows x (ld + 1)
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x / tiles_per_chunk, tile = blockIdx.x % tiles_per_chunk;
  const int64_t c0 = chunk_off[chunk], c1 = chunk_off[chunk + 1];
  const int64_t pbase = c0 + (int64_t)tile * 64;
  if (pbase >= c1) return;
  const int np = (int)min<int64_t>(64, c1 - pbase);
  const int xs = ld + 1;
  for (int i = lane; i < np * ld; i += kWave) {
    const int row = i / ld, c = i % ld;
    s_xr[row * xs + c] = items[(pbase + row) * ld + c];
  }
  __syncthreads();
  const float* xr = s_xr + (lane < np ? lane : 0) * xs;
  const float* cbase = protos + (int64_t)chunk * k * ld;
  double best = INFINITY;
  int bj = 0;
  for (int j = 0; j < k; ++j) {
    const float4* crow = reinterpret_cast<const float4*>(cbase + (int64_t)j * ld);
    double a0 = 0.0, a1 = 0.0;
    for (int i = 0; i < ld / 4; ++i) {
      const float4 cv = crow[i];
      const double d0 = (double)xr[4 * i] - (double)cv.x, d1 = (double)xr[4 * i + 1] - (double)cv.y,
                   d2 = (double)xr[4 * i + 2] - (double)cv.z, d3 = (double)xr[4 * i + 3] - (double)cv.w;
      if (METRIC == 0) {
        a0 = fma(d0, d0, a0); a1 = fma(d1, d1, a1); a0 = fma(d2, d2, a0); a1 = fma(d3, d3, a1);
      } else {
        a0 += fabs(d0); a1 += fabs(d1); a0 += fabs(d2); a1 += fabs(d3);
      }
    }
    const double dd = a0 + a1;
    if (dd < best) { best = dd; bj = j; }  // ascending j: ties keep the lower
  }
  if (lane < np) labels[pbase + lane] = chunk * k + bj;
}

// Order-preserving map of float bits to unsigned keys.
__device__ inline uint32_t float_key(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// k-medians update (L1): one wave per prototype, lanes over dimensions; each
// new coordinate is the lower median (order statistic floor((m-1)/2)) of the
// members' values, found by a most-significant-bit-first radix select over
// the order-preserving keys (32 passes over the member list); an empty
// prototype keeps its value.  Also the FP64 L1 inertia under the old
// prototype.
template <int J>
__global__ __launch_bounds__(kBlock) void k_update_l1(
    const float* __restrict__ items, int ld, const uint32_t* __restrict__ members,
    const uint32_t* __restrict__ member_off, int64_t n_protos, float* __restrict__ protos,
    double* __restrict__ proto_inertia) {
  const int lane = threadIdx.x % kWave;
  const int64_t p = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (p >= n_protos) return;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  const uint32_t cnt = m1 - m0;
  float c_old[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = lane + j * kWave;
    c_old[j] = (c < ld) ? protos[p * ld + c] : 0.f;
  }
  double inert = 0.0;
  for (uint32_t m = m0; m < m1; ++m) {
    const float* row = items + (int64_t)members[m] * ld;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int c = lane + j * kWave;
      if (c < ld) inert += fabs((double)row[c] - (double)c_old[j]);
    }
  }
  if (cnt > 0) {
    const uint32_t t = (cnt - 1) / 2;
    uint32_t prefix[J], rank[J];
#pragma unroll
    for (int j = 0; j < J; ++j) { prefix[j] = 0; rank[j] = t; }
    for (int b = 31; b >= 0; --b) {
      const uint32_t hi_mask = (b == 31) ? 0u : (0xffffffffu << (b + 1));
      uint32_t zeros[J];
#pragma unroll
      for (int j = 0; j < J; ++j) zeros[j] = 0;
      for (uint32_t m = m0; m < m1; ++m) {
        const float* row = items + (int64_t)members[m] * ld;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const int c = lane + j * kWave;
          if (c < ld) {
            const uint32_t key = float_key(row[c]);
            zeros[j] += ((key & hi_mask) == prefix[j]) && !((key >> b) & 1u);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (rank[j] >= zeros[j]) {  // the wanted value has bit b set
          rank[j] -= zeros[j];
          prefix[j] |= 1u << b;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int c = lane + j * kWave;
      if (c < ld) protos[p * ld + c] = key_float(prefix[j]);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) inert += __shfl_xor(inert, o);
  if (lane == 0) proto_inertia[p] = inert;
}

__global__ void k_row_norms64(const float* __restrict__ x, int ld, int64_t n,
                              double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* r = x + i * ld;
  double acc = 0.0;
  for (int c = 0; c < ld; ++c) acc = fma((double)r[c], (double)r[c], acc);
  out[i] = acc;
}

__global__ void k_init_first(const float* __restrict__ items, int ld,
                             const int64_t* __restrict__ chunk_off, int n_chunks, int k,
                             float* __restrict__ protos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_chunks * k * ld;
  if (t >= total) return;
  const int64_t row = t / ld;
  const int c = (int)(t % ld);
  const int chunk = (int)(row / k), j = (int)(row % k);
  // a group smaller than k starts from its members taken cyclically
  const int64_t m = chunk_off[chunk + 1] - chunk_off[chunk];
  protos[t] = items[(chunk_off[chunk] + j % m) * ld + c];
}

__global__ void k_labels_to_keys(const int32_t* __restrict__ labels, int64_t n,
                                 uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = (uint32_t)labels[i];
  vals[i] = (uint32_t)i;
}

int bits_for(int64_t n) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  return b;
}

template <int DP, int PB, int TN, int MINB = 2>
void launch_assign(const float* items, int ld, int dim, const ChunkPlan& plan,
                   const float* protos, int32_t* labels, KmeansWork& w, hipStream_t s) {
  constexpr int BM = 4 * 32 * PB;
  const int tiles = (int)((plan.max_chunk + BM - 1) / BM);
  const unsigned grid = (unsigned)(tiles * plan.n_chunks);
  const float err_coef = (float)(dim + 4) * 5.9604644775390625e-08f;  // (d+4) * 2^-24
  ScopedTiming timing("assign_l2_mfma", s);
  k_assign_l2_mfma<DP, PB, TN, MINB><<<grid, kBlock, 0, s>>>(
      items, ld, protos, w.proto_norms, w.item_norms, plan.d_off, plan.k, tiles, labels,
      w.refine_count, w.small_list, w.small_cand, w.full_cnt, w.full_list, err_coef);
  check_launch("assign_l2_mfma");
}

template <int METRIC>
void launch_full(const float* items, int ld, const ChunkPlan& plan, const float* protos,
                 KmeansWork& w, hipStream_t s) {
  const dim3 grid(w.full_grid, w.full_splits);
  const size_t shm = (size_t)64 * (ld + 4) * sizeof(float);
  k_refine_full<METRIC><<<grid, kWave, shm, s>>>(
      items, ld, protos, plan.d_off, plan.k, w.full_cnt, w.full_list, w.tiles, w.tile_total,
      w.full_splits, w.partial_d, w.partial_j);
}

template <int DP>
void launch_full_f64(const float* items, int ld, const ChunkPlan& plan, const float* protos,
                     KmeansWork& w, hipStream_t s) {
  const dim3 grid(w.full_grid, w.full_splits);
  k_refine_f64<DP><<<grid, kBlock, 0, s>>>(items, ld, protos, w.proto_norms64, plan.d_off,
                                           plan.k, w.full_cnt, w.full_list, w.tiles,
                                           w.tile_total, w.full_splits, w.partial_d,
                                           w.partial_j);
}

template <int DP, int PB, int TN, int MINB>
void launch_assign_bf16(const ChunkPlan& plan, int32_t* labels, KmeansWork& w, hipStream_t s) {
  constexpr int BM = 4 * 32 * PB;
  const int tiles = (int)((plan.max_chunk + BM - 1) / BM);
  ScopedTiming timing("assign_bf16_mfma", s);
  k_assign_bf16<DP, PB, TN, MINB><<<(unsigned)(tiles * plan.n_chunks), kBlock, 0, s>>>(
      w.items_b, w.ldb, w.protos_b, w.proto_norms_b, plan.d_off, plan.k, tiles, labels);
  check_launch("assign_bf16_mfma");
}

void launch_refine(const float* items, int ld, const ChunkPlan& plan, const float* protos,
                   int32_t* labels, KmeansWork& w, int metric, hipStream_t s) {
  unsigned long long* stats = timing_refine_counter();
  ScopedTiming timing("refine", s);
  if (metric == MASK_L2)
    k_refine_small<0><<<1024, kBlock, 0, s>>>(items, ld, protos, plan.d_off, plan.n_chunks,
                                              plan.k, w.refine_count, w.small_list, w.small_cand,
                                              labels, stats);
  else
    k_refine_small<1><<<1024, kBlock, 0, s>>>(items, ld, protos, plan.d_off, plan.n_chunks,
                                              plan.k, w.refine_count, w.small_list, w.small_cand,
                                              labels, stats);
  check_launch("refine_small");
  k_full_tiles<<<1, kBlock, 0, s>>>(w.full_cnt, plan.n_chunks, w.tiles, w.tile_total);
  check_launch("full_tiles");
  if (metric == MASK_L2) {
    const int dp = (ld + 15) & ~15;
    if (dp <= 16) launch_full_f64<16>(items, ld, plan, protos, w, s);
    else if (dp <= 32) launch_full_f64<32>(items, ld, plan, protos, w, s);
    else if (dp <= 64) launch_full_f64<64>(items, ld, plan, protos, w, s);
    else if (dp <= 96) launch_full_f64<96>(items, ld, plan, protos, w, s);
    else if (dp <= 128) launch_full_f64<128>(items, ld, plan, protos, w, s);
    else launch_full<0>(items, ld, plan, protos, w, s);
  } else {
    launch_full<1>(items, ld, plan, protos, w, s);
  }
  check_launch("refine_full");
  k_refine_merge<<<256, kBlock, 0, s>>>(plan.d_off, plan.k, w.full_cnt, w.full_list, w.tiles,
                                        w.tile_total, w.full_splits, w.partial_d, w.partial_j,
                                        labels, stats);
  check_launch("refine_merge");
}

}  // namespace

void kmeans_alloc(KmeansWork& w, int64_t n_items, int n_chunks, int k, int ld, Arena& a) {
  const int64_t n_protos = (int64_t)n_chunks * k;
  w.sort_keys = a.alloc<uint32_t>(n_items);
  w.sort_vals = a.alloc<uint32_t>(n_items);
  sort_work_alloc(w.sort, n_items, false, a);
  w.member_off = a.alloc<uint32_t>(n_protos + 1);
  w.proto_inertia = a.alloc<double>(n_protos);
  w.refine_count = a.alloc<uint32_t>(4);
  w.small_list = a.alloc<uint32_t>(n_items);
  w.small_cand = a.alloc<int32_t>(3 * n_items);
  w.full_cnt = a.alloc<uint32_t>(n_chunks);
  w.full_list = a.alloc<uint32_t>(n_items);
  const int64_t max_tiles = n_items / 64 + n_chunks + 1;
  w.tiles = a.alloc<uint2>(max_tiles);
  w.tile_total = a.alloc<uint32_t>(4);
  // prototype ranges of about 128 per wave, at most 64 ranges
  w.full_splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, (k + 127) / 128));
  w.full_grid = (int)std::min<int64_t>(max_tiles, 1024);
  w.partial_d = a.alloc<double>(n_items * w.full_splits);
  w.partial_j = a.alloc<int32_t>(n_items * w.full_splits);
  w.item_norms = a.alloc<float>(n_items);
  w.proto_norms = a.alloc<float>(n_protos);
  w.proto_norms64 = a.alloc<double>(n_protos);
  // update work items (see k_update_slots)
  const int64_t n_slots = n_protos + n_items / kUpdChunk;
  w.slot_proto = a.alloc<int32_t>(n_slots);
  w.upd_sum = a.alloc<double>(n_slots * ld);
  w.upd_inert = a.alloc<double>(n_slots);
}

void kmeans_proto_norms(const float* protos, int ld, int64_t n_protos, KmeansWork& w,
                        hipStream_t s) {
  row_norms(protos, ld, n_protos, w.proto_norms, s);
  k_row_norms64<<<grid_for(n_protos, kBlock), kBlock, 0, s>>>(protos, ld, n_protos,
                                                            w.proto_norms64);
  check_launch("row_norms64");
}

void kmeans_init_first(const float* items, int ld, const ChunkPlan& plan, float* protos,
                       hipStream_t s) {
  const int64_t total = (int64_t)plan.n_chunks * plan.k * ld;
  k_init_first<<<grid_for(total, kBlock), kBlock, 0, s>>>(items, ld, plan.d_off, plan.n_chunks,
                                                        plan.k, protos);
  check_launch("init_first");
}

void quantize_bf16(const float* x, int ld, int64_t n, uint16_t* out, int ldb, float* norms,
                   hipStream_t s) {
  if (n <= 0) return;
  const int c8 = ldb / 8;
  if (c8 <= 4)
    k_quantize_bf16<4><<<grid_for(n * 4, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldb, norms);
  else if (c8 <= 8)
    k_quantize_bf16<8><<<grid_for(n * 8, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldb, norms);
  else if (c8 <= 16)
    k_quantize_bf16<16><<<grid_for(n * 16, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldb, norms);
  else
    k_quantize_bf16<32><<<grid_for(n * 32, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldb, norms);
  check_launch("quantize_bf16");
}

void kmeans_assign(const float* items, int ld, int dim, const ChunkPlan& plan,
                   const float* protos, int32_t* labels, KmeansWork& w, int metric,
                   hipStream_t s) {
  if (w.precision == MASK_BF16 && metric == MASK_L2) {
    // re-quantise the current prototypes, then screen in BF16
    quantize_bf16(protos, ld, (int64_t)plan.n_chunks * plan.k, w.protos_b, w.ldb,
                  w.proto_norms_b, s);
    const int dp = (w.ldb + 15) & ~15;
    if (dp <= 16) launch_assign_bf16<16, 4, 128, 2>(plan, labels, w, s);
    else if (dp <= 32) launch_assign_bf16<32, 4, 64, 2>(plan, labels, w, s);
    else if (dp <= 64) launch_assign_bf16<64, 2, 64, 2>(plan, labels, w, s);
    else if (dp <= 96) {
      // Many rows: 512 per workgroup and tiles of 128 prototypes (fewer LDS
      // reads and barriers per MFMA; about 4% faster on 10 groups of 1M rows
      // x 10,000 prototypes, MI355X).  Few rows: smaller workgroups, so that
      // the grid still covers the chip.
      const int64_t rows = plan.max_chunk * plan.n_chunks;
      if (rows >= ((int64_t)1 << 19)) launch_assign_bf16<96, 4, 128, 2>(plan, labels, w, s);
      else if (rows >= ((int64_t)1 << 16)) launch_assign_bf16<96, 2, 64, 2>(plan, labels, w, s);
      else launch_assign_bf16<96, 1, 64, 2>(plan, labels, w, s);
    }
    else if (dp <= 128) launch_assign_bf16<128, 2, 64, 2>(plan, labels, w, s);
    else if (dp <= 256) launch_assign_bf16<256, 1, 64, 2>(plan, labels, w, s);
    else throw Error{MASK_ERR_UNSUPPORTED, "BF16 dimension above 256"};
    return;
  }
  if (metric == MASK_L1 || dim > kMaxDenseDim) {
    const int tiles = (int)((plan.max_chunk + 63) / 64);
    const size_t shm = (size_t)64 * (ld + 1) * sizeof(float);
    ScopedTiming timing("assign_direct", s);
    if (metric == MASK_L1)
      k_assign_direct<1><<<(unsigned)(tiles * plan.n_chunks), kWave, shm, s>>>(
          items, ld, protos, plan.d_off, plan.k, tiles, labels);
    else
      k_assign_direct<0><<<(unsigned)(tiles * plan.n_chunks), kWave, shm, s>>>(
          items, ld, protos, plan.d_off, plan.k, tiles, labels);
    check_launch("assign_direct");
    return;
  }
  fill_u32(w.refine_count, 2, 0u, s);
  fill_u32(w.full_cnt, plan.n_chunks, 0u, s);
  const int dp = (dim + 7) & ~7;
  if (dp <= 16) launch_assign<16, 2, 64>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 32) launch_assign<32, 2, 64>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 64) launch_assign<64, 2, 64>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 96) launch_assign<96, 2, 32>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 128) launch_assign<128, 1, 32, 3>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 192) launch_assign<192, 1, 32>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 256) launch_assign<256, 1, 32>(items, ld, dim, plan, protos, labels, w, s);
  else throw Error{MASK_ERR_UNSUPPORTED, "dense dimension above 256"};
  launch_refine(items, ld, plan, protos, labels, w, metric, s);
}

void kmeans_update(const float* items, int ld, int dim, const ChunkPlan& plan,
                   const int32_t* labels, float* protos, KmeansWork& w, int metric,
                   double* inertia_out, hipStream_t s) {
  (void)dim;
  const int64_t n = plan.n_items;
  const int64_t np = (int64_t)plan.n_chunks * plan.k;
  {
    ScopedTiming timing("member_sort", s);
    k_labels_to_keys<<<grid_for(n, kBlock), kBlock, 0, s>>>(labels, n, w.sort_keys, w.sort_vals);
    check_launch("labels_to_keys");
    radix_sort_u32(w.sort_keys, w.sort_vals, n, bits_for(np), w.sort, s);
    offsets_from_sorted(w.sort_keys, n, np, w.member_off, s);
  }
  const int J = (ld + kWave - 1) / kWave;
  const unsigned grid = grid_for(np * kWave, kBlock);
  if (metric == MASK_L1) {
    ScopedTiming timing("update_l1", s);
    if (J <= 1)
      k_update_l1<1><<<grid, kBlock, 0, s>>>(items, ld, w.sort_vals, w.member_off, np, protos,
                                             w.proto_inertia);
    else if (J <= 2)
      k_update_l1<2><<<grid, kBlock, 0, s>>>(items, ld, w.sort_vals, w.member_off, np, protos,
                                             w.proto_inertia);
    else if (J <= 4)
      k_update_l1<4><<<grid, kBlock, 0, s>>>(items, ld, w.sort_vals, w.member_off, np, protos,
                                             w.proto_inertia);
    else
      throw Error{MASK_ERR_UNSUPPORTED, "L1 update of rows wider than 256"};
    check_launch("update_l1");
  } else {
  ScopedTiming timing("update_l2", s);
  const int64_t n_slots = np + n / kUpdChunk;
  k_update_slots<<<grid_for(np, kBlock), kBlock, 0, s>>>(w.member_off, np, w.slot_proto);
  check_launch("update_slots");
  const unsigned gi = grid_for(n_slots * kWave, kBlock);
  const unsigned gf = grid_for(np * kWave, kBlock);
  const int f4 = ld / 4;
#define MASK_UPDATE(LPR, U)                                                                   \
  do {                                                                                        \
    k_update_items<LPR, U><<<gi, kBlock, 0, s>>>(items, ld, w.sort_vals, w.member_off,         \
                                                 w.slot_proto, n_slots, protos, w.proto_norms, \
                                                 w.proto_norms64, w.proto_inertia, w.upd_sum,  \
                                                 w.upd_inert);                                 \
    k_update_finish<LPR><<<gf, kBlock, 0, s>>>(ld, w.member_off, np, protos, w.proto_norms,    \
                                               w.proto_norms64, w.proto_inertia, w.upd_sum,    \
                                               w.upd_inert);                                   \
  } while (0)
  if (f4 <= 4) MASK_UPDATE(4, 4);
  else if (f4 <= 8) MASK_UPDATE(8, 4);
  else if (f4 <= 16) MASK_UPDATE(16, 4);
  else if (f4 <= 32) MASK_UPDATE(32, 4);
  else MASK_UPDATE(64, 8);
#undef MASK_UPDATE
  check_launch("update_l2");
  }
  if (inertia_out) {
    k_chunk_inertia<<<grid_for((int64_t)plan.n_chunks * kWave, kBlock), kBlock, 0, s>>>(
        w.proto_inertia, plan.n_chunks, plan.k, inertia_out);
    check_launch("chunk_inertia");
  }
}

}  // namespace mask

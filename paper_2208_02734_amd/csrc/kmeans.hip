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
#include "internal.hpp"

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
    uint32_t* __restrict__ full_list, float err_coef) {
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
            const uint32_t slot = atomicAdd(&refine_count[1], 1u);
            full_list[slot] = (uint32_t)p;
          }
        }
      }
    }
  }
}

// Direct-form distance in a fixed order: four partial sums over the float4
// lanes of the row, combined as (p0+p1)+(p2+p3).  ld is a multiple of 4 and
// the padding is zero in both rows.
template <int METRIC>
__device__ inline float direct_dist(const float* __restrict__ x, const float* __restrict__ c,
                                    int ld) {
  const float4* x4 = reinterpret_cast<const float4*>(x);
  const float4* c4 = reinterpret_cast<const float4*>(c);
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
  for (int i = 0; i < ld / 4; ++i) {
    const float4 a = x4[i], b = c4[i];
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
    if (METRIC == 0) {
      p0 = fmaf(dx, dx, p0); p1 = fmaf(dy, dy, p1); p2 = fmaf(dz, dz, p2); p3 = fmaf(dw, dw, p3);
    } else {
      p0 += fabsf(dx); p1 += fabsf(dy); p2 += fabsf(dz); p3 += fabsf(dw);
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
    float dist = INFINITY;
    int cand = 0x7fffffff;
    int64_t p = 0;
    int chunk = 0;
    if (valid) {
      p = small_list[e];
      chunk = find_chunk(chunk_off, n_chunks, p);
      const int c = slot < 3 ? small_cand[3 * e + slot] : -1;
      if (c >= 0) {
        cand = c;
        dist = direct_dist<METRIC>(items + p * ld, protos + ((int64_t)chunk * k + c) * ld, ld);
      }
    }
#pragma unroll
    for (int o = 1; o <= 2; o <<= 1) {
      const float od = __shfl_xor(dist, o);
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

// Points whose uncertainty window holds four or more prototypes: one wave
// per point, lanes over every prototype of its group.
template <int METRIC>
__global__ __launch_bounds__(kBlock) void k_refine_full(
    const float* __restrict__ items, int ld, const float* __restrict__ protos,
    const int64_t* __restrict__ chunk_off, int n_chunks, int k,
    const uint32_t* __restrict__ refine_count, const uint32_t* __restrict__ full_list,
    int32_t* __restrict__ labels, unsigned long long* __restrict__ stats) {
  const int lane = threadIdx.x % kWave;
  const int64_t wave0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t n_waves = (int64_t)gridDim.x * (kBlock / kWave);
  const uint32_t count = refine_count[1];
  for (int64_t e = wave0; e < (int64_t)count; e += n_waves) {
    const int64_t p = full_list[e];
    const int chunk = find_chunk(chunk_off, n_chunks, p);
    const float* x = items + p * ld;
    const float* cbase = protos + (int64_t)chunk * k * ld;
    float best = INFINITY;
    int bi = 0x7fffffff;
    for (int j = lane; j < k; j += kWave) {
      const float dj = direct_dist<METRIC>(x, cbase + (int64_t)j * ld, ld);
      if (dj < best) { best = dj; bi = j; }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float od = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (od < best || (od == best && oi < bi)) { best = od; bi = oi; }
    }
    if (lane == 0) {
      labels[p] = chunk * k + bi;
      if (stats) atomicAdd(&stats[1], 1ull);
    }
  }
}

// One wave per prototype: FP64 sums of the members in item order, the new
// prototype (unchanged when empty), its FP32 squared norm, and the FP64
// inertia of the members under the old prototype.
template <int J>
__global__ __launch_bounds__(kBlock) void k_update_l2(
    const float* __restrict__ items, int ld, const uint32_t* __restrict__ members,
    const uint32_t* __restrict__ member_off, int64_t n_protos, float* __restrict__ protos,
    float* __restrict__ pnorm, double* __restrict__ proto_inertia) {
  const int lane = threadIdx.x % kWave;
  const int64_t p = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (p >= n_protos) return;
  float c_old[J];
  double sum[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = lane + j * kWave;
    c_old[j] = (c < ld) ? protos[p * ld + c] : 0.f;
    sum[j] = 0.0;
  }
  double inert = 0.0;
  const uint32_t m0 = member_off[p], m1 = member_off[p + 1];
  for (uint32_t m = m0; m < m1; ++m) {
    const float* row = items + (int64_t)members[m] * ld;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int c = lane + j * kWave;
      if (c < ld) {
        const float x = row[c];
        sum[j] += (double)x;
        const double d = (double)x - (double)c_old[j];
        inert = fma(d, d, inert);
      }
    }
  }
  const uint32_t cnt = m1 - m0;
  float nrm = 0.f;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = lane + j * kWave;
    float v = c_old[j];
    if (cnt > 0) v = (float)(sum[j] / (double)cnt);
    if (c < ld) {
      protos[p * ld + c] = v;
      nrm = fmaf(v, v, nrm);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    nrm += __shfl_xor(nrm, o);
    inert += __shfl_xor(inert, o);
  }
  if (lane == 0) {
    pnorm[p] = nrm;
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

__global__ void k_init_first(const float* __restrict__ items, int ld,
                             const int64_t* __restrict__ chunk_off, int n_chunks, int k,
                             float* __restrict__ protos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_chunks * k * ld;
  if (t >= total) return;
  const int64_t row = t / ld;
  const int c = (int)(t % ld);
  const int chunk = (int)(row / k), j = (int)(row % k);
  protos[t] = items[(chunk_off[chunk] + j) * ld + c];
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
      w.refine_count, w.small_list, w.small_cand, w.full_list, err_coef);
  check_launch("assign_l2_mfma");
}

void launch_refine(const float* items, int ld, const ChunkPlan& plan, const float* protos,
                   int32_t* labels, KmeansWork& w, int metric, hipStream_t s) {
  unsigned long long* stats = timing_refine_counter();
  ScopedTiming timing("refine", s);
  if (metric == MASK_L2) {
    k_refine_small<0><<<1024, kBlock, 0, s>>>(items, ld, protos, plan.d_off, plan.n_chunks,
                                              plan.k, w.refine_count, w.small_list, w.small_cand,
                                              labels, stats);
    k_refine_full<0><<<512, kBlock, 0, s>>>(items, ld, protos, plan.d_off, plan.n_chunks, plan.k,
                                            w.refine_count, w.full_list, labels, stats);
  } else {
    k_refine_small<1><<<1024, kBlock, 0, s>>>(items, ld, protos, plan.d_off, plan.n_chunks,
                                              plan.k, w.refine_count, w.small_list, w.small_cand,
                                              labels, stats);
    k_refine_full<1><<<512, kBlock, 0, s>>>(items, ld, protos, plan.d_off, plan.n_chunks, plan.k,
                                            w.refine_count, w.full_list, labels, stats);
  }
  check_launch("refine");
}

}  // namespace

void kmeans_alloc(KmeansWork& w, int64_t n_items, int64_t n_protos, Arena& a) {
  w.sort_keys = a.alloc<uint32_t>(n_items);
  w.sort_vals = a.alloc<uint32_t>(n_items);
  sort_work_alloc(w.sort, n_items, false, a);
  w.member_off = a.alloc<uint32_t>(n_protos + 1);
  w.proto_inertia = a.alloc<double>(n_protos);
  w.refine_count = a.alloc<uint32_t>(4);
  w.small_list = a.alloc<uint32_t>(n_items);
  w.small_cand = a.alloc<int32_t>(3 * n_items);
  w.full_list = a.alloc<uint32_t>(n_items);
  w.item_norms = a.alloc<float>(n_items);
  w.proto_norms = a.alloc<float>(n_protos);
}

void kmeans_init_first(const float* items, int ld, const ChunkPlan& plan, float* protos,
                       hipStream_t s) {
  const int64_t total = (int64_t)plan.n_chunks * plan.k * ld;
  k_init_first<<<grid_for(total, kBlock), kBlock, 0, s>>>(items, ld, plan.d_off, plan.n_chunks,
                                                        plan.k, protos);
  check_launch("init_first");
}

void kmeans_assign(const float* items, int ld, int dim, const ChunkPlan& plan,
                   const float* protos, int32_t* labels, KmeansWork& w, int metric,
                   hipStream_t s) {
  if (metric != MASK_L2) throw Error{MASK_ERR_UNSUPPORTED, "assignment metric"};
  fill_u32(w.refine_count, 2, 0u, s);
  const int dp = (dim + 7) & ~7;
  if (dp <= 16) launch_assign<16, 2, 64>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 32) launch_assign<32, 2, 64>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 64) launch_assign<64, 2, 64>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 96) launch_assign<96, 2, 32>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 128) launch_assign<128, 2, 64, 1>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 192) launch_assign<192, 1, 32>(items, ld, dim, plan, protos, labels, w, s);
  else if (dp <= 256) launch_assign<256, 1, 32>(items, ld, dim, plan, protos, labels, w, s);
  else throw Error{MASK_ERR_UNSUPPORTED, "dense dimension above 256"};
  launch_refine(items, ld, plan, protos, labels, w, metric, s);
}

void kmeans_update(const float* items, int ld, int dim, const ChunkPlan& plan,
                   const int32_t* labels, float* protos, KmeansWork& w, int metric,
                   double* inertia_out, hipStream_t s) {
  (void)dim;
  if (metric != MASK_L2) throw Error{MASK_ERR_UNSUPPORTED, "update metric"};
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
  ScopedTiming timing("update_l2", s);
  if (J <= 1)
    k_update_l2<1><<<grid, kBlock, 0, s>>>(items, ld, w.sort_vals, w.member_off, np, protos,
                                           w.proto_norms, w.proto_inertia);
  else if (J <= 2)
    k_update_l2<2><<<grid, kBlock, 0, s>>>(items, ld, w.sort_vals, w.member_off, np, protos,
                                           w.proto_norms, w.proto_inertia);
  else
    k_update_l2<4><<<grid, kBlock, 0, s>>>(items, ld, w.sort_vals, w.member_off, np, protos,
                                           w.proto_norms, w.proto_inertia);
  check_launch("update_l2");
  if (inertia_out) {
    k_chunk_inertia<<<grid_for((int64_t)plan.n_chunks * kWave, kBlock), kBlock, 0, s>>>(
        w.proto_inertia, plan.n_chunks, plan.k, inertia_out);
    check_launch("chunk_inertia");
  }
}

}  // namespace mask

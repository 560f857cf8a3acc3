// FP8 variant of the precision form: rows stored as OCP e4m3 (largest
// finite value 448, the format gfx950's conversions and MFMA use) with one
// FP32 scale per row, s = max|x| / 448 (1 for a zero row), so that a row is
// x ~ s * q.  The assignment screens with v_mfma_f32_32x32x16_fp8_fp8 (FP32
// accumulate) on the quantised rows, score_ij = s_i s_j (q_i . q_j) -
// |c^_j|^2 / 2 with c^_j = s_j q_j, no certification; sums stay FP64 on
// the FP32 rows (the update is the plain form's).
#include <cmath>
#include <type_traits>

#include "internal.hpp"

namespace mask {
namespace {

constexpr int kBlock = 256;
typedef float floatx16 __attribute__((ext_vector_type(16)));

inline unsigned grid_for(int64_t work, int per_block) {
  return (unsigned)((work + per_block - 1) / per_block);
}

__device__ inline unsigned xcd_remap8(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, i = b >> 3;
  const unsigned q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + i;
}

__device__ inline uint32_t fp8x4(float a, float b, float c, float d) {
  // clamped to the finite range: values past 448 would convert to NaN
  a = fminf(fmaxf(a, -448.f), 448.f);
  b = fminf(fmaxf(b, -448.f), 448.f);
  c = fminf(fmaxf(c, -448.f), 448.f);
  d = fminf(fmaxf(d, -448.f), 448.f);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}

__device__ inline float fp8_sq4(uint32_t w, float s) {
  const float v0 = s * __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
  const float v1 = s * __builtin_amdgcn_cvt_f32_fp8((int)w, 1);
  const float v2 = s * __builtin_amdgcn_cvt_f32_fp8((int)w, 2);
  const float v3 = s * __builtin_amdgcn_cvt_f32_fp8((int)w, 3);
  return fmaf(v0, v0, fmaf(v1, v1, fmaf(v2, v2, v3 * v3)));
}

// G lanes per row; a lane handles 16 consecutive values per step (four
// float4 loads, one 16-byte store).  Pass 1: max |x| over the group; pass 2:
// quantise and add the squares of the dequantised values.
template <int G>
__global__ __launch_bounds__(kBlock) void k_quantize_fp8(const float* __restrict__ x, int ld,
                                                         int64_t n, uint8_t* __restrict__ out,
                                                         int ldq, float* __restrict__ scale,
                                                         float* __restrict__ norms) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = t / G;
  const int gl = (int)(t % G);
  const bool live = i < n;
  float mx = 0.f;
  if (live) {
    for (int c = 4 * gl; c < ld; c += 4 * G) {
      const float4 v = *reinterpret_cast<const float4*>(x + i * ld + c);
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  const float s = mx > 0.f ? mx / 448.f : 1.f;
  const float inv = mx > 0.f ? 448.f / mx : 1.f;
  float acc = 0.f;
  if (live) {
    for (int c = 16 * gl; c < ldq; c += 16 * G) {
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int cc = c + 4 * e;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (cc < ld) v = *reinterpret_cast<const float4*>(x + i * ld + cc);
        w[e] = fp8x4(v.x * inv, v.y * inv, v.z * inv, v.w * inv);
        acc += fp8_sq4(w[e], s);
      }
      *reinterpret_cast<uint4*>(out + i * ldq + c) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if (live && gl == 0) {
    scale[i] = s;
    if (norms) norms[i] = acc;
  }
}

typedef int v8i32 __attribute__((ext_vector_type(8)));

// FP8 screening, same tiling as the BF16 kernel: prototypes are MFMA rows
// (staged through LDS, TN per tile), points are columns (PB x 32 per wave,
// held in registers).  The accumulators start at 0; the epilogue forms
// s_i s_j acc - |c^_j|^2/2 and keeps the running best.
// Rows of 64 bytes or more use the K = 64 shape
// (v_mfma_scale_f32_32x32x64_f8f6f4, both scales 2^0, twice the FP8 rate of
// the K = 16 shape): in step s a lane feeds the 32 bytes 64s + 32h .. of its
// row (h = lane / 32), zero past the row's end.  A and B take their K values
// from the same lane and register positions, so the product runs over every
// byte of both rows exactly once.  Shorter rows use
// v_mfma_f32_32x32x16_fp8_fp8, k-slot (s, h, e) = dimension 16s + 8h + e.
template <int DP, int PB, int TN, int MINB>
__global__ __launch_bounds__(kBlock, MINB) void k_assign_fp8(
    const uint8_t* __restrict__ items, const float* __restrict__ iscale, int ldq,
    const uint8_t* __restrict__ protos, const float* __restrict__ pscale,
    const float* __restrict__ pnorm, const int64_t* __restrict__ chunk_off, int k,
    int tiles_per_chunk, int32_t* __restrict__ labels) {
  constexpr bool K64 = DP >= 64;
  constexpr int KB = K64 ? 64 : 16;           // K of one MFMA
  constexpr int KS = (DP + KB - 1) / KB;      // MFMA steps per row
  constexpr int LDW = KS * KB + 16;  // bytes per LDS row (whole K blocks, 16-byte pad)
  constexpr int BM = 4 * 32 * PB;
  constexpr int V_PER_ROW = DP / 16;  // 16-byte vectors per row
  constexpr int LOADS = (TN * V_PER_ROW + kBlock - 1) / kBlock;
  __shared__ uint4 s_c[2][TN * LDW / 16];
  __shared__ float s_hn[2][TN];
  __shared__ float s_sc[2][TN];

  const unsigned lb = xcd_remap8(blockIdx.x, gridDim.x);
  const int chunk = (int)(lb / (unsigned)tiles_per_chunk);
  const int tile = (int)(lb % (unsigned)tiles_per_chunk);
  const int64_t c0 = chunk_off[chunk], c1 = chunk_off[chunk + 1];
  const int64_t pbase = c0 + (int64_t)tile * BM;
  if (pbase >= c1) return;

  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int h = lane >> 5, col = lane & 31;
  using BOp = typename std::conditional<K64, v8i32, long>::type;
  BOp bq[PB][KS];
  float sx[PB];
  int64_t pidx[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t p = pbase + (wave * PB + pb) * 32 + col;
    pidx[pb] = p;
    const bool ok = p < c1;
    const uint8_t* row = items + (ok ? p : c0) * (int64_t)ldq;
    sx[pb] = iscale[ok ? p : c0];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if constexpr (K64) {
        const int c = 64 * s + 32 * h;  // two 16-byte halves, zero past the row
        uint4 lo = make_uint4(0u, 0u, 0u, 0u), hi = lo;
        if (ok && c < ldq) lo = *reinterpret_cast<const uint4*>(row + c);
        if (ok && c + 16 < ldq) hi = *reinterpret_cast<const uint4*>(row + c + 16);
        v8i32 v;
        v[0] = (int)lo.x; v[1] = (int)lo.y; v[2] = (int)lo.z; v[3] = (int)lo.w;
        v[4] = (int)hi.x; v[5] = (int)hi.y; v[6] = (int)hi.z; v[7] = (int)hi.w;
        bq[pb][s] = v;
      } else {
        const int c = 16 * s + 8 * h;
        long v = 0;
        if (ok && c < ldq) v = *reinterpret_cast<const long*>(row + c);
        bq[pb][s] = v;
      }
    }
  }
  const uint8_t* cbase = protos + (int64_t)chunk * k * ldq;
  const float* nbase = pnorm + (int64_t)chunk * k;
  const float* sbase = pscale + (int64_t)chunk * k;
  const int ntiles = (k + TN - 1) / TN;
  uint4 stage[LOADS];
  float hstage = 0.f, sstage = 0.f;
  int tile_base = 0;
  auto load_tile = [&](int t) {
    tile_base = t * TN;
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int idx = threadIdx.x + i * kBlock;
      const int row = idx / V_PER_ROW, v16 = idx % V_PER_ROW;
      const int j = min(t * TN + row, k - 1);
      const bool in = idx < TN * V_PER_ROW && v16 * 16 < ldq;
      const uint4 v =
          *reinterpret_cast<const uint4*>(cbase + (int64_t)j * ldq + (in ? v16 * 16 : 0));
      stage[i] = in ? v : make_uint4(0, 0, 0, 0);
    }
    if (threadIdx.x < TN) {
      const int j = min(t * TN + (int)threadIdx.x, k - 1);
      hstage = nbase[j];
      sstage = sbase[j];
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int idx = threadIdx.x + i * kBlock;
      if (idx < TN * V_PER_ROW) {
        const int row = idx / V_PER_ROW, v16 = idx % V_PER_ROW;
        s_c[buf][(row * LDW) / 16 + v16] = stage[i];
      }
    }
    if (threadIdx.x < TN) {
      const bool real = tile_base + (int)threadIdx.x < k;
      s_hn[buf][threadIdx.x] = real ? -0.5f * hstage : -INFINITY;
      s_sc[buf][threadIdx.x] = sstage;
    }
  };
  load_tile(0);
  store_tile(0);
  __syncthreads();

  float b1[PB];
  int i1[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) { b1[pb] = -INFINITY; i1[pb] = 0; }

  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    if (t + 1 < ntiles) load_tile(t + 1);
#pragma unroll
    for (int cb = 0; cb < TN / 32; ++cb) {
      floatx16 acc[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[pb][i] = 0.f;
      if constexpr (K64) {
        const uint8_t* arow =
            reinterpret_cast<const uint8_t*>(&s_c[buf][0]) + (cb * 32 + col) * LDW + 32 * h;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          // bytes 64s + 32h .. + 31 of the prototype row (inside the padded
          // LDS row), zero past the row's end
          const int c = 64 * s + 32 * h;
          uint4 lo = *reinterpret_cast<const uint4*>(arow + 64 * s);
          uint4 hi = *reinterpret_cast<const uint4*>(arow + 64 * s + 16);
          if (c >= DP) lo = make_uint4(0u, 0u, 0u, 0u);
          if (c + 16 >= DP) hi = make_uint4(0u, 0u, 0u, 0u);
          v8i32 a;
          a[0] = (int)lo.x; a[1] = (int)lo.y; a[2] = (int)lo.z; a[3] = (int)lo.w;
          a[4] = (int)hi.x; a[5] = (int)hi.y; a[6] = (int)hi.z; a[7] = (int)hi.w;
#pragma unroll
          for (int pb = 0; pb < PB; ++pb)
            acc[pb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, bq[pb][s], acc[pb], 0, 0,
                                                                     0, 127, 0, 127);
        }
      } else {
        const uint8_t* arow =
            reinterpret_cast<const uint8_t*>(&s_c[buf][0]) + (cb * 32 + col) * LDW + 8 * h;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const long a = *reinterpret_cast<const long*>(arow + 16 * s);  // dims 16s + 8h .. +7
#pragma unroll
          for (int pb = 0; pb < PB; ++pb)
            acc[pb] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, bq[pb][s], acc[pb], 0, 0, 0);
        }
      }
      const int jbase = t * TN + cb * 32 + 4 * h;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = cb * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
        const float hv = s_hn[buf][r], sc = s_sc[buf][r];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) acc[pb][i] = fmaf(acc[pb][i], sc * sx[pb], hv);
      }
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        float m = fmaxf(fmaxf(acc[pb][0], acc[pb][1]), acc[pb][2]);
#pragma unroll
        for (int i = 3; i < 15; i += 2) m = fmaxf(fmaxf(m, acc[pb][i]), acc[pb][i + 1]);
        m = fmaxf(m, acc[pb][15]);
        if (m > b1[pb]) {
          int ii = 15;
#pragma unroll
          for (int i = 14; i >= 0; --i) ii = (acc[pb][i] == m) ? i : ii;
          b1[pb] = m;
          i1[pb] = jbase + 8 * (ii >> 2) + (ii & 3);
        }
      }
    }
    if (t + 1 < ntiles) store_tile(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const float o = __shfl_xor(b1[pb], 32);
    const int oi = __shfl_xor(i1[pb], 32);
    if (o > b1[pb] || (o == b1[pb] && oi < i1[pb])) { b1[pb] = o; i1[pb] = oi; }
    if (h == 0 && pidx[pb] < c1) labels[pidx[pb]] = chunk * k + i1[pb];
  }
}

template <int DP, int PB, int TN, int MINB>
void launch_fp8(const ChunkPlan& plan, int32_t* labels, KmeansWork& w, hipStream_t s) {
  constexpr int BM = 4 * 32 * PB;
  const int tiles = (int)((plan.max_chunk + BM - 1) / BM);
  ScopedTiming timing("assign_fp8_mfma", s);
  k_assign_fp8<DP, PB, TN, MINB><<<(unsigned)(tiles * plan.n_chunks), kBlock, 0, s>>>(
      w.items_q, w.items_qs, w.ldq, w.protos_q, w.protos_qs, w.proto_norms_q, plan.d_off,
      plan.k, tiles, labels);
  check_launch("assign_fp8_mfma");
}

}  // namespace

int fp8_stride(int ld) { return (ld + 15) & ~15; }

void quantize_fp8(const float* x, int ld, int64_t n, uint8_t* out, int ldq, float* scale,
                  float* norms, hipStream_t s) {
  if (n <= 0) return;
  const int c16 = ldq / 16;
  if (c16 <= 1)
    k_quantize_fp8<1><<<grid_for(n, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldq, scale, norms);
  else if (c16 <= 2)
    k_quantize_fp8<2><<<grid_for(n * 2, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldq, scale,
                                                                 norms);
  else if (c16 <= 4)
    k_quantize_fp8<4><<<grid_for(n * 4, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldq, scale,
                                                                 norms);
  else if (c16 <= 8)
    k_quantize_fp8<8><<<grid_for(n * 8, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldq, scale,
                                                                 norms);
  else
    k_quantize_fp8<16><<<grid_for(n * 16, kBlock), kBlock, 0, s>>>(x, ld, n, out, ldq, scale,
                                                                   norms);
  check_launch("quantize_fp8");
}

void kmeans_assign_fp8(int ld, const ChunkPlan& plan, const float* protos, int32_t* labels,
                       KmeansWork& w, hipStream_t s) {
  quantize_fp8(protos, ld, (int64_t)plan.n_chunks * plan.k, w.protos_q, w.ldq, w.protos_qs,
               w.proto_norms_q, s);
  const int dp = w.ldq;  // a multiple of 16
  if (dp <= 16) launch_fp8<16, 4, 128, 2>(plan, labels, w, s);
  else if (dp <= 32) launch_fp8<32, 4, 64, 2>(plan, labels, w, s);
  else if (dp <= 64) launch_fp8<64, 2, 64, 2>(plan, labels, w, s);
  else if (dp <= 96) launch_fp8<96, 2, 64, 2>(plan, labels, w, s);
  else if (dp <= 128) launch_fp8<128, 2, 64, 2>(plan, labels, w, s);
  else if (dp <= 256) launch_fp8<256, 1, 64, 2>(plan, labels, w, s);
  else throw Error{MASK_ERR_UNSUPPORTED, "FP8 dimension above 256"};
}

}  // namespace mask

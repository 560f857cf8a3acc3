// Multilevel descent of Algorithm 2 with a beam of r prototypes per level.
//
// One workgroup (256 threads) runs the whole descent of one query, so a
// query's result never depends on the rest of the batch.  At each level the
// candidates are the children of the prototypes kept one level up (the top
// level: every prototype); children are contiguous in the level's position
// order.  Groups of TPR lanes compute direct-form distances (float4 loads,
// a fixed per-lane order, then a butterfly over the group), pack them with
// the candidate's original id into a 64-bit key (distance bits high, id
// low: a total order that breaks ties by the lower id), and append the keys
// that beat the current threshold to an LDS buffer.  Whenever the buffer
// may overflow, a radix select keeps the r smallest keys and the threshold
// drops to the largest kept key.  The data layer keeps the k smallest and
// ranks them.
#include "internal.hpp"

#include <cmath>

namespace mask {
namespace {

constexpr int kBlock = 256;
constexpr int kCap = 2560;  // LDS key buffer; kCap - kMaxBeam >= 2048 new keys per round

struct SelShared {
  uint64_t kmin, kmax, thr;
  uint32_t cnt, n_out, bin, below, bin_cnt;
};

__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}
__device__ inline uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

// Keeps the `want` smallest of buf[0..m) in buf[0..want) (any order) and
// sets sh.thr to the largest kept key.  Keys must be distinct.  Called by
// every thread of the block; m > want >= 1.
__device__ void block_select(uint64_t* buf, uint32_t m, uint32_t want, uint64_t* out,
                             uint32_t* hist, SelShared& sh, uint64_t* red) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  uint64_t lo = ~0ull, hi = 0ull;
  for (uint32_t i = tid; i < m; i += kBlock) {
    const uint64_t v = buf[i];
    lo = v < lo ? v : lo;
    hi = v > hi ? v : hi;
  }
  lo = wave_min_u64(lo);
  hi = wave_max_u64(hi);
  if (lane == 0) { red[wave] = lo; red[4 + wave] = hi; }
  __syncthreads();
  if (tid == 0) {
    uint64_t a = red[0], b = red[4];
    for (int w = 1; w < 4; ++w) {
      a = red[w] < a ? red[w] : a;
      b = red[4 + w] > b ? red[4 + w] : b;
    }
    sh.kmin = a;
    sh.kmax = b;
    sh.n_out = 0;
    sh.thr = 0;
  }
  __syncthreads();
  const uint64_t diff = sh.kmin ^ sh.kmax;  // non-zero: keys are distinct and m >= 2
  int top = 64 - __clzll((long long)diff);  // bits [top, 64) are common to all keys
  uint64_t prefix = (top >= 64) ? 0ull : (sh.kmin >> top) << top;
  uint32_t need = want;
  int shift = top;
  for (;;) {
    const int w = shift < 8 ? shift : 8;
    const int hi_bit = shift;  // bits >= hi_bit must equal prefix
    shift -= w;
    const uint32_t nb = 1u << w;
    for (uint32_t i = tid; i < nb; i += kBlock) hist[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < m; i += kBlock) {
      const uint64_t v = buf[i];
      const bool match = (hi_bit >= 64) || (((v ^ prefix) >> hi_bit) == 0);
      if (match) atomicAdd(&hist[(uint32_t)(v >> shift) & (nb - 1)], 1u);
    }
    __syncthreads();
    if (wave == 0) {
      // inclusive scan of nb <= 256 bins, 4 per lane
      uint32_t c[4], s = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t b = lane * 4 + j;
        c[j] = b < nb ? hist[b] : 0u;
        s += c[j];
      }
      uint32_t x = s;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
      }
      uint32_t run = x - s;  // exclusive prefix of this lane's 4 bins
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t b = lane * 4 + j;
        if (b < nb && run < need && run + c[j] >= need) {
          sh.bin = b;
          sh.below = run;
          sh.bin_cnt = c[j];
        }
        run += c[j];
      }
    }
    __syncthreads();
    const uint32_t b = sh.bin, below = sh.below, bin_cnt = sh.bin_cnt;
    need -= below;
    prefix |= (uint64_t)b << shift;
    __syncthreads();
    if (bin_cnt == need || shift == 0) break;
  }
  // Kept: every key whose bits at and above `shift` do not exceed the prefix.
  const uint64_t lim = prefix >> shift;
  for (uint32_t i = tid; i < m; i += kBlock) {
    const uint64_t v = buf[i];
    if ((v >> shift) <= lim) {
      const uint32_t slot = atomicAdd(&sh.n_out, 1u);
      if (slot < want) {  // exactly `want` keys qualify when keys are distinct
        out[slot] = v;
        atomicMax((unsigned long long*)&sh.thr, (unsigned long long)v);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < want; i += kBlock) buf[i] = out[i];
  __syncthreads();
}

// TPR lanes per candidate row; NV float4 of the row per lane (0: any number,
// looped); U rows in flight per lane group.
template <int TPR, int NV, int U, int METRIC>
__global__ __launch_bounds__(kBlock) void k_descent(DescentArgs a, const float* __restrict__ Q,
                                                    int ldq, int64_t nq, int k, int r,
                                                    int32_t* __restrict__ out_ids,
                                                    float* __restrict__ out_dist,
                                                    int32_t* __restrict__ sel_out,
                                                    unsigned long long* __restrict__ rows_out) {
  extern __shared__ float4 s_q4[];  // ld/4 float4
  __shared__ uint64_t s_buf[kCap];
  __shared__ uint64_t s_out[kMaxBeam];
  __shared__ int32_t s_par[kMaxBeam];       // kept positions one level up
  __shared__ uint32_t s_beg[kMaxBeam];      // first child position of each
  __shared__ uint32_t s_pre[kMaxBeam + 1];  // prefix of child counts
  __shared__ uint32_t s_hist[256];
  __shared__ uint64_t s_red[8];
  __shared__ SelShared sh;

  const int64_t qi = blockIdx.x;
  if (qi >= nq) return;
  const int tid = threadIdx.x, lane = tid % kWave;
  const int ld = a.ld, ld4 = ld / 4;
  float* s_q = reinterpret_cast<float*>(s_q4);
  for (int c = tid; c < ld; c += kBlock) s_q[c] = (c < a.dim) ? Q[qi * ldq + c] : 0.f;

  const int L = a.n_levels;
  int n_par = 1;
  if (tid == 0) { s_beg[0] = 0; s_pre[0] = 0; s_pre[1] = (uint32_t)a.lv[L].n; }
  __syncthreads();

  const int grp = tid / TPR, gl = tid % TPR;
  constexpr int kGroups = kBlock / TPR;
  constexpr int NQ = NV > 0 ? NV : 1;
  float4 qv[NQ];
#pragma unroll
  for (int v = 0; v < NQ; ++v) {
    const int c4 = gl + v * TPR;
    qv[v] = (NV > 0 && c4 < ld4) ? s_q4[c4] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  unsigned long long rows_seen = 0;

  for (int lev = L; lev >= 0; --lev) {
    const LevelView V = a.lv[lev];
    const uint32_t m = s_pre[n_par];
    rows_seen += m;
    const uint32_t want = (lev == 0) ? (uint32_t)k : (uint32_t)r;
    const uint32_t round = kCap - want;
    if (tid == 0) { sh.cnt = 0; sh.thr = ~0ull; }
    __syncthreads();
    uint64_t thr = ~0ull;
    for (uint32_t base = 0; base < m; base += round) {
      const uint32_t end = (m - base < round) ? m : base + round;
      for (uint32_t i0 = base + grp * U; i0 < end; i0 += kGroups * U) {
        // parent of i0: the last j with s_pre[j] <= i0; later rows walk forward
        int lo = 0, hi = n_par - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= i0) lo = mid; else hi = mid - 1;
        }
        int64_t pos[U];
        bool val[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t idx = i0 + u;
          val[u] = idx < end;
          while (val[u] && lo + 1 < n_par && s_pre[lo + 1] <= idx) ++lo;
          pos[u] = (int64_t)s_beg[lo] + (idx - s_pre[lo]);
        }
        float acc[U];
        if constexpr (NV > 0) {
          float4 x[U][NV];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const float4* row = reinterpret_cast<const float4*>(V.protos + (val[u] ? pos[u] : 0) * ld);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const int c4 = gl + v * TPR;
              x[u][v] = (val[u] && c4 < ld4) ? row[c4] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            float s0 = 0.f;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const float dx = x[u][v].x - qv[v].x, dy = x[u][v].y - qv[v].y,
                          dz = x[u][v].z - qv[v].z, dw = x[u][v].w - qv[v].w;
              if (METRIC == 0) {
                s0 = fmaf(dx, dx, s0); s0 = fmaf(dy, dy, s0);
                s0 = fmaf(dz, dz, s0); s0 = fmaf(dw, dw, s0);
              } else {
                s0 += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
              }
            }
            acc[u] = s0;
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const float4* row = reinterpret_cast<const float4*>(V.protos + (val[u] ? pos[u] : 0) * ld);
            float s0 = 0.f;
            for (int c4 = gl; c4 < ld4; c4 += TPR) {
              const float4 xv = val[u] ? row[c4] : make_float4(0.f, 0.f, 0.f, 0.f);
              const float4 q = s_q4[c4];
              const float dx = xv.x - q.x, dy = xv.y - q.y, dz = xv.z - q.z, dw = xv.w - q.w;
              if (METRIC == 0) {
                s0 = fmaf(dx, dx, s0); s0 = fmaf(dy, dy, s0);
                s0 = fmaf(dz, dz, s0); s0 = fmaf(dw, dw, s0);
              } else {
                s0 += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
              }
            }
            acc[u] = s0;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
          for (int o = TPR / 2; o >= 1; o >>= 1) acc[u] += __shfl_xor(acc[u], o);
        }
        if (gl == 0) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (!val[u]) continue;
            const uint32_t id = (uint32_t)V.orig[pos[u]];
            const uint64_t key = ((uint64_t)__float_as_uint(acc[u]) << 32) | id;
            if (key < thr) {
              const uint32_t slot = atomicAdd(&sh.cnt, 1u);
              if (slot < (uint32_t)kCap) s_buf[slot] = key;  // rounds keep slot < kCap
            }
          }
        }
      }
      __syncthreads();
      const uint32_t cnt = sh.cnt < (uint32_t)kCap ? sh.cnt : (uint32_t)kCap;
      if (cnt > want) {
        block_select(s_buf, cnt, want, s_out, s_hist, sh, s_red);
        if (tid == 0) sh.cnt = want;
        __syncthreads();
        thr = sh.thr;
      }
    }
    const uint32_t kept = sh.cnt < want ? sh.cnt : want;
    if (lev > 0) {
      // next level's parents: positions of the kept prototypes
      for (uint32_t j = tid; j < kept; j += kBlock) {
        const uint32_t id = (uint32_t)s_buf[j];
        const int32_t pos = V.inv[id];
        s_par[j] = pos;
        s_beg[j] = V.child_off[pos];
      }
      if (sel_out) {
        int32_t* so = sel_out + ((int64_t)qi * L + (L - lev)) * r;
        for (int j = tid; j < r; j += kBlock)
          so[j] = (uint32_t)j < kept ? (int32_t)(uint32_t)s_buf[j] : -1;
      }
      __syncthreads();
      if (tid < kWave) {
        // exclusive prefix of child counts, kMaxBeam / 64 = 8 per lane
        constexpr int P = kMaxBeam / kWave;
        uint32_t c[P], s = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const uint32_t e = lane * P + j;
          c[j] = 0;
          if (e < kept) c[j] = V.child_off[s_par[e] + 1] - s_beg[e];
          s += c[j];
        }
        uint32_t x = s;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const uint32_t y = __shfl_up(x, o);
          if (lane >= o) x += y;
        }
        uint32_t run = x - s;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const uint32_t e = lane * P + j;
          if (e < kept) s_pre[e] = run;
          run += c[j];
        }
        if (lane == kWave - 1) s_pre[kept] = x;
      }
      n_par = (int)kept;
      __syncthreads();
      if (n_par == 0) {
        if (tid == 0) s_pre[0] = 0;
        n_par = 1;  // one empty range
        if (tid == 0) { s_beg[0] = 0; s_pre[1] = 0; }
        __syncthreads();
      }
    } else {
      // rank the kept keys and write the result row
      for (uint32_t j = tid; j < kept; j += kBlock) {
        const uint64_t v = s_buf[j];
        uint32_t rank = 0;
        for (uint32_t t = 0; t < kept; ++t) rank += s_buf[t] < v;
        s_out[rank] = v;
      }
      __syncthreads();
      for (int j = tid; j < k; j += kBlock) {
        int32_t id = -1;
        float dist = INFINITY;
        if ((uint32_t)j < kept) {
          const uint64_t v = s_out[j];
          id = (int32_t)(uint32_t)v;
          const float d2 = __uint_as_float((uint32_t)(v >> 32));
          dist = METRIC == 0 ? sqrtf(d2) : d2;
        }
        out_ids[qi * k + j] = id;
        out_dist[qi * k + j] = dist;
      }
    }
  }
  if (rows_out && tid == 0) atomicAdd(rows_out, rows_seen);
}

template <int TPR, int NV, int U>
void launch_descent(const DescentArgs& a, const float* q, int ldq, int64_t nq, int k, int r,
                    int32_t* out_ids, float* out_dist, int32_t* sel, unsigned long long* rows,
                    hipStream_t s) {
  const size_t shm = (size_t)a.ld * sizeof(float);
  ScopedTiming timing("descent", s);
  if (a.metric == MASK_L2)
    k_descent<TPR, NV, U, 0><<<(unsigned)nq, kBlock, shm, s>>>(a, q, ldq, nq, k, r, out_ids,
                                                              out_dist, sel, rows);
  else
    k_descent<TPR, NV, U, 1><<<(unsigned)nq, kBlock, shm, s>>>(a, q, ldq, nq, k, r, out_ids,
                                                              out_dist, sel, rows);
  check_launch("descent");
}

}  // namespace

void descent(const DescentArgs& a, const float* q, int ldq, int64_t nq, int k, int r,
             int32_t* out_ids, float* out_dist, int32_t* sel, unsigned long long* rows,
             hipStream_t s) {
  if (nq <= 0) return;
  const int f4 = a.ld / 4;
  if (f4 <= 1) launch_descent<1, 1, 4>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else if (f4 <= 2) launch_descent<2, 1, 4>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else if (f4 <= 4) launch_descent<4, 1, 4>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else if (f4 <= 8) launch_descent<8, 1, 4>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else if (f4 <= 16) launch_descent<16, 1, 4>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else if (f4 <= 32) launch_descent<16, 2, 4>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else if (f4 <= 64) launch_descent<16, 4, 2>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else if (f4 <= 128) launch_descent<16, 8, 1>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
  else launch_descent<16, 0, 1>(a, q, ldq, nq, k, r, out_ids, out_dist, sel, rows, s);
}

}  // namespace mask

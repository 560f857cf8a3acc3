// Multilevel descent of Algorithm 2 with a beam of r prototypes per level.
//
// Precision form (BF16): every level's rows are read as BF16 (half the
// bytes) and ranked with FP32 arithmetic against the FP32 query; at the data
// layer the rerank_factor * k nearest by BF16 distance are re-ranked in
// FP32 direct form on the FP32 rows, and the k nearest of those are returned.
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

#include <algorithm>
#include <cfloat>
#include <cmath>

namespace mask {
namespace {

constexpr int kBlock = 256;

struct SelShared {
  uint64_t kmin, kmax, thr;
  uint32_t cnt, n_out, bin, below, bin_cnt;
  uint32_t in_range;  // range search: data rows within the radius
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
// every thread of the block; m > want >= 1.  Most-significant-digit radix
// select over the bits below the keys' common prefix, 8 bits per pass.  The
// digit histograms rotate over three buffers and every wave scans the
// histogram itself, so a pass costs one barrier: pass p counts into buffer
// p % 3 and clears buffer (p + 1) % 3, which was last read in pass p - 2
// (before the barrier of pass p - 1) and is next counted into after the
// barrier of pass p.  hist: 3 * 256 counters.
// Sets of at most kRankSelect keys are selected by rank instead (measured:
// above 128 keys the radix passes are faster): every key counts the keys
// below it (broadcast LDS reads, two keys per read), and a key of rank < want
// goes to slot `rank` of out (ranks of distinct keys are distinct, so no slot
// is written twice).  The kept keys come out sorted.
constexpr uint32_t kRankSelect = 128;

__device__ void block_select(uint64_t* buf, uint32_t m, uint32_t want, uint64_t* out,
                             uint32_t* hist, SelShared& sh, uint64_t* red) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  if (m <= kRankSelect) {
    const uint32_t pairs = m / 2;
    const ulonglong2* b2 = reinterpret_cast<const ulonglong2*>(buf);  // buf is 16-byte aligned
    for (uint32_t i = tid; i < m; i += kBlock) {
      const uint64_t v = buf[i];
      uint32_t rank = 0;
      for (uint32_t j = 0; j < pairs; ++j) {
        const ulonglong2 w = b2[j];
        rank += (w.x < v) + (w.y < v);
      }
      if (m & 1u) rank += buf[m - 1] < v;
      if (rank < want) out[rank] = v;
      if (rank == want - 1) sh.thr = v;
    }
    __syncthreads();
    for (uint32_t i = tid; i < want; i += kBlock) buf[i] = out[i];
    __syncthreads();
    return;
  }
  uint64_t lo = ~0ull, hi = 0ull;
  for (uint32_t i = tid; i < m; i += kBlock) {
    const uint64_t v = buf[i];
    lo = v < lo ? v : lo;
    hi = v > hi ? v : hi;
  }
  lo = wave_min_u64(lo);
  hi = wave_max_u64(hi);
  if (lane == 0) { red[wave] = lo; red[4 + wave] = hi; }
  for (uint32_t i = tid; i < 256; i += kBlock) hist[i] = 0;
  if (tid == 0) { sh.n_out = 0; sh.thr = 0; }
  __syncthreads();
  uint64_t kmin = red[0], kmax = red[4];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    kmin = red[w] < kmin ? red[w] : kmin;
    kmax = red[4 + w] > kmax ? red[4 + w] : kmax;
  }
  const uint64_t diff = kmin ^ kmax;  // non-zero: keys are distinct and m >= 2
  const int top = 64 - __clzll((long long)diff);  // bits [top, 64) are common to all keys
  uint64_t prefix = (top >= 64) ? 0ull : (kmin >> top) << top;
  uint32_t need = want;
  int shift = top;
  int pass = 0;
  for (;;) {
    const int w = shift < 8 ? shift : 8;
    const int hi_bit = shift;  // bits >= hi_bit equal the prefix
    shift -= w;
    const uint32_t nb = 1u << w;
    uint32_t* h = hist + (pass % 3) * 256;
    uint32_t* h_next = hist + ((pass + 1) % 3) * 256;
    for (uint32_t i = tid; i < 256; i += kBlock) h_next[i] = 0;
    for (uint32_t i = tid; i < m; i += kBlock) {
      const uint64_t v = buf[i];
      const bool match = (hi_bit >= 64) || (((v ^ prefix) >> hi_bit) == 0);
      if (match) atomicAdd(&h[(uint32_t)(v >> shift) & (nb - 1)], 1u);
    }
    __syncthreads();
    // every wave finds the bin holding the need-th key: 4 bins per lane
    uint32_t c[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t b = lane * 4 + j;
      c[j] = b < nb ? h[b] : 0u;
      sum += c[j];
    }
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    uint32_t run = x - sum;
    uint32_t found = 0;  // (bin + 1) on the lane that holds it
    uint32_t f_below = 0, f_cnt = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t b = lane * 4 + j;
      if (b < nb && run < need && run + c[j] >= need) {
        found = b + 1;
        f_below = run;
        f_cnt = c[j];
      }
      run += c[j];
    }
    const uint64_t fm = __ballot(found != 0);
    const int src = __ffsll((long long)fm) - 1;
    const uint32_t b = __shfl(found, src) - 1;
    const uint32_t below = __shfl(f_below, src);
    const uint32_t bin_cnt = __shfl(f_cnt, src);
    need -= below;
    prefix |= (uint64_t)b << shift;
    ++pass;
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

template <int NV, int TPR>
struct QFrag {
  float4 v[NV > 0 ? NV : 1][2];
};

__device__ inline float4 bf16_lo4(uint2 w) {
  return make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u),
                     __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xffff0000u));
}

template <int METRIC>
__device__ inline float acc4(float s, float4 x, float4 q) {
  const float dx = x.x - q.x, dy = x.y - q.y, dz = x.z - q.z, dw = x.w - q.w;
  if (METRIC == 0) {
    s = fmaf(dx, dx, s); s = fmaf(dy, dy, s); s = fmaf(dz, dz, s); s = fmaf(dw, dw, s);
  } else {
    s += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
  }
  return s;
}

// Butterfly step within a lane group: lane ^ O.  Within a quad (O = 1, 2)
// a DPP quad permutation on the vector unit; otherwise a cross-lane shuffle.
// Both move the value exactly, so sums equal the __shfl_xor butterfly's.
template <int O>
__device__ inline float xor_lane(float v) {
  if constexpr (O == 1)  // quad_perm(1, 0, 3, 2)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
  else if constexpr (O == 2)  // quad_perm(2, 3, 0, 1)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
  else
    return __shfl_xor(v, O);
}

// Sum over a lane group of TPR lanes (the butterfly from the widest step).
template <int TPR>
__device__ inline float group_sum(float v) {
  if constexpr (TPR >= 16) v += xor_lane<8>(v);
  if constexpr (TPR >= 8) v += xor_lane<4>(v);
  if constexpr (TPR >= 4) v += xor_lane<2>(v);
  if constexpr (TPR >= 2) v += xor_lane<1>(v);
  return v;
}

// Descent of one query per workgroup.
//   TPR lanes per candidate row, NV 16-byte vectors of the row per lane
//   (0: any number, looped), U rows in flight per lane group; B16: rows are
//   BF16; BEAMB: largest prototype beam; CAPB: largest beam / k / re-rank
//   set; CAP: LDS key buffer.
//   SP: CSR index.  The query row is scattered into the dense LDS vector and
//   its non-zeros are listed in LDS (the first kQList); CSR data rows are
//   walked against the dense vector, dense prototype rows are gathered at the
//   query's columns; dot products and |q|^2 + |c|^2 - 2 q.c in FP64.  The
//   query's norm and a data row's norm are summed on the fly with the same
//   lane split and order as their dot product, so a data row equal to the
//   query is at distance exactly 0.
constexpr int kQList = 1024;

//   MODE 0: dense rows; 1: CSR index (SP); 2: FP8 data rows with one FP32
//   scale per row (the FP8 variant of the precision form: prototype levels
//   in FP32, the data layer in FP8, re-ranked like BF16).
// The BF16 class with rounds of 2,048 candidates is held to 102 VGPRs (a few
// spill) so that five waves per SIMD fit, as its LDS allows: with the launch
// order the descent is bound by latency, and the fifth wave is worth more
// than the spills (measured on MI355X).
template <int TPR, int NV, int U, int METRIC, bool B16, int BEAMB, int CAPB, int CAP, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    B16 && CAP == 2048 ? 5 : 1))) void k_descent(DescentArgs a, QueryArgs qa) {
  constexpr bool SP = MODE == 1, F8 = MODE == 2, LOWP = B16 || F8;
  extern __shared__ float4 s_q4[];  // ld/4 float4
  __shared__ int32_t s_qc[SP ? kQList : 1];
  __shared__ float s_qv[SP ? kQList : 1];
  __shared__ __align__(16) uint64_t s_buf[CAP];
  __shared__ uint64_t s_out[CAPB];
  __shared__ uint32_t s_cnt[BEAMB];      // child count of each kept prototype
  __shared__ uint32_t s_beg[BEAMB];      // first child position of each
  __shared__ uint32_t s_pre[BEAMB + 1];  // prefix of child counts
  __shared__ uint32_t s_hist[3 * 256];
  __shared__ uint64_t s_red[8];
  __shared__ SelShared sh;

  int64_t qi = blockIdx.x;
  if (qa.order) {
    const int64_t pos = (int64_t)(blockIdx.x % kXcds) * qa.per_xcd + blockIdx.x / kXcds;
    if (pos >= qa.nq) return;
    qi = qa.order[pos];
  }
  if (qi >= qa.nq) return;
  const int tid = threadIdx.x, lane = tid % kWave;
  const int ld = a.ld, ld4 = ld / 4, ldb = a.ldb;
  const int k = qa.k_arr ? min(max(qa.k_arr[qi], 1), qa.k) : qa.k;
  const int r = qa.r_arr ? min(max(qa.r_arr[qi], 1), qa.r) : qa.r;
  const int64_t obase = qa.out_off ? qa.out_off[qi] : qi * (int64_t)qa.k;
  // Range search (Algorithm 3): keys are admitted at every level only when
  // their squared distance is at most radius^2 (any id), and the per-level
  // beam becomes a cap; otherwise every key is admitted.
  const bool range = qa.radius != nullptr;
  uint64_t thr0 = ~0ull;
  if (range) {
    const float rq = qa.radius[qi];
    thr0 = (rq >= 0.f && rq <= FLT_MAX)
               ? (((uint64_t)__float_as_uint(rq * rq) << 32) | 0xffffffffull)
               : 0ull;
  }
  float* s_q = reinterpret_cast<float*>(s_q4);
  int64_t qb = 0;
  int nq_e = 0;
  if constexpr (SP) {
    qb = qa.q_ptr[qi];
    nq_e = (int)(qa.q_ptr[qi + 1] - qb);
    for (int c = tid; c < ld; c += kBlock) s_q[c] = 0.f;
    __syncthreads();
    // query rows are not checked by the library: a column id out of range
    // is dropped (value 0 at column 0) rather than read or written out of
    // bounds
    for (int t = tid; t < nq_e; t += kBlock) {
      int32_t c = qa.q_col[qb + t];
      float v = qa.q_val[qb + t];
      if (c < 0 || c >= a.dim) { c = 0; v = 0.f; }
      if (v != 0.f) s_q[c] = v;
      if (t < kQList) { s_qc[t] = c; s_qv[t] = v; }
    }
  } else {
    for (int c = tid; c < ld; c += kBlock) s_q[c] = (c < a.dim) ? qa.Q[qi * qa.ldq + c] : 0.f;
  }

  const int L = a.n_levels;
  int n_par = 1;
  int lev_first = L;
  if (qa.leaf_mode == 2) {
    // the data layer only, from the leaves the first launch kept (slot
    // order), with the candidate offsets it wrote
    const int64_t lb = qi * (int64_t)qa.leaf_cap;
    const int nk = min((int)qa.n_kept[qi], qa.leaf_cap);
    for (int j = tid; j < nk; j += kBlock) {
      s_beg[j] = qa.leaf_b0[lb + j];
      s_cnt[j] = qa.leaf_cnt[lb + j];
      s_pre[j] = qa.leaf_off[lb + j];
    }
    if (tid == 0) {
      if (nk > 0) {
        s_pre[nk] = qa.leaf_off[lb + nk - 1] + qa.leaf_cnt[lb + nk - 1];
      } else {  // one empty range
        s_beg[0] = 0; s_pre[0] = 0; s_pre[1] = 0;
      }
    }
    n_par = nk > 0 ? nk : 1;
    lev_first = 0;
  } else if (tid == 0) {
    s_beg[0] = 0; s_pre[0] = 0; s_pre[1] = (uint32_t)a.lv[L].n;
  }
  __syncthreads();

  const int grp = tid / TPR, gl = tid % TPR;
  // |q|^2 of a CSR query, split over a lane group like a data row's dot product
  double qn = 0.0;
  if constexpr (SP) {
    for (int t = gl; t < nq_e; t += TPR) {
      double v = t < kQList ? s_qv[t] : qa.q_val[qb + t];
      if (t >= kQList && (qa.q_col[qb + t] < 0 || qa.q_col[qb + t] >= a.dim)) v = 0.0;
      qn = fma(v, v, qn);
    }
#pragma unroll
    for (int o = TPR / 2; o >= 1; o >>= 1) qn += __shfl_xor(qn, o);
  }
  constexpr int kGroups = kBlock / TPR;
  constexpr int NQ = NV > 0 ? NV : 1;
  // query fragment: FP32 rows use 4 dims per vector, BF16 rows 8
  float4 qv[NQ][2];
#pragma unroll
  for (int v = 0; v < NQ; ++v) {
    const int c = gl + v * TPR;
    // plain loads under a condition (a select between an LDS and a private
    // address would turn into flat loads and a scratch slot)
    qv[v][0] = make_float4(0.f, 0.f, 0.f, 0.f);
    qv[v][1] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (B16) {
      if (NV > 0 && 2 * c < ld4) qv[v][0] = s_q4[2 * c];
      if (NV > 0 && 2 * c + 1 < ld4) qv[v][1] = s_q4[2 * c + 1];
    } else {
      if (NV > 0 && c < ld4) qv[v][0] = s_q4[c];
    }
  }
  unsigned long long rows_seen = 0;
  // This query's beam at level l (top level first in r_lev / the profile).
  auto beam_at = [&](int l) -> int {
    if (qa.r_lev[l] > 0) return qa.r_lev[l];
    if (qa.beam_e8[l] > 0) return min((r * qa.beam_e8[l] + 7) / 8, BEAMB);
    return r;
  };
  // Re-rank set of the precision forms: rerank_factor * k candidates, or
  // with a negative factor f, |f| * k * (the level-1 beam); capped at 512
  // when it, k and every beam are at most 512, else at 2048, so that a
  // query's result does not depend on the other queries of a ragged batch
  // (the LDS class, CAPB, covers the whole batch and so every query's cap).
  const int64_t R0 = a.rerank_factor > 0
                         ? (int64_t)a.rerank_factor * k
                         : (int64_t)(-a.rerank_factor) * k * (int64_t)beam_at(1);
  bool big = k > 512 || r > 512 || R0 > 512;
  for (int l = 1; l <= L; ++l) big = big || beam_at(l) > 512;
  const int64_t rerank_cap = big ? 2048 : 512;

  for (int lev = lev_first; lev >= 0; --lev) {
    const LevelView V = a.lv[lev];
    const float* scr = qa.scr[lev];
    const int64_t sbase = qi * qa.scr_ld[lev];
    const uint32_t m = s_pre[n_par];
    // the data layer of the BF16 form keeps an oversized set for the FP32 re-rank
    uint32_t want = (lev == 0) ? (uint32_t)k : (uint32_t)beam_at(lev);
    // rows read in BF16 at every level, or in FP8 at the data layer only:
    // three mantissa bits are too coarse to choose prototypes
    bool low = B16 || (F8 && lev == 0);
    bool rerank = false;
    if (lev == 0 && LOWP) {
      const int64_t R = min(min(R0, rerank_cap), (int64_t)CAPB);
      if ((int64_t)m > R && R > k) {
        want = (uint32_t)R;
        rerank = true;
      } else {
        low = false;
      }
    }
    // the data layer of the leaf-batched descent: the BF16 distances are read
    const bool from_cand = qa.leaf_mode == 2 && lev == 0 && B16 && low;
    const int64_t cbase = from_cand ? (int64_t)qa.cand_off[qi] : 0;
    if (scr == nullptr && !from_cand) rows_seen += m;  // rows read, not scores
    // The first round is short (2 * want keys, at least 256): its exact
    // selection sets the threshold cheaply.  Later rounds take as many
    // candidates as the buffer has room for and append only keys below the
    // threshold; a selection runs when the buffer has less than 256 slots
    // left, and after the last round.
    const uint32_t first = min(CAP - want, max(2 * want, 256u));
    if (tid == 0) { sh.cnt = 0; sh.thr = thr0; sh.in_range = 0; }
    __syncthreads();
    uint64_t thr = thr0;
    uint32_t held = 0;  // keys in the buffer when a round starts (the same in every thread)
    for (uint32_t base = 0; base < m;) {
      const uint32_t len = (base == 0) ? first : (uint32_t)CAP - held;
      const uint32_t end = (m - base < len) ? m : base + len;
      if (scr != nullptr || from_cand) {
        // screened level (or the leaf-batched data layer): the distances were
        // computed for the whole batch, so every lane takes candidates of its
        // own (a binary search over the parents' prefix each)
        for (uint32_t idx = base + tid; idx < end; idx += kBlock) {
          int lo = 0, hi = n_par - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= idx) lo = mid; else hi = mid - 1;
          }
          const int64_t p = (int64_t)s_beg[lo] + (idx - s_pre[lo]);
          const float dv = from_cand ? qa.cand[cbase + idx] : scr[sbase + p];
          const uint64_t key = ((uint64_t)__float_as_uint(dv) << 32) | (uint32_t)V.orig[p];
          if (key < thr) {
            const uint32_t slot = atomicAdd(&sh.cnt, 1u);
            if (slot < (uint32_t)CAP) s_buf[slot] = key;  // rounds keep slot < CAP
          }
        }
      } else {
      // Each lane group takes a contiguous chunk of kChunk candidates: one
      // binary search over the parents' prefix per chunk, then a forward walk.
      // chunk = ceil(rows / groups) rounded up to U, between U and 8U
      const uint32_t per = (end - base + kGroups - 1) / kGroups;
      const uint32_t kChunk = min((uint32_t)(8 * U), max((uint32_t)U, (per + U - 1) / U * U));
      for (uint32_t c0 = base + grp * kChunk; c0 < end; c0 += kGroups * kChunk) {
      const uint32_t c1 = min(end, c0 + kChunk);
      int lo = 0;
      {
        int hi = n_par - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= c0) lo = mid; else hi = mid - 1;
        }
      }
      for (uint32_t i0 = c0; i0 < c1; i0 += U) {
        int64_t pos[U];
        bool val[U];
        uint32_t ids[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t idx = i0 + u;
          val[u] = idx < c1;
          while (val[u] && lo + 1 < n_par && s_pre[lo + 1] <= idx) ++lo;
          // an empty slot reads row 0 (present whenever the level has rows)
          pos[u] = val[u] ? (int64_t)s_beg[lo] + (idx - s_pre[lo]) : 0;
        }
        // Every load below is unconditional (indexes are clamped, values
        // selected afterwards), so the id and row loads of all U slots are in
        // flight together instead of each waiting behind a branch.
#pragma unroll
        for (int u = 0; u < U; ++u) ids[u] = (uint32_t)V.orig[pos[u]];
        float acc[U];
        if constexpr (SP) {
          double dot[U], cn[U];
#pragma unroll
          for (int u = 0; u < U; ++u) { dot[u] = 0.0; cn[u] = 0.0; }
          if (lev == 0) {
            // CSR data rows against the dense query in LDS
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int64_t b = V.sp_ptr[pos[u]], e = V.sp_ptr[pos[u] + 1];
#pragma unroll 4
              for (int64_t t = b + gl; t < e; t += TPR) {
                const double v = V.sp_val[t];
                dot[u] = fma(v, (double)s_q[V.sp_col[t]], dot[u]);
                cn[u] = fma(v, v, cn[u]);
              }
            }
          } else {
            // dense prototype rows gathered at the query's columns, U rows at once
            const float* rows[U];
#pragma unroll
            for (int u = 0; u < U; ++u) rows[u] = V.protos + pos[u] * ld;
#pragma unroll 2
            for (int t = gl; t < nq_e; t += TPR) {
              const bool in = t < kQList;
              int32_t c = in ? s_qc[t] : qa.q_col[qb + t];
              float v = in ? s_qv[t] : qa.q_val[qb + t];
              if (c < 0 || c >= a.dim) { c = 0; v = 0.f; }
              float x[U];
#pragma unroll
              for (int u = 0; u < U; ++u) x[u] = rows[u][c];
#pragma unroll
              for (int u = 0; u < U; ++u) dot[u] = fma((double)v, (double)x[u], dot[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int o = TPR / 2; o >= 1; o >>= 1) {
              dot[u] += __shfl_xor(dot[u], o);
              cn[u] += __shfl_xor(cn[u], o);
            }
            const double c2 = lev > 0 ? V.norm64[pos[u]] : cn[u];
            const double d = qn + c2 - 2.0 * dot[u];
            acc[u] = d > 0.0 ? (float)d : 0.f;
          }
        } else if (B16 && low) {
          const int nb = ldb / 8;
          if constexpr (NV > 0) {
            uint4 x[U][NV];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const uint4* row = reinterpret_cast<const uint4*>(V.protos_b + pos[u] * ldb);
#pragma unroll
              for (int v = 0; v < NV; ++v) {
                const int c = gl + v * TPR;
                const uint4 t = row[c < nb ? c : 0];
                x[u][v] = c < nb ? t : make_uint4(0, 0, 0, 0);
              }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              float s0 = 0.f;
#pragma unroll
              for (int v = 0; v < NV; ++v) {
                s0 = acc4<METRIC>(s0, bf16_lo4(make_uint2(x[u][v].x, x[u][v].y)), qv[v][0]);
                s0 = acc4<METRIC>(s0, bf16_lo4(make_uint2(x[u][v].z, x[u][v].w)), qv[v][1]);
              }
              acc[u] = s0;
            }
          } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const uint4* row = reinterpret_cast<const uint4*>(V.protos_b + pos[u] * ldb);
              float s0 = 0.f;
              for (int c = gl; c < nb; c += TPR) {
                const uint4 xv = row[c];
                const float4 q0 = 2 * c < ld4 ? s_q4[2 * c] : make_float4(0.f, 0.f, 0.f, 0.f);
                const float4 q1 = 2 * c + 1 < ld4 ? s_q4[2 * c + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
                s0 = acc4<METRIC>(s0, bf16_lo4(make_uint2(xv.x, xv.y)), q0);
                s0 = acc4<METRIC>(s0, bf16_lo4(make_uint2(xv.z, xv.w)), q1);
              }
              acc[u] = s0;
            }
          }
        } else if (F8 && low) {
          // FP8 rows: 16 dimensions per 16-byte chunk, dequantised with the
          // row's scale, FP32 direct form against the query in LDS
          const int nc = a.ldq / 16;
          const uint4* rowq[U];
          float rs[U], au[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            rowq[u] = reinterpret_cast<const uint4*>(V.protos_q + pos[u] * (int64_t)a.ldq);
            rs[u] = V.scale_q[pos[u]];
            au[u] = 0.f;
          }
          for (int c = gl; c < nc; c += TPR) {
            uint4 x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = rowq[u][c];
            float4 q[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
              q[e] = (4 * c + e < ld4) ? s_q4[4 * c + e] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const uint32_t w[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const float d0 = fmaf(rs[u], __builtin_amdgcn_cvt_f32_fp8((int)w[e], 0), -q[e].x);
                const float d1 = fmaf(rs[u], __builtin_amdgcn_cvt_f32_fp8((int)w[e], 1), -q[e].y);
                const float d2 = fmaf(rs[u], __builtin_amdgcn_cvt_f32_fp8((int)w[e], 2), -q[e].z);
                const float d3 = fmaf(rs[u], __builtin_amdgcn_cvt_f32_fp8((int)w[e], 3), -q[e].w);
                au[u] = fmaf(d0, d0, au[u]);
                au[u] = fmaf(d1, d1, au[u]);
                au[u] = fmaf(d2, d2, au[u]);
                au[u] = fmaf(d3, d3, au[u]);
              }
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) acc[u] = au[u];
        } else if (!B16 && NV > 0) {
          float4 x[U][NQ];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const float4* row = reinterpret_cast<const float4*>(V.protos + pos[u] * ld);
#pragma unroll
            for (int v = 0; v < NQ; ++v) {
              const int c4 = gl + v * TPR;
              const float4 t = row[c4 < ld4 ? c4 : 0];
              x[u][v] = c4 < ld4 ? t : make_float4(0.f, 0.f, 0.f, 0.f);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            float s0 = 0.f;
#pragma unroll
            for (int v = 0; v < NQ; ++v) s0 = acc4<METRIC>(s0, x[u][v], qv[v][0]);
            acc[u] = s0;
          }
        } else {
          // FP32 rows, any width (also the data layer of the BF16 form when
          // the re-rank set would hold every candidate)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const float4* row = reinterpret_cast<const float4*>(V.protos + pos[u] * ld);
            float s0 = 0.f;
            for (int c4 = gl; c4 < ld4; c4 += TPR) s0 = acc4<METRIC>(s0, row[c4], s_q4[c4]);
            acc[u] = s0;
          }
        }
        if constexpr (!SP) {
#pragma unroll
          for (int u = 0; u < U; ++u) acc[u] = group_sum<TPR>(acc[u]);
        }
        if (gl == 0) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (!val[u]) continue;
            // insertion descent: a prototype above level 1 without children
            // leads to no leaf and is not a candidate
            if (qa.skip_empty && lev >= 2 && V.child_off[pos[u] + 1] == V.child_off[pos[u]])
              continue;
            const uint64_t key = ((uint64_t)__float_as_uint(acc[u]) << 32) | ids[u];
            if (range && lev == 0 && key < thr0) atomicAdd(&sh.in_range, 1u);
            if (key < thr) {
              const uint32_t slot = atomicAdd(&sh.cnt, 1u);
              if (slot < (uint32_t)CAP) s_buf[slot] = key;  // rounds keep slot < CAP
            }
          }
        }
      }
      }
      }  // lane groups
      __syncthreads();
      const uint32_t cnt = sh.cnt < (uint32_t)CAP ? sh.cnt : (uint32_t)CAP;
      if (cnt > want && (base == 0 || end == m || cnt + 256 > (uint32_t)CAP)) {
        block_select(s_buf, cnt, want, s_out, s_hist, sh, s_red);
        if (tid == 0) sh.cnt = want;
        __syncthreads();
        thr = sh.thr;
        held = want;
      } else {
        // every thread has read the count before the next round appends to it
        __syncthreads();
        held = cnt;
      }
      base = end;
    }
    uint32_t kept = sh.cnt < want ? sh.cnt : want;
    if (lev > 0) {
      for (uint32_t j = tid; j < kept; j += kBlock) {
        const uint32_t id = (uint32_t)s_buf[j];
        const int32_t pos = V.inv[id];
        const uint32_t b0 = V.child_off[pos], b1 = V.child_off[pos + 1];
        s_beg[j] = b0;
        s_cnt[j] = b1 - b0;
      }
      if (qa.out_leaf && lev == 1 && tid == 0)
        qa.out_leaf[qi] = kept ? (int32_t)(uint32_t)s_buf[0] : -1;
      if (qa.sel) {
        int32_t* so = qa.sel + ((int64_t)qi * L + (L - lev)) * qa.r;
        for (int j = tid; j < qa.r; j += kBlock)
          so[j] = (uint32_t)j < kept ? (int32_t)(uint32_t)s_buf[j] : -1;
      }
      __syncthreads();
      if (tid < kWave) {
        constexpr int P = BEAMB / kWave;
        uint32_t c[P], s = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const uint32_t e = lane * P + j;
          c[j] = 0;
          if (e < kept) c[j] = s_cnt[e];
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
        n_par = 1;  // one empty range
        if (tid == 0) { s_beg[0] = 0; s_pre[0] = 0; s_pre[1] = 0; }
        __syncthreads();
      }
      if (qa.leaf_mode == 1 && lev == 1) {
        // the kept leaves, in slot order, for the leaf-by-leaf data layer
        const int64_t lb = qi * (int64_t)qa.leaf_cap;
        const uint32_t nk = min(kept, (uint32_t)qa.leaf_cap);
        for (uint32_t j = tid; j < (uint32_t)qa.leaf_cap; j += kBlock) {
          uint32_t key = (uint32_t)V.n, b0 = 0, cnt = 0, off = 0;
          if (j < nk) {
            b0 = s_beg[j];
            cnt = s_cnt[j];
            off = s_pre[j];
            if (cnt > 0) key = (uint32_t)V.inv[(uint32_t)s_buf[j]];
          }
          qa.leaf_b0[lb + j] = b0;
          qa.leaf_cnt[lb + j] = cnt;
          qa.leaf_off[lb + j] = off;
          qa.leaf_key[lb + j] = key;
          qa.leaf_val[lb + j] = (uint32_t)(lb + j);
        }
        if (tid == 0) {
          qa.n_kept[qi] = nk;
          qa.n_cand[qi] = nk > 0 ? s_pre[nk] : 0u;
          if (qa.rows) atomicAdd(qa.rows + blockIdx.x % kCounterShards, rows_seen);
        }
        return;  // every thread of the workgroup
      }
    } else {
      if (LOWP && rerank) {
        // FP32 direct form on the FP32 rows of the kept set, then the k nearest
        for (uint32_t j = grp; j < kept; j += kGroups) {
          const uint32_t id = (uint32_t)s_buf[j];
          const int64_t pos = a.inv0[id];
          const float4* row = reinterpret_cast<const float4*>(V.protos + pos * ld);
          float s0 = 0.f;
          for (int c4 = gl; c4 < ld4; c4 += TPR) s0 = acc4<METRIC>(s0, row[c4], s_q4[c4]);
          s0 = group_sum<TPR>(s0);
          if (gl == 0) s_out[j] = ((uint64_t)__float_as_uint(s0) << 32) | id;
        }
        __syncthreads();
        for (uint32_t j = tid; j < kept; j += kBlock) s_buf[j] = s_out[j];
        __syncthreads();
        if (kept > (uint32_t)k) {
          block_select(s_buf, kept, (uint32_t)k, s_out, s_hist, sh, s_red);
          kept = k;
        }
      }
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
        qa.out_ids[obase + j] = id;
        qa.out_dist[obase + j] = dist;
      }
      if (range && tid == 0) qa.out_count[qi] = (int32_t)sh.in_range;
    }
  }
  if (qa.rows && tid == 0) atomicAdd(qa.rows + blockIdx.x % kCounterShards, rows_seen);
}

template <int TPR, int NV, int U, bool B16, int BEAMB, int CAPB, int CAP, int MODE>
void launch3(const DescentArgs& a, const QueryArgs& qa, hipStream_t s) {
  const size_t shm = (size_t)a.ld * sizeof(float);
  const unsigned grid = (unsigned)(qa.order ? kXcds * qa.per_xcd : qa.nq);
  if constexpr (MODE != 0 || B16)  // CSR, FP8 and BF16 indexes are L2 only
    k_descent<TPR, NV, U, 0, B16, BEAMB, CAPB, CAP, MODE><<<grid, kBlock, shm, s>>>(a, qa);
  else if (a.metric == MASK_L2)
    k_descent<TPR, NV, U, 0, B16, BEAMB, CAPB, CAP, MODE><<<grid, kBlock, shm, s>>>(a, qa);
  else
    k_descent<TPR, NV, U, 1, B16, BEAMB, CAPB, CAP, MODE><<<grid, kBlock, shm, s>>>(a, qa);
}

// LDS classes: everything at most 512; k or the re-rank set above 512 with
// prototype beams of at most 512 (the per-prototype arrays stay small, so
// three workgroups fit a CU instead of one); beams above 512.
template <int TPR, int NV, int U, bool B16, int MODE = 0>
void launch2(const DescentArgs& a, const QueryArgs& qa, int need, int need_beam,
             hipStream_t s) {
  if (B16 && MODE == 0 && need <= 512) launch3<TPR, NV, U, B16, 512, 512, 2048, MODE>(a, qa, s);
  else if (need <= 512) launch3<TPR, NV, U, B16, 512, 512, 2560, MODE>(a, qa, s);
  else if (need_beam <= 512) launch3<TPR, NV, U, B16, 512, 2048, 3072, MODE>(a, qa, s);
  else launch3<TPR, NV, U, B16, 2048, 2048, 4096, MODE>(a, qa, s);
}

// The leaf-batched data layer: the (leaf, query) pairs sorted by leaf are
// cut into chunks of kQStage, one workgroup per chunk; for each run of pairs
// of one leaf in its chunk, the workgroup computes the BF16 distance of every
// row of the leaf to each of those queries, so a leaf's rows are read once
// per chunk instead of once per query, and no workgroup holds more than
// kQStage queries of a popular leaf.  The lane split (TPR lanes per row,
// 16-byte chunks gl, gl + TPR, ... with the low then the high half of each,
// then the butterfly) and the query's zero padding are those of the
// descent's BF16 row evaluation for the same row width, so every distance is
// bit for bit the descent's.  Each lane group keeps two rows in registers
// across the run's queries.
constexpr int kQStage = 32;

template <int TPR, int NV>
__global__ __launch_bounds__(kBlock) void k_leaf_scan(
    const uint16_t* __restrict__ rows_b, int ldb, const uint32_t* __restrict__ child_off1,
    int64_t n1, const uint32_t* __restrict__ pair_key, const uint32_t* __restrict__ pair_val,
    int64_t n_pairs, int cap, const uint32_t* __restrict__ leaf_off,
    const uint32_t* __restrict__ cand_off, const float* __restrict__ Q, int ldq, int dim,
    int ld, float* __restrict__ cand, unsigned long long* __restrict__ n_eval) {
  constexpr int kGroups = kBlock / TPR;
  constexpr int kRows = 2;  // rows per lane group and pass
  extern __shared__ float4 s_q4[];  // kQStage rows of ld floats
  __shared__ int64_t s_base[kQStage];
  __shared__ int64_t s_qrow[kQStage];
  __shared__ uint32_t s_leaf[kQStage];
  const int tid = threadIdx.x, grp = tid / TPR, gl = tid % TPR;
  const int64_t c0 = (int64_t)blockIdx.x * kQStage;
  const int nqs = (int)min<int64_t>(kQStage, n_pairs - c0);
  if (nqs <= 0) return;
  const int nb = ldb / 8, ld4 = ld / 4;
  float* s_q = reinterpret_cast<float*>(s_q4);
  if (tid < nqs) {
    const uint32_t v = pair_val[c0 + tid];
    const int64_t qi = v / (uint32_t)cap;
    s_qrow[tid] = qi * ldq;
    s_base[tid] = (int64_t)cand_off[qi] + leaf_off[v];
    s_leaf[tid] = pair_key[c0 + tid];
  }
  __syncthreads();
  // the chunk's queries (zero past dim, as the descent stages them), many
  // loads in flight per thread; 16-byte loads when the rows allow them
  if (dim % 4 == 0 && ldq % 4 == 0 && reinterpret_cast<uintptr_t>(Q) % 16 == 0) {
    const int d4 = dim / 4;
    const int per = (nqs * ld4 + kBlock - 1) / kBlock;
#pragma unroll 4
    for (int i = 0; i < per; ++i) {
      const int e = tid + i * kBlock;
      if (e < nqs * ld4) {
        const int qq = e / ld4, c = e - qq * ld4;
        s_q4[e] = c < d4 ? *reinterpret_cast<const float4*>(Q + s_qrow[qq] + 4 * c)
                         : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  } else {
    const int per = (nqs * ld + kBlock - 1) / kBlock;
#pragma unroll 4
    for (int i = 0; i < per; ++i) {
      const int e = tid + i * kBlock;
      if (e < nqs * ld) {
        const int qq = e / ld, c = e - qq * ld;
        s_q[e] = c < dim ? Q[s_qrow[qq] + c] : 0.f;
      }
    }
  }
  __syncthreads();
  unsigned long long evals = 0;
  for (int j0 = 0; j0 < nqs;) {
    // the run of pairs of one leaf
    const uint32_t leaf = s_leaf[j0];
    int j1 = j0 + 1;
    while (j1 < nqs && s_leaf[j1] == leaf) ++j1;
    if (leaf < n1) {
      const uint32_t b0 = child_off1[leaf], b1 = child_off1[leaf + 1];
      evals += (unsigned long long)(b1 - b0) * (unsigned long long)(j1 - j0);
      for (uint32_t r0 = b0; r0 < b1; r0 += kRows * kGroups) {
        // the chunks of the descent's class (NV per lane; chunks past the row
        // are zero on both sides there and here), widened to FP32 once for
        // all the run's queries
        float4 x[kRows][NV][2];
        bool live[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
          const uint32_t r = r0 + grp + u * kGroups;
          live[u] = r < b1;
          const uint4* row =
              reinterpret_cast<const uint4*>(rows_b + (int64_t)(live[u] ? r : b0) * ldb);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int c = gl + v * TPR;
            const uint4 t = row[c < nb ? c : 0];
            const uint4 w = c < nb ? t : make_uint4(0, 0, 0, 0);
            x[u][v][0] = bf16_lo4(make_uint2(w.x, w.y));
            x[u][v][1] = bf16_lo4(make_uint2(w.z, w.w));
          }
        }
        // every chunk of the class inside the row and the query (the usual
        // case): no selects on the query
        const bool full = NV * TPR == nb && 2 * NV * TPR <= ld4;
        // when no group of this wave has a second row in the leaf, the wave
        // evaluates one row per group
        const bool two = __any(live[1]);
        // a wave with no row of the leaf in this pass has nothing to evaluate
        const bool one = __any(live[0]);
        for (int qq = j0; one && qq < j1; ++qq) {
          const float4* qr = s_q4 + qq * ld4;
          float acc[kRows];
#pragma unroll
          for (int u = 0; u < kRows; ++u) acc[u] = 0.f;
          if (two) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int c = gl + v * TPR;
            float4 qa0, qa1;
            if (full) {
              qa0 = qr[2 * c];
              qa1 = qr[2 * c + 1];
            } else {
              const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
              const float4 t0 = qr[min(2 * c, ld4 - 1)], t1 = qr[min(2 * c + 1, ld4 - 1)];
              qa0 = 2 * c < ld4 ? t0 : z;
              qa1 = 2 * c + 1 < ld4 ? t1 : z;
            }
#pragma unroll
            for (int u = 0; u < kRows; ++u) {
              acc[u] = acc4<0>(acc[u], x[u][v][0], qa0);
              acc[u] = acc4<0>(acc[u], x[u][v][1], qa1);
            }
          }
#pragma unroll
          for (int u = 0; u < kRows; ++u) {
            acc[u] = group_sum<TPR>(acc[u]);
            if (gl == 0 && live[u]) cand[s_base[qq] + (r0 + grp + u * kGroups - b0)] = acc[u];
          }
          } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int c = gl + v * TPR;
            float4 qa0, qa1;
            if (full) {
              qa0 = qr[2 * c];
              qa1 = qr[2 * c + 1];
            } else {
              const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
              const float4 t0 = qr[min(2 * c, ld4 - 1)], t1 = qr[min(2 * c + 1, ld4 - 1)];
              qa0 = 2 * c < ld4 ? t0 : z;
              qa1 = 2 * c + 1 < ld4 ? t1 : z;
            }
            acc[0] = acc4<0>(acc[0], x[0][v][0], qa0);
            acc[0] = acc4<0>(acc[0], x[0][v][1], qa1);
          }
          acc[0] = group_sum<TPR>(acc[0]);
          if (gl == 0 && live[0]) cand[s_base[qq] + (r0 + grp - b0)] = acc[0];
          }
        }
      }
    }
    j0 = j1;
  }
  if (n_eval && tid == 0) atomicAdd(n_eval + blockIdx.x % kCounterShards, evals);
}

// The data layer of the leaf-batched descent with one wave per query (four
// queries per workgroup, no workgroup barriers).  The query's candidates
// (the BF16 distances of its kept leaves' rows, in the order of its kept
// leaves) stream through a buffer of kSelBuf keys in the wave's LDS that
// takes only keys below the current threshold; whenever the buffer runs
// short of room, a bitwise radix selection keeps the W smallest and lowers
// the threshold.  The re-rank set then gets its FP32 distances with the lane
// split and butterfly of the descent's class, and the k nearest are written
// in order.  Keys (distance bits, id) are distinct, so every selected set,
// and with it the result, is the one the workgroup-per-query data layer
// takes.  When the re-rank set would hold every candidate (or is not larger
// than k) the FP32 distances of all candidates are ranked instead, as there.
constexpr int kSelBuf = 512;     // keys per wave
constexpr int kSelMax = 192;     // largest re-rank set and k
constexpr int kSelLeaves = 128;  // largest level-1 beam
constexpr int kSelWaves = kBlock / kWave;

// lanes below this one whose bit is set in mask
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Orders the wave's LDS accesses: LDS operations of one wave complete in
// order; the fences keep the compiler from moving accesses across.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int o) {
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
  return ((uint64_t)hi << 32) | lo;
}

template <bool MAX>
__device__ inline uint64_t wave_reduce_u64(uint64_t v) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const uint64_t w = shfl_xor_u64(v, o);
    v = MAX ? (w > v ? w : v) : (w < v ? w : v);
  }
  return v;
}

// Keeps the w smallest of the n keys at buf[0, n) (2 <= n <= kSelBuf,
// 1 <= w < n, keys distinct) at buf[0, w), in no particular order, and
// returns the largest of them.  Every lane of the wave calls it with the same
// arguments.  The w-th smallest key is found bit by bit from the highest bit
// in which the keys differ; the search stops as soon as the keys sharing the
// bits found so far are exactly the ones still needed.
__device__ uint64_t wave_keep_smallest(uint64_t* buf, uint32_t n, uint32_t w, int lane) {
  constexpr int P = kSelBuf / kWave;
  uint64_t key[P];
  bool ok[P];
  uint64_t kmin = ~0ull, kmax = 0;
  wave_sync();
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint32_t i = lane + j * kWave;
    ok[j] = i < n;
    key[j] = 0;
    if (ok[j]) {
      key[j] = buf[i];
      kmin = key[j] < kmin ? key[j] : kmin;
      kmax = key[j] > kmax ? key[j] : kmax;
    }
  }
  kmin = wave_reduce_u64<false>(kmin);
  kmax = wave_reduce_u64<true>(kmax);
  const int np = (int)((n + kWave - 1) / kWave);
  // the highest bit in which the keys differ; bits above it are common
  int b = kmin == kmax ? 0 : 63 - __clzll((long long)(kmin ^ kmax));
  uint64_t prefix = kmin == kmax ? kmin : b >= 63 ? 0ull : (kmin >> (b + 1)) << (b + 1);
  uint32_t need = w, in_s = kmin == kmax ? w : n;  // keys sharing the prefix's bits above b
  for (; b > 0; --b) {
    const uint64_t hi = prefix >> b;  // bit b clear
    uint32_t c0 = 0;
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (j < np) c0 += (uint32_t)__popcll(__ballot(ok[j] && (key[j] >> b) == hi));
    if (c0 >= need) {
      in_s = c0;
    } else {
      need -= c0;
      in_s -= c0;
      prefix |= 1ull << b;
    }
    if (in_s == need) break;
  }
  // kept: the keys whose bits at and above b do not exceed the prefix's
  // (exactly w of them; at b = 0 the w-th smallest key itself bounds them)
  if (b == 0 && in_s != need) {
    uint32_t c0 = 0;
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (j < np) c0 += (uint32_t)__popcll(__ballot(ok[j] && key[j] == prefix));
    if (c0 < need) prefix |= 1ull;
  }
  const uint64_t lim = prefix >> b;
  uint32_t base = 0;
  uint64_t top = 0;
  wave_sync();
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (j < np) {
      const bool sel = ok[j] && (key[j] >> b) <= lim;
      const uint64_t m = __ballot(sel);
      const uint32_t slot = base + lanes_below(m);
      if (sel && slot < w) {
        buf[slot] = key[j];
        top = key[j] > top ? key[j] : top;
      }
      base += (uint32_t)__popcll(m);
    }
  }
  wave_sync();
  return wave_reduce_u64<true>(top);
}

template <int TPR>
__global__ __launch_bounds__(kBlock) void k_leaf_select(DescentArgs a, QueryArgs qa,
                                                        int rerank) {
  __shared__ uint64_t s_buf[kSelWaves][kSelBuf];
  __shared__ float4 s_q4w[kSelWaves][kMaxBatchedLd / 4];
  __shared__ uint32_t s_b0[kSelWaves][kSelLeaves + 1];
  __shared__ uint32_t s_lo[kSelWaves][kSelLeaves + 1];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  // queries in launch order; each XCD takes a contiguous run of workgroups
  const int64_t n_wg = (qa.nq + kSelWaves - 1) / kSelWaves;
  const int64_t per_xcd = (n_wg + kXcds - 1) / kXcds;
  const int64_t run = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  const int64_t pos = run * kSelWaves + wv;
  if (run >= n_wg || pos >= qa.nq) return;  // the whole wave
  const int64_t qi = qa.order ? (int64_t)qa.order[pos] : pos;
  uint64_t* buf = s_buf[wv];
  float4* sq4 = s_q4w[wv];
  float* sq = reinterpret_cast<float*>(sq4);
  uint32_t* sb0 = s_b0[wv];
  uint32_t* slo = s_lo[wv];
  const int ld = a.ld, ld4 = ld / 4;
  const int k = qa.k;
  const int64_t obase = qi * (int64_t)k;
  for (int c = lane; c < ld; c += kWave) sq[c] = c < a.dim ? qa.Q[qi * qa.ldq + c] : 0.f;
  const int64_t lb = qi * (int64_t)qa.leaf_cap;
  const int nk = min((int)qa.n_kept[qi], qa.leaf_cap);
  for (int j = lane; j < nk; j += kWave) {
    sb0[j] = qa.leaf_b0[lb + j];
    slo[j] = qa.leaf_off[lb + j];
  }
  const uint32_t m = nk > 0 ? qa.leaf_off[lb + nk - 1] + qa.leaf_cnt[lb + nk - 1] : 0u;
  if (lane == 0) slo[nk] = m;
  wave_sync();
  const LevelView V = a.lv[0];
  const bool low = (int64_t)m > rerank && rerank > k;
  const uint32_t want = low ? (uint32_t)rerank : (uint32_t)k;
  const int grp = lane / TPR, gl = lane % TPR;
  constexpr int kGroups = kWave / TPR;
  uint64_t thr = ~0ull;
  uint32_t cnt = 0;
  int lo = 0;  // this lane's leaf (candidates are walked forward)
  // the first candidate of the next leaf, and position - candidate index in
  // this one (modulo 2^32)
  uint32_t nxt = nk > 1 ? slo[1] : UINT32_MAX;
  uint32_t shift = nk > 0 ? sb0[0] - slo[0] : 0u;
  if (low) {
    // the BF16 distances the leaf scan wrote: four candidates per lane and step
    const int64_t cbase = (int64_t)qa.cand_off[qi];
    for (uint32_t base = 0; base < m; base += 4 * kWave) {
      if (cnt > kSelBuf - 4 * kWave) {
        thr = wave_keep_smallest(buf, cnt, want, lane);
        cnt = want;
      }
      uint32_t idx[4];
      int64_t p[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        idx[u] = base + lane + u * kWave;
        const uint32_t ic = idx[u] < m ? idx[u] : m - 1;
        while (ic >= nxt) {
          ++lo;
          shift = sb0[lo] - slo[lo];
          nxt = lo + 1 < nk ? slo[lo + 1] : UINT32_MAX;
        }
        p[u] = (int64_t)(uint32_t)(shift + ic);
      }
      float dv[4];
      int32_t id[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        dv[u] = qa.cand[cbase + (idx[u] < m ? idx[u] : m - 1)];
        id[u] = V.orig[p[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t key = ((uint64_t)__float_as_uint(dv[u]) << 32) | (uint32_t)id[u];
        const bool pass = idx[u] < m && key < thr;
        const uint64_t mk = __ballot(pass);
        if (pass) buf[cnt + lanes_below(mk)] = key;
        cnt += (uint32_t)__popcll(mk);
      }
    }
  } else {
    // FP32 distances of every candidate row
    for (uint32_t base = 0; base < m; base += kGroups) {
      if (cnt > kSelBuf - kGroups) {
        thr = wave_keep_smallest(buf, cnt, want, lane);
        cnt = want;
      }
      const uint32_t idx = base + grp;
      const uint32_t ic = idx < m ? idx : m - 1;
      while (ic >= nxt) {
        ++lo;
        shift = sb0[lo] - slo[lo];
        nxt = lo + 1 < nk ? slo[lo + 1] : UINT32_MAX;
      }
      const int64_t p = (int64_t)(uint32_t)(shift + ic);
      const float4* row = reinterpret_cast<const float4*>(V.protos + p * ld);
      float s0 = 0.f;
      for (int c4 = gl; c4 < ld4; c4 += TPR) s0 = acc4<0>(s0, row[c4], sq4[c4]);
      s0 = group_sum<TPR>(s0);
      const uint64_t key = ((uint64_t)__float_as_uint(s0) << 32) | (uint32_t)V.orig[p];
      const bool pass = gl == 0 && idx < m && key < thr;
      const uint64_t mk = __ballot(pass);
      if (pass) buf[cnt + lanes_below(mk)] = key;
      cnt += (uint32_t)__popcll(mk);
    }
    if (qa.rows && lane == 0) atomicAdd(qa.rows + blockIdx.x % kCounterShards, (unsigned long long)m);
  }
  wave_sync();
  if (cnt > want) {
    thr = wave_keep_smallest(buf, cnt, want, lane);
    cnt = want;
  }
  uint64_t* fin = buf;
  if (low) {
    // FP32 direct form on the FP32 rows of the re-rank set (at buf[cnt, 2 cnt))
    for (uint32_t j0 = 0; j0 < cnt; j0 += kGroups) {
      const uint32_t j = j0 + grp;
      const uint32_t id = (uint32_t)buf[j < cnt ? j : 0];
      const int64_t p = a.inv0[id];
      const float4* row = reinterpret_cast<const float4*>(V.protos + p * ld);
      float s0 = 0.f;
      for (int c4 = gl; c4 < ld4; c4 += TPR) s0 = acc4<0>(s0, row[c4], sq4[c4]);
      s0 = group_sum<TPR>(s0);
      if (gl == 0 && j < cnt) buf[cnt + j] = ((uint64_t)__float_as_uint(s0) << 32) | id;
    }
    wave_sync();
    fin = buf + cnt;
    if (cnt > (uint32_t)k) {
      wave_keep_smallest(fin, cnt, (uint32_t)k, lane);
      cnt = (uint32_t)k;
    }
  }
  // rank the kept keys and write the result row
  const uint32_t kept = cnt < (uint32_t)k ? cnt : (uint32_t)k;
  for (uint32_t j = lane; j < (uint32_t)k; j += kWave) {
    if (j < kept) {
      const uint64_t v = fin[j];
      uint32_t rank = 0;
      for (uint32_t t = 0; t < kept; ++t) rank += fin[t] < v;
      qa.out_ids[obase + rank] = (int32_t)(uint32_t)v;
      qa.out_dist[obase + rank] = sqrtf(__uint_as_float((uint32_t)(v >> 32)));
    } else {
      qa.out_ids[obase + j] = -1;
      qa.out_dist[obase + j] = INFINITY;
    }
  }
}

// The prototype levels of the leaf-batched descent with one wave per query
// (four per workgroup, no workgroup barriers).  At each level the children
// of the kept prototypes stream through the wave's key buffer -- a screened
// level's keys from the batch's scores, another level's from its BF16 rows
// with the lane split and arithmetic of the descent's class -- and the
// beam's nearest are kept; after level 1 the kept leaves are written for the
// leaf scan.  Keys are distinct, so every kept set equals the
// workgroup-per-query descent's; only the slot order may differ.
constexpr int kSelSlots = (kSelMax + kWave - 1) / kWave;  // kept slots per lane

template <int TPR, int NV>
__global__ __launch_bounds__(kBlock) void k_level_select(DescentArgs a, QueryArgs qa) {
  __shared__ uint64_t s_buf[kSelWaves][kSelBuf];
  __shared__ float4 s_q4w[kSelWaves][kMaxBatchedLd / 4];
  __shared__ uint32_t s_b0[kSelWaves][kSelMax + 1];
  __shared__ uint32_t s_lo[kSelWaves][kSelMax + 1];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int64_t n_wg = (qa.nq + kSelWaves - 1) / kSelWaves;
  const int64_t per_xcd = (n_wg + kXcds - 1) / kXcds;
  const int64_t run = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  const int64_t pos = run * kSelWaves + wv;
  if (run >= n_wg || pos >= qa.nq) return;  // the whole wave
  const int64_t qi = qa.order ? (int64_t)qa.order[pos] : pos;
  uint64_t* buf = s_buf[wv];
  float4* sq4 = s_q4w[wv];
  float* sq = reinterpret_cast<float*>(sq4);
  uint32_t* sb0 = s_b0[wv];
  uint32_t* slo = s_lo[wv];
  const int ld = a.ld, ld4 = ld / 4, ldb = a.ldb, nb = ldb / 8;
  const int L = a.n_levels;
  for (int c = lane; c < ld; c += kWave) sq[c] = c < a.dim ? qa.Q[qi * qa.ldq + c] : 0.f;
  if (lane == 0) {
    sb0[0] = 0;
    slo[0] = 0;
    slo[1] = (uint32_t)a.lv[L].n;
  }
  wave_sync();
  const int grp = lane / TPR, gl = lane % TPR;
  constexpr int kGroups = kWave / TPR;
  float4 qv[NV][2];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int c = gl + v * TPR;
    qv[v][0] = make_float4(0.f, 0.f, 0.f, 0.f);
    qv[v][1] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (2 * c < ld4) qv[v][0] = sq4[2 * c];
    if (2 * c + 1 < ld4) qv[v][1] = sq4[2 * c + 1];
  }
  unsigned long long rows_seen = 0;
  int n_par = 1;
  for (int lev = L; lev >= 1; --lev) {
    const LevelView V = a.lv[lev];
    const float* scr = qa.scr[lev];
    const int64_t sbase = qi * qa.scr_ld[lev];
    const uint32_t m = slo[n_par];
    const uint32_t want = (uint32_t)qa.r_lev[lev];
    uint64_t thr = ~0ull;
    uint32_t cnt = 0;
    int lo = 0;  // this lane's parent (candidates are walked forward)
    // the first candidate of the next parent, and position - candidate index
    // in this one (modulo 2^32)
    uint32_t nxt = n_par > 1 ? slo[1] : UINT32_MAX;
    uint32_t shift = sb0[0] - slo[0];
    if (scr != nullptr) {
      for (uint32_t base = 0; base < m; base += 4 * kWave) {
        if (cnt > kSelBuf - 4 * kWave) {
          thr = wave_keep_smallest(buf, cnt, want, lane);
          cnt = want;
        }
        uint32_t idx[4];
        int64_t p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          idx[u] = base + lane + u * kWave;
          const uint32_t ic = idx[u] < m ? idx[u] : m - 1;
          while (ic >= nxt) {
            ++lo;
            shift = sb0[lo] - slo[lo];
            nxt = lo + 1 < n_par ? slo[lo + 1] : UINT32_MAX;
          }
          p[u] = (int64_t)(uint32_t)(shift + ic);
        }
        float dv[4];
        int32_t id[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          dv[u] = scr[sbase + p[u]];
          id[u] = V.orig[p[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint64_t key = ((uint64_t)__float_as_uint(dv[u]) << 32) | (uint32_t)id[u];
          const bool pass = idx[u] < m && key < thr;
          const uint64_t mk = __ballot(pass);
          if (pass) buf[cnt + lanes_below(mk)] = key;
          cnt += (uint32_t)__popcll(mk);
        }
      }
    } else {
      rows_seen += m;
      for (uint32_t base = 0; base < m; base += kGroups) {
        if (cnt > kSelBuf - kGroups) {
          thr = wave_keep_smallest(buf, cnt, want, lane);
          cnt = want;
        }
        const uint32_t idx = base + grp;
        const uint32_t ic = idx < m ? idx : m - 1;
        while (ic >= nxt) {
          ++lo;
          shift = sb0[lo] - slo[lo];
          nxt = lo + 1 < n_par ? slo[lo + 1] : UINT32_MAX;
        }
        const int64_t p = (int64_t)(uint32_t)(shift + ic);
        const uint4* row = reinterpret_cast<const uint4*>(V.protos_b + p * ldb);
        uint4 x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int c = gl + v * TPR;
          const uint4 t = row[c < nb ? c : 0];
          x[v] = c < nb ? t : make_uint4(0, 0, 0, 0);
        }
        const int32_t id = V.orig[p];
        float s0 = 0.f;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          s0 = acc4<0>(s0, bf16_lo4(make_uint2(x[v].x, x[v].y)), qv[v][0]);
          s0 = acc4<0>(s0, bf16_lo4(make_uint2(x[v].z, x[v].w)), qv[v][1]);
        }
        s0 = group_sum<TPR>(s0);
        const uint64_t key = ((uint64_t)__float_as_uint(s0) << 32) | (uint32_t)id;
        const bool pass = gl == 0 && idx < m && key < thr;
        const uint64_t mk = __ballot(pass);
        if (pass) buf[cnt + lanes_below(mk)] = key;
        cnt += (uint32_t)__popcll(mk);
      }
    }
    wave_sync();
    if (cnt > want) {
      wave_keep_smallest(buf, cnt, want, lane);
      cnt = want;
    }
    const uint32_t kept = cnt;
    if (qa.sel) {
      int32_t* so = qa.sel + ((int64_t)qi * L + (L - lev)) * qa.r;
      for (int j = lane; j < qa.r; j += kWave)
        so[j] = (uint32_t)j < kept ? (int32_t)(uint32_t)buf[j] : -1;
    }
    // the kept prototypes' children: counts, first positions, prefix
    uint32_t c[kSelSlots], b0v[kSelSlots], pv[kSelSlots], off[kSelSlots], sum = 0;
#pragma unroll
    for (int t = 0; t < kSelSlots; ++t) {
      const uint32_t e = lane * kSelSlots + t;
      c[t] = 0;
      b0v[t] = 0;
      pv[t] = (uint32_t)V.n;
      if (e < kept) {
        const int32_t q = V.inv[(uint32_t)buf[e]];
        b0v[t] = V.child_off[q];
        c[t] = V.child_off[q + 1] - b0v[t];
        pv[t] = (uint32_t)q;
      }
      sum += c[t];
    }
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    const uint32_t total = __shfl(x, kWave - 1);
    uint32_t acc = x - sum;
#pragma unroll
    for (int t = 0; t < kSelSlots; ++t) {
      off[t] = acc;
      acc += c[t];
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < kSelSlots; ++t) {
      const uint32_t e = lane * kSelSlots + t;
      if (e < kept) {
        sb0[e] = b0v[t];
        slo[e] = off[t];
      }
    }
    if (lane == 0) {
      if (kept > 0) {
        slo[kept] = total;
      } else {  // one empty range
        sb0[0] = 0;
        slo[0] = 0;
        slo[1] = 0;
      }
    }
    n_par = kept > 0 ? (int)kept : 1;
    wave_sync();
    if (lev == 1) {
      // the kept leaves for the leaf-by-leaf data layer
      const int64_t lb = qi * (int64_t)qa.leaf_cap;
#pragma unroll
      for (int t = 0; t < kSelSlots; ++t) {
        const uint32_t e = lane * kSelSlots + t;
        if (e < (uint32_t)qa.leaf_cap) {
          const bool in = e < kept;
          qa.leaf_b0[lb + e] = in ? b0v[t] : 0u;
          qa.leaf_cnt[lb + e] = in ? c[t] : 0u;
          qa.leaf_off[lb + e] = in ? off[t] : 0u;
          qa.leaf_key[lb + e] = in && c[t] > 0 ? pv[t] : (uint32_t)V.n;
          qa.leaf_val[lb + e] = (uint32_t)(lb + e);
        }
      }
      if (lane == 0) {
        qa.n_kept[qi] = kept;
        qa.n_cand[qi] = kept > 0 ? total : 0u;
        if (qa.rows) atomicAdd(qa.rows + blockIdx.x % kCounterShards, rows_seen);
      }
    }
  }
}

}  // namespace

typedef __bf16 sbf16x8 __attribute__((ext_vector_type(8)));
typedef float sfloatx16 __attribute__((ext_vector_type(16)));

__device__ inline uint32_t bf16_rne_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// A workgroup scores 128 queries (32 per wave) against kScoreTiles tiles of
// 32 prototypes: each tile is staged once in LDS (rows padded by 16 bytes)
// and read by all four waves, and every wave keeps its 32 queries' MFMA
// fragments in registers across the tiles.  MFMA k-slot (s, h, e) is
// dimension 16 s + 8 h + e: lane l feeds query row l % 32 (as q = hi + lo,
// two BF16 terms) and prototype row l % 32, 8 consecutive dimensions each;
// output register i of lane l is query 8 (i / 4) + 4 (l / 32) + i % 4,
// prototype l % 32.
constexpr int kScoreTiles = 16;
constexpr int kScoreLdsRow = 256 + 8;  // BF16 per staged row (dense dims <= 256)

template <int KS, bool V4>
__global__ __launch_bounds__(kBlock) void k_level_scores(
    const float* __restrict__ Q, int ldq, int64_t nq, int dim, const uint16_t* __restrict__ P,
    int ldb, int64_t n, const float* __restrict__ pn, float* __restrict__ S, int64_t ldS) {
  __shared__ uint4 s_b4[32 * kScoreLdsRow / 8];
  uint16_t* s_b = reinterpret_cast<uint16_t*>(s_b4);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t q0 = (int64_t)blockIdx.y * 128 + 32 * wave;
  const int64_t pb = (int64_t)blockIdx.x * 32 * kScoreTiles;
  const int r = lane % 32, h = lane / 32;
  const int row_ld = ldb + 8;  // staged row stride (BF16)
  const bool qok = q0 + r < nq;
  const float* qrow = Q + (qok ? q0 + r : 0) * (int64_t)ldq;
  sbf16x8 a_hi[KS], a_lo[KS];
  float qsq = 0.f;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int kk = 16 * ks + 8 * h;
    uint32_t hw[4], lw[4];
    float v[8];
    if constexpr (V4) {  // rows 16-byte aligned, dim a multiple of 8
      const bool in = qok && kk < dim;
      const float4 x0 = in ? *reinterpret_cast<const float4*>(qrow + kk) : make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 x1 = in ? *reinterpret_cast<const float4*>(qrow + kk + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
      v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
      v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (qok && kk + e < dim) ? qrow[kk + e] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float v0 = v[2 * e], v1 = v[2 * e + 1];
      qsq = fmaf(v0, v0, qsq);
      qsq = fmaf(v1, v1, qsq);
      const uint32_t h0 = bf16_rne_bits(v0), h1 = bf16_rne_bits(v1);
      const uint32_t l0 = bf16_rne_bits(v0 - __uint_as_float(h0 << 16));
      const uint32_t l1 = bf16_rne_bits(v1 - __uint_as_float(h1 << 16));
      hw[e] = h0 | (h1 << 16);
      lw[e] = l0 | (l1 << 16);
    }
    __builtin_memcpy(&a_hi[ks], hw, sizeof(sbf16x8));
    __builtin_memcpy(&a_lo[ks], lw, sizeof(sbf16x8));
  }
  qsq += __shfl_xor(qsq, 32);  // the two halves hold disjoint dimensions of row r
  // |q|^2 of the 16 output rows of this lane, and their offsets in S
  float qn_row[16];
  int64_t so_row[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = 8 * (i / 4) + 4 * h + (i % 4);
    qn_row[i] = __shfl(qsq, row);
    so_row[i] = (q0 + row) * ldS;
  }
  const int c8 = ldb / 8;      // 16-byte chunks per prototype row
  for (int t = 0; t < kScoreTiles; ++t) {
    const int64_t p0 = pb + 32 * t;
    if (p0 >= n) break;  // uniform across the workgroup
    __syncthreads();     // the previous tile is no longer read
    for (int c = threadIdx.x; c < 32 * c8; c += kBlock) {
      const int row = c / c8, col = c % c8;
      const uint4 v = p0 + row < n
                          ? *reinterpret_cast<const uint4*>(P + (p0 + row) * (int64_t)ldb + 8 * col)
                          : make_uint4(0u, 0u, 0u, 0u);
      *reinterpret_cast<uint4*>(s_b + row * row_ld + 8 * col) = v;
    }
    __syncthreads();
    sfloatx16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kk = 16 * ks + 8 * h;
      const uint4 bv = kk < ldb ? *reinterpret_cast<const uint4*>(s_b + r * row_ld + kk)
                                : make_uint4(0u, 0u, 0u, 0u);
      sbf16x8 b;
      __builtin_memcpy(&b, &bv, sizeof(b));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi[ks], b, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_lo[ks], b, acc, 0, 0, 0);
    }
    const int64_t pp = p0 + r;
    const float pnp = pp < n ? pn[pp] : 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 8 * (i / 4) + 4 * h + (i % 4);
      if (q0 + row < nq && pp < n) S[so_row[i] + pp] = fmaxf(0.f, qn_row[i] + pnp - 2.f * acc[i]);
    }
  }
}

void level_scores(const float* Q, int ldq, int64_t nq, int dim, const uint16_t* protos_b,
                  int ldb, int64_t n, const float* pn, float* S, int64_t ldS, hipStream_t s) {
  if (nq <= 0 || n <= 0) return;
  ScopedTiming timing("level_scores", s);
  MASK_CHECK(ldb <= 256, "level_scores: rows above 256 dimensions");
  const int64_t per_block = 32 * kScoreTiles;
  const dim3 grid((unsigned)((n + per_block - 1) / per_block), (unsigned)((nq + 127) / 128));
  const int ks = (ldb + 15) / 16;
  const bool v4 = dim % 8 == 0 && ldq % 4 == 0 && reinterpret_cast<uintptr_t>(Q) % 16 == 0;
#define MASK_SCORES(K)                                                                     \
  (v4 ? k_level_scores<K, true><<<grid, kBlock, 0, s>>>(Q, ldq, nq, dim, protos_b, ldb, n, pn, S, ldS) \
      : k_level_scores<K, false><<<grid, kBlock, 0, s>>>(Q, ldq, nq, dim, protos_b, ldb, n, pn, S, ldS))
  if (ks <= 1) MASK_SCORES(1);
  else if (ks <= 2) MASK_SCORES(2);
  else if (ks <= 4) MASK_SCORES(4);
  else if (ks <= 6) MASK_SCORES(6);
  else if (ks <= 8) MASK_SCORES(8);
  else if (ks <= 12) MASK_SCORES(12);
  else MASK_SCORES(16);
#undef MASK_SCORES
  check_launch("level_scores");
}

// The smallest score of row[lo .. hi) and its position (the lowest on
// ties), by one wave.
__device__ inline int64_t wave_argmin(const float* __restrict__ row, int64_t lo, int64_t hi,
                                      int lane) {
  float best = INFINITY;
  int64_t at = hi;
  for (int64_t p = lo + lane; p < hi; p += kWave) {
    const float v = row[p];
    if (v < best) {
      best = v;
      at = p;
    }
  }
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const float ob = __shfl_xor(best, o);
    const int64_t oa = __shfl_xor(at, o);
    if (ob < best || (ob == best && oa < at)) {
      best = ob;
      at = oa;
    }
  }
  return at < hi ? at : lo;
}

// Key of every query: the greedy path through the screened levels (the
// nearest prototype of the top level, then the nearest of its children, down
// to the lowest screened level), by its scores; one wave per query.
__global__ __launch_bounds__(kBlock) void k_greedy_key(ScreenPath sp, int64_t nq,
                                                       uint32_t* __restrict__ keys) {
  const int lane = threadIdx.x % kWave;
  const int64_t q = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (q >= nq) return;  // uniform across the wave
  int64_t p = wave_argmin(sp.S[sp.top] + q * sp.ld[sp.top], 0, sp.n_top, lane);
  for (int l = sp.top - 1; l >= sp.low; --l) {
    const int64_t lo = sp.child_off[l + 1][p], hi = sp.child_off[l + 1][p + 1];
    p = hi > lo ? wave_argmin(sp.S[l] + q * sp.ld[l], lo, hi, lane) : lo;
  }
  if (lane == 0) keys[q] = (uint32_t)p;
}

// Counting sort of the queries by key (< n <= 16384) in one workgroup: an
// LDS histogram, its exclusive scan, then every query takes the next slot of
// its key.  The order within a key is not fixed; the descent's results do
// not depend on it.
constexpr int kOrderBlock = 1024;
__global__ __launch_bounds__(kOrderBlock) void k_order_by_key(const uint32_t* __restrict__ keys,
                                                              int64_t nq, int n,
                                                              uint32_t* __restrict__ order) {
  __shared__ uint32_t s_cnt[16384];
  __shared__ uint32_t s_part[kOrderBlock];
  const int tid = threadIdx.x;
  for (int j = tid; j < n; j += kOrderBlock) s_cnt[j] = 0;
  __syncthreads();
  for (int64_t q = tid; q < nq; q += kOrderBlock) atomicAdd(&s_cnt[min(keys[q], (uint32_t)n - 1)], 1u);
  __syncthreads();
  // exclusive scan: thread t owns keys [t * per, (t + 1) * per)
  const int per = (n + kOrderBlock - 1) / kOrderBlock;
  uint32_t sum = 0;
  for (int j = tid * per; j < min(n, (tid + 1) * per); ++j) sum += s_cnt[j];
  s_part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < kOrderBlock; o <<= 1) {
    const uint32_t v = tid >= o ? s_part[tid - o] : 0u;
    __syncthreads();
    s_part[tid] += v;
    __syncthreads();
  }
  uint32_t run = s_part[tid] - sum;
  for (int j = tid * per; j < min(n, (tid + 1) * per); ++j) {
    const uint32_t c = s_cnt[j];
    s_cnt[j] = run;
    run += c;
  }
  __syncthreads();
  for (int64_t q = tid; q < nq; q += kOrderBlock)
    order[atomicAdd(&s_cnt[min(keys[q], (uint32_t)n - 1)], 1u)] = (uint32_t)q;
}

void order_queries(const ScreenPath& sp, int64_t nq, uint32_t* keys, uint32_t* order,
                   hipStream_t s) {
  if (nq <= 0) return;
  const int64_t n_low = sp.n_low;
  MASK_CHECK(n_low >= 1 && n_low <= 16384, "order_queries: level above 16384 prototypes");
  ScopedTiming timing("order_queries", s);
  k_greedy_key<<<(unsigned)((nq * kWave + kBlock - 1) / kBlock), kBlock, 0, s>>>(sp, nq, keys);
  k_order_by_key<<<1, kOrderBlock, 0, s>>>(keys, nq, (int)n_low, order);
  check_launch("order_queries");
}

// One wave per query: lanes stride over the data rows of the leaf and
// compare every coordinate; the wave keeps the lowest matching row id.
__global__ __launch_bounds__(kBlock) void k_point_match(
    const float* __restrict__ Q, int ldq, int64_t nq, int dim, const float* __restrict__ rows,
    int ld, const int32_t* __restrict__ orig0, const int32_t* __restrict__ inv1,
    const uint32_t* __restrict__ child_off1, const int32_t* __restrict__ leaf,
    int32_t* __restrict__ match) {
  const int lane = threadIdx.x % kWave;
  const int64_t qi = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (qi >= nq) return;  // uniform across the wave
  const int32_t p = leaf[qi];
  int32_t best = INT32_MAX;
  if (p >= 0) {
    const int32_t pos = inv1[p];
    const uint32_t b0 = child_off1[pos], b1 = child_off1[pos + 1];
    const float* q = Q + qi * ldq;
    for (uint32_t c = b0 + lane; c < b1; c += kWave) {
      const float* x = rows + (int64_t)c * ld;
      bool eq = true;
      for (int d = 0; d < dim && eq; ++d) eq = x[d] == q[d];
      if (eq) best = min(best, orig0[c]);
    }
  }
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) best = min(best, __shfl_xor(best, o));
  if (lane == 0) match[qi] = best == INT32_MAX ? -1 : best;
}

void point_match(const DescentArgs& a, const float* Q, int ldq, int64_t nq,
                 const int32_t* leaf, int32_t* match, hipStream_t s) {
  if (nq <= 0) return;
  ScopedTiming timing("point_match", s);
  k_point_match<<<(unsigned)((nq * kWave + kBlock - 1) / kBlock), kBlock, 0, s>>>(
      Q, ldq, nq, a.dim, a.lv[0].protos, a.ld, a.lv[0].orig, a.lv[1].inv, a.lv[1].child_off,
      leaf, match);
  check_launch("point_match");
}

void descent(const DescentArgs& a, const QueryArgs& qa, hipStream_t s) {
  if (qa.nq <= 0) return;
  ScopedTiming timing(a.sparse ? "descent_csr"
                               : (a.precision == MASK_BF16       ? "descent_bf16"
                                  : a.precision == MASK_FP8_E4M3 ? "descent_fp8"
                                                                 : "descent"),
                      s);
  const bool b16 = a.precision == MASK_BF16;
  // LDS class from the beams and k; the BF16 re-rank set fits the class
  int need_beam = qa.r;  // the largest prototype beam of the launch
  int r1 = qa.r;         // the largest level-1 beam of the launch
  for (int l = 1; l <= a.n_levels; ++l) {
    const int pb = qa.r_lev[l] > 0   ? qa.r_lev[l]
                   : qa.beam_e8[l] > 0 ? (qa.r * qa.beam_e8[l] + 7) / 8  // the profile's largest
                                       : qa.r;
    need_beam = pb > need_beam ? pb : need_beam;
    if (l == 1) r1 = pb;
  }
  int need = qa.k > need_beam ? qa.k : need_beam;
  if (a.precision != MASK_FP32 && !a.sparse) {
    // the largest re-rank set of the launch (kMaxBeam at most)
    const int64_t R = a.rerank_factor > 0 ? (int64_t)a.rerank_factor * qa.k
                                          : (int64_t)(-a.rerank_factor) * qa.k * r1;
    need = (int)std::max<int64_t>(need, std::min<int64_t>(R, kMaxBeam));
  }
  if (a.sparse) {
    // beams above 2048 (the library admits them for at most 12,288 columns:
    // 103 KB of static LDS beside the dense query vector)
    if (need > kMaxBeam) launch3<16, 0, 4, false, kMaxBeamCsr, kMaxBeamCsr, 4096, 1>(a, qa, s);
    else launch2<16, 0, 4, false, 1>(a, qa, need, need_beam, s);
    check_launch("descent_csr");
    return;
  }
  if (a.precision == MASK_FP8_E4M3) {
    const int nc = a.ldq / 16;
    if (nc <= 2) launch2<2, 0, 2, false, 2>(a, qa, need, need_beam, s);
    else if (nc <= 4) launch2<4, 0, 2, false, 2>(a, qa, need, need_beam, s);
    else if (nc <= 8) launch2<8, 0, 2, false, 2>(a, qa, need, need_beam, s);
    else launch2<16, 0, 2, false, 2>(a, qa, need, need_beam, s);
    check_launch("descent_fp8");
    return;
  }
  // Lane groups per row width, measured on MI355X (1M-point mixtures, beams
  // 16/96/160): few lanes per row, each with several 16-byte vectors, and one
  // or two rows in flight per group beat wide groups -- more rows per wave
  // means more independent loads in flight and less per-row bookkeeping.
  if (!b16) {
    const int f4 = a.ld / 4;
    if (f4 <= 1) launch2<1, 1, 4, false>(a, qa, need, need_beam, s);
    else if (f4 <= 2) launch2<1, 2, 2, false>(a, qa, need, need_beam, s);
    else if (f4 <= 4) launch2<1, 4, 1, false>(a, qa, need, need_beam, s);
    else if (f4 <= 8) launch2<2, 4, 2, false>(a, qa, need, need_beam, s);
    else if (f4 <= 16) launch2<4, 4, 2, false>(a, qa, need, need_beam, s);
    else if (f4 <= 32) launch2<8, 4, 2, false>(a, qa, need, need_beam, s);
    else if (f4 <= 64) launch2<8, 8, 1, false>(a, qa, need, need_beam, s);
    else launch2<16, 0, 1, false>(a, qa, need, need_beam, s);
  } else {
    const int c8 = a.ldb / 8;
    if (c8 <= 1) launch2<1, 1, 4, true>(a, qa, need, need_beam, s);
    else if (c8 <= 2) launch2<1, 2, 2, true>(a, qa, need, need_beam, s);
    else if (c8 <= 4) launch2<1, 4, 1, true>(a, qa, need, need_beam, s);
    else if (c8 <= 8) launch2<2, 4, 1, true>(a, qa, need, need_beam, s);
    else if (c8 <= 12) launch2<4, 3, 1, true>(a, qa, need, need_beam, s);
    else if (c8 <= 16) launch2<4, 4, 1, true>(a, qa, need, need_beam, s);
    else if (c8 <= 32) launch2<8, 4, 1, true>(a, qa, need, need_beam, s);
    else launch2<16, 0, 1, true>(a, qa, need, need_beam, s);
  }
  check_launch("descent");
}

void leaf_scan(const DescentArgs& a, const uint32_t* pair_key, const uint32_t* pair_val,
               int64_t n_pairs, int cap, const uint32_t* leaf_off, const uint32_t* cand_off,
               const float* Q, int ldq, float* cand, hipStream_t s) {
  if (n_pairs <= 0 || a.lv[1].n <= 0) return;
  if (a.ld > kMaxBatchedLd) throw Error{MASK_ERR_UNSUPPORTED, "leaf-batched descent: dim above 256"};
  ScopedTiming timing("leaf_scan", s);
  const unsigned grid = (unsigned)((n_pairs + kQStage - 1) / kQStage);
  const uint16_t* rows = a.lv[0].protos_b;
  const uint32_t* co = a.lv[1].child_off;
  const int64_t n1 = a.lv[1].n;
  // the lanes per row and chunks per lane of the descent's BF16 class for
  // this row width
  const int c8 = a.ldb / 8;
  const size_t shm = (size_t)kQStage * a.ld * sizeof(float);
  unsigned long long* n_eval = timing_leaf_counter();
#define MASK_LEAF_SCAN(T, NV)                                                             \
  k_leaf_scan<T, NV><<<grid, kBlock, shm, s>>>(rows, a.ldb, co, n1, pair_key, pair_val,     \
                                              n_pairs, cap, leaf_off, cand_off, Q, ldq, a.dim, \
                                              a.ld, cand, n_eval)
  if (c8 <= 1) MASK_LEAF_SCAN(1, 1);
  else if (c8 <= 2) MASK_LEAF_SCAN(1, 2);
  else if (c8 <= 4) MASK_LEAF_SCAN(1, 4);
  else if (c8 <= 8) MASK_LEAF_SCAN(2, 4);
  else if (c8 <= 12) MASK_LEAF_SCAN(4, 3);
  else if (c8 <= 16) MASK_LEAF_SCAN(4, 4);
  else MASK_LEAF_SCAN(8, 4);
#undef MASK_LEAF_SCAN
  check_launch("leaf_scan");
}

bool level_select(const DescentArgs& a, const QueryArgs& qa, hipStream_t s) {
  if (a.precision != MASK_BF16 || a.sparse || a.metric != MASK_L2 || qa.k_arr || qa.r_arr ||
      qa.radius || qa.out_leaf || qa.out_off || qa.skip_empty || qa.leaf_mode != 1 ||
      a.ld > kMaxBatchedLd || qa.leaf_cap > kSelLeaves || qa.r_lev[1] != qa.leaf_cap)
    return false;
  for (int l = 1; l <= a.n_levels; ++l)
    if (qa.r_lev[l] < 1 || qa.r_lev[l] > kSelMax || qa.beam_e8[l] != 0) return false;
  if (qa.nq <= 0) return true;
  ScopedTiming timing("level_select", s);
  const int64_t n_wg = (qa.nq + kSelWaves - 1) / kSelWaves;
  const unsigned grid = (unsigned)(kXcds * ((n_wg + kXcds - 1) / kXcds));
  // the descent's BF16 class for this row width (lanes per row, 16-byte
  // chunks per lane)
  const int c8 = a.ldb / 8;
  if (c8 <= 1) k_level_select<1, 1><<<grid, kBlock, 0, s>>>(a, qa);
  else if (c8 <= 2) k_level_select<1, 2><<<grid, kBlock, 0, s>>>(a, qa);
  else if (c8 <= 4) k_level_select<1, 4><<<grid, kBlock, 0, s>>>(a, qa);
  else if (c8 <= 8) k_level_select<2, 4><<<grid, kBlock, 0, s>>>(a, qa);
  else if (c8 <= 12) k_level_select<4, 3><<<grid, kBlock, 0, s>>>(a, qa);
  else if (c8 <= 16) k_level_select<4, 4><<<grid, kBlock, 0, s>>>(a, qa);
  else k_level_select<8, 4><<<grid, kBlock, 0, s>>>(a, qa);
  check_launch("level_select");
  return true;
}

bool leaf_select(const DescentArgs& a, const QueryArgs& qa, hipStream_t s) {
  if (a.precision != MASK_BF16 || a.sparse || a.metric != MASK_L2 || qa.k_arr || qa.r_arr ||
      qa.radius || qa.sel || qa.out_leaf || qa.out_off || a.ld > kMaxBatchedLd)
    return false;
  const int64_t r1 = qa.r_lev[1] > 0 ? qa.r_lev[1] : qa.r;
  const int64_t R = a.rerank_factor > 0 ? (int64_t)a.rerank_factor * qa.k
                                        : (int64_t)(-a.rerank_factor) * qa.k * r1;
  if (qa.k > kSelMax || R > kSelMax || qa.leaf_cap > kSelLeaves) return false;
  if (qa.nq <= 0) return true;
  ScopedTiming timing("leaf_select", s);
  const int64_t n_wg = (qa.nq + kSelWaves - 1) / kSelWaves;
  const unsigned grid = (unsigned)(kXcds * ((n_wg + kXcds - 1) / kXcds));
  const int c8 = a.ldb / 8;
  // the lanes per row of the descent's BF16 class for this row width
  if (c8 <= 4) k_leaf_select<1><<<grid, kBlock, 0, s>>>(a, qa, (int)R);
  else if (c8 <= 8) k_leaf_select<2><<<grid, kBlock, 0, s>>>(a, qa, (int)R);
  else if (c8 <= 16) k_leaf_select<4><<<grid, kBlock, 0, s>>>(a, qa, (int)R);
  else k_leaf_select<8><<<grid, kBlock, 0, s>>>(a, qa, (int)R);
  check_launch("leaf_select");
  return true;
}

}  // namespace mask

// k-means++ seeding (Arthur and Vassilvitskii 2007; Section 3.1 names it as
// the remedy for initial prototypes placed badly) for every group of a level
// at once.  The k draws are sequential; each is two launches: a pick (one
// wave per group, with further workgroups that repeat it and compute the
// distances of the new prototype to the group's earlier ones) and a D^2
// update over the rows the triangle inequality cannot rule out (one
// workgroup per tile of consecutive members) that also sums D^2 per tile.
// The skip is exact: the D^2 values are those of reading every row.
//
// Draw t of group c uses u = the top 53 bits of the SplitMix64 output at
// counter tag + c * k + t.  Draw 0 picks member floor(u * m); draw t > 0 picks
// the first member whose running sum of D^2 (in group order) exceeds
// u * sum D^2, where D^2 is the squared distance (FP64, direct form) to the
// nearest prototype chosen so far.  With sum D^2 = 0 the pick is uniform as
// for draw 0.  The sums are taken in a fixed tree order (wave sums and
// scans), so a pick can differ from a sequential running sum only when the
// target lies within rounding of a member boundary.
#include <algorithm>
#include <cfloat>

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

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline double wave_incl_scan(double v, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  return v;
}

// The members of group c are cut into tiles of T_c consecutive members: a
// multiple of 64, at least tmin and large enough for at most kMaxTiles tiles
// per group.  Tiles of all groups are numbered consecutively from
// tile_base[c]; tile b covers rows [tile_row[b], tile_row[b + 1]) of group
// tile_grp[b].
constexpr int kMaxTiles = 2048;

// Shortest tile: 256 members where one draw's rows take 64 MiB or more (the
// update is bound by bytes, and a long tile keeps many rows in flight per
// workgroup), else 128 (fewer, shorter round trips per draw).
constexpr int64_t kLongTileBytes = (int64_t)64 << 20;

__host__ __device__ inline int64_t tile_len(int64_t m, int tmin) {
  const int64_t T =
      (int64_t)kWave * ((m + (int64_t)kWave * kMaxTiles - 1) / ((int64_t)kWave * kMaxTiles));
  return T > tmin ? T : tmin;
}

// Squared distance (FP64, direct form) of FP32 row x to FP32 row y: G lanes
// per row, U float4 columns each in flight, a butterfly over the lane group.
// Every lane of the group returns the same value; the order of the sums
// depends only on (G, U, ld), so every kernel below gets the same bits for
// the same pair.
template <int G, int U>
__device__ inline double row_d2(const float4* __restrict__ x, const float4* __restrict__ y,
                                int ld4, int gl) {
  double acc = 0.0;
  for (int q0 = gl; q0 < ld4; q0 += G * U) {
    float4 a[U], b[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int q = q0 + j * G;
      a[j] = q < ld4 ? x[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      b[j] = q < ld4 ? y[q] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const double e0 = (double)a[j].x - (double)b[j].x, e1 = (double)a[j].y - (double)b[j].y;
      const double e2 = (double)a[j].z - (double)b[j].z, e3 = (double)a[j].w - (double)b[j].w;
      acc = fma(e0, e0, acc);
      acc = fma(e1, e1, acc);
      acc = fma(e2, e2, acc);
      acc = fma(e3, e3, acc);
    }
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  return acc;
}

// Draw t of group c, by one wave (lane = lane id): returns the item index
// of the chosen member.  Lane l holds the sums of tiles l R .. l R + R - 1
// (R = ceil(tiles / 64)); the lane totals, an inclusive wave scan of them and
// one sequential pass in the lane whose range holds the target find the tile;
// in the tile, each lane sums 8 consecutive members, a wave scan of those
// sums finds the lane and a walk through its 8 members the member.  If rounding leaves the
// target unreached, the last member with D^2 > 0 of that tile (or of the
// group) is taken.  Deterministic: every wave that runs it gets the same
// member.  NR >= R registers per lane hold the tile sums.
template <int NR>
__device__ int64_t pp_pick(const int64_t* __restrict__ chunk_off,
                           const int64_t* __restrict__ tile_base, int tmin, int k, int t,
                           uint64_t seed, uint64_t tag, const double* __restrict__ d2,
                           const double* __restrict__ tsum, int c, int lane) {
  const int64_t c0 = chunk_off[c], c1 = chunk_off[c + 1], m = c1 - c0;
  const double u = uniform01(seed, tag + (uint64_t)c * (uint64_t)k + (uint64_t)t);
  const int64_t T = tile_len(m, tmin);
  const int64_t tb = tile_base[c];
  const int nt = (int)(tile_base[c + 1] - tb);
  int64_t pick = -1;
  if (t > 0) {
    constexpr int kRegs = NR;
    const int R = (nt + kWave - 1) / kWave;
    double v[kRegs];
    double own = 0.0;
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {
      const int b = lane * R + j;
      v[j] = (j < R && b < nt) ? tsum[tb + b] : 0.0;
      own += v[j];
    }
    const double incl = wave_incl_scan(own, lane);
    const double total = __shfl(incl, kWave - 1);
    if (total > 0.0) {
      const double target = u * total;
      const double up = __shfl_up(incl, 1);  // by every lane: a shuffle reads active lanes only
      const double before = lane > 0 ? up : 0.0;
      // every lane walks its own range; the hit lane's result is used
      double run = before;
      int j_hit = -1, j_pos = -1;
#pragma unroll
      for (int j = 0; j < kRegs; ++j) {
        if (j < R && lane * R + j < nt) {
          if (j_hit < 0) {
            if (run + v[j] > target) j_hit = j;
            else run += v[j];
          }
          if (v[j] > 0.0) j_pos = j;
        }
      }
      const unsigned long long hit = __ballot(incl > target);
      int64_t lo = c0, hi = c1;  // where the fallback looks
      bool scan = false;
      if (hit) {
        const int L = __ffsll((long long)hit) - 1;
        const int jh = __shfl(j_hit, L), jp = __shfl(j_pos, L);
        run = __shfl(run, L);
        // jh < 0 only by rounding: then the last positive member of the
        // lane's last positive tile, or of the group when it has none
        if (jh >= 0 || jp >= 0) {
          const int tile = L * R + (jh >= 0 ? jh : jp);
          scan = jh >= 0;
          lo = c0 + (int64_t)tile * T;
          hi = min(c1, lo + T);
        }
      }
      if (scan) {
        // the tile's D^2 in spans of 64 x kSpan members, one load of kSpan
        // consecutive members per lane (all in flight together): lane sums,
        // a wave scan of them, then a walk through the hit lane's members
        constexpr int kSpan = 8;
        for (int64_t i0 = lo; i0 < hi && pick < 0; i0 += kWave * kSpan) {
          const int64_t l0 = i0 + (int64_t)lane * kSpan;
          double dv[kSpan];
          double lsum = 0.0;
#pragma unroll
          for (int e = 0; e < kSpan; ++e) {
            dv[e] = l0 + e < hi ? d2[l0 + e < hi ? l0 + e : lo] : 0.0;
            lsum += dv[e];
          }
          const double ci = wave_incl_scan(lsum, lane);
          const unsigned long long h = __ballot(run + ci > target);
          if (h) {
            const int L = __ffsll((long long)h) - 1;
            const double up2 = __shfl_up(ci, 1);
            double acc = run + (lane > 0 ? up2 : 0.0);
            int e_hit = -1, e_pos = -1;
#pragma unroll
            for (int e = 0; e < kSpan; ++e) {
              if (e_hit < 0) {
                if (acc + dv[e] > target) e_hit = e;
                else acc += dv[e];
              }
              if (dv[e] > 0.0) e_pos = e;
            }
            // by rounding the walk can end short of the target: then the
            // lane's last member with D^2 > 0 (it has one: its sum moved the
            // scan past the target)
            const int e = __shfl(e_hit >= 0 ? e_hit : e_pos, L);
            if (e >= 0) pick = i0 + (int64_t)L * kSpan + e - c0;
          } else {
            run += __shfl(ci, kWave - 1);
          }
        }
      }
      for (int64_t i1 = hi; i1 > lo && pick < 0; i1 -= kWave) {
        const int64_t i = i1 - kWave + lane;
        const unsigned long long pos = __ballot(i >= lo && d2[i >= lo ? i : lo] > 0.0);
        if (pos) pick = (i1 - kWave + (63 - __clzll((long long)pos))) - c0;
      }
    }
  }
  if (pick < 0) {
    pick = (int64_t)(u * (double)m);
    if (pick >= m) pick = m - 1;
  }
  return c0 + pick;
}

// Draw t of every group, and the distances of the new prototype to the
// group's earlier ones: cc[c * k + j] = |p_{c,j} - p_{c,t}|^2 for j < t when
// the launch has more than one workgroup row.  Workgroup (c, 0) makes the
// pick and copies the chosen row to prototype c * k + t; every workgroup
// (c, y > 0) repeats the pick (the same member) and computes `passes` times
// 4 * 64 / G of the distances against the chosen item row (equal to the
// copy), G lanes per prototype.
template <int G, int U, int NR>
__global__ __launch_bounds__(kBlock) void k_pp_pick(
    const float* __restrict__ items, int ld, const int64_t* __restrict__ chunk_off,
    const int64_t* __restrict__ tile_base, int tmin, int k, int t, uint64_t seed, uint64_t tag,
    const double* __restrict__ d2, const double* __restrict__ tsum,
    float* __restrict__ protos, int32_t* __restrict__ chosen, double* __restrict__ cc,
    int passes) {
  constexpr int R = kWave / G;
  __shared__ int64_t s_item;
  const int c = blockIdx.x, lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (wave == 0) {
    const int64_t pi = pp_pick<NR>(chunk_off, tile_base, tmin, k, t, seed, tag, d2, tsum, c, lane);
    if (blockIdx.y == 0) {
      const int64_t slot = (int64_t)c * k + t;
      for (int q = lane; q < ld; q += kWave) protos[slot * ld + q] = items[pi * ld + q];
      if (lane == 0 && chosen) chosen[slot] = (int32_t)pi;
    }
    if (lane == 0) s_item = pi;
  }
  if (blockIdx.y == 0) return;  // uniform across the workgroup
  __syncthreads();
  const int slot = lane / G, gl = lane % G;
  const float4* y = reinterpret_cast<const float4*>(items + s_item * ld);
  for (int ps = 0; ps < passes; ++ps) {
    const int j = (((blockIdx.y - 1) * passes + ps) * (kBlock / kWave) + wave) * R + slot;
    const bool live = j < t;
    const float4* x =
        reinterpret_cast<const float4*>(protos + ((int64_t)c * k + (live ? j : 0)) * ld);
    const double acc = row_d2<G, U>(x, y, ld / 4, gl);
    if (live && gl == 0) cc[(int64_t)c * k + j] = acc;
  }
}

// BF16 rounding bound of the screen below: a row's BF16 copy x~ (round to
// nearest even, 8 significant bits) is within 2^-8 |x_i| of x in every
// component, so |x - x~| <= 2^-8 |x| <= 2^-8 |x~| / (1 - 2^-8).
constexpr double kBf16RelErr = 0.00390625 / (1.0 - 0.00390625);

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// D^2 after draw t, one workgroup per tile, in rounds of 512 members (two
// per thread, whose state loads are in flight together).  Rows
// are skipped by the triangle inequality: near[i] is the prototype (index in
// the group) at D^2 of row i, and when |p_near - p_t|^2 exceeds
// 4 D^2 (1 + 1e-6), |x - p_t| > |x - p_near| holds with room to spare for
// the rounding of both FP64 sums, so D^2 keeps its value exactly and the row
// is not read.  From draw 1 on, a remaining row is screened on its BF16 copy
// first: |x~ - p_t| (FP32 sums, shrunk by their rounding bound) minus the
// BF16 rounding bound 2^-8 |x~| / (1 - 2^-8) is a lower bound of |x - p_t|,
// and when its square exceeds D^2 (1 + 1e-12) the row's D^2 cannot fall (its
// exact FP64 distance is within 1e-14 of the true one), so its FP32 row is
// not read.  The other
// rows (every row at draw 0) get the exact distance: a lane group of G lanes
// computes each one (64 / G rows per wave and pass, the four waves on
// interleaved rows) and hands the new D^2 to the chunk's thread of that
// member through LDS; thread j adds members j, j + 256, ... of the tile in
// turn (the same order whatever the round length), then wave sums and the four waves in order give the tile's sum.
// Draw 0 reads every row and sets near = 0.  Both skips leave every D^2 as
// reading every row exactly would.
template <int G, int U, int SB>
__global__ __launch_bounds__(kBlock) void k_pp_update(
    const float* __restrict__ items, int ld, const uint16_t* __restrict__ items_b, int ldb,
    const int64_t* __restrict__ tile_row, const int32_t* __restrict__ tile_grp, int k, int t,
    const float* __restrict__ protos, const double* __restrict__ cc, double* __restrict__ d2,
    int32_t* __restrict__ near, double* __restrict__ tsum, unsigned long long* __restrict__ tile_cnt) {
  constexpr int R = kWave / G;                 // rows per wave and pass
  constexpr int W = kBlock / kWave;            // waves per tile
  constexpr int RT = 2;                        // rows per thread and round
  constexpr int TR = kBlock * RT;              // rows per round
  __shared__ double s_wave[W];
  __shared__ double s_val[TR];
  __shared__ double s_cur[TR];
  __shared__ int32_t s_rows[TR];
  __shared__ int32_t s_exact[TR];
  __shared__ float4 s_ctr[kMaxDenseDim / 4];  // the new prototype, for the screen
  __shared__ int s_n, s_ne, s_low;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t tile = blockIdx.x;
  const int grp = tile_grp[tile];
  const int64_t r0 = tile_row[tile], r1 = tile_row[tile + 1];
  const float* ctr_row = protos + ((int64_t)grp * k + t) * ld;
  const float4* ctr = reinterpret_cast<const float4*>(ctr_row);
  const int ld4 = ld / 4, nb8 = ldb / 8, slot = lane / G, gl = lane % G;
  const bool screen = t > 0 && items_b != nullptr;
  // the screen: 4 lanes per row, SB 16-byte BF16 chunks per lane (all of
  // them in flight at once), the prototype's row from LDS
  constexpr int GS = 4, RS = kWave / GS;
  const int sslot = lane / GS, sgl = lane % GS;
  if (screen)
    for (int c = threadIdx.x; c < 2 * SB * GS; c += kBlock)
      s_ctr[c] = 4 * c < ld ? ctr[c] : make_float4(0.f, 0.f, 0.f, 0.f);
  double own = 0.0;
  unsigned long long n_rows = 0, n_exact = 0;  // thread 0 only
  if (threadIdx.x == 0) s_low = 0;
  // A round covers TR rows; thread x owns rows x and x + kBlock of it (the
  // order in which it adds their D^2 into the tile sum).
  for (int64_t b0 = r0; b0 < r1; b0 += TR) {
    if (threadIdx.x == 0) { s_n = 0; s_ne = 0; }
    __syncthreads();
    double cur[RT];
    bool read[RT];
    if (t > 0) {
      // every row's state loads are in flight together (indexes clamped to
      // the tile, values selected afterwards), then the prototype distances
      int32_t nr[RT];
#pragma unroll
      for (int j = 0; j < RT; ++j) {
        const int64_t i = b0 + threadIdx.x + j * kBlock;
        const int64_t ic = i < r1 ? i : r0;
        cur[j] = d2[ic];
        nr[j] = near[ic];
      }
#pragma unroll
      for (int j = 0; j < RT; ++j) {
        const bool mine = b0 + threadIdx.x + j * kBlock < r1;
        read[j] = mine && cc[(int64_t)grp * k + nr[j]] <= 4.0 * cur[j] * (1.0 + 1e-6);
      }
    } else {
#pragma unroll
      for (int j = 0; j < RT; ++j) {
        cur[j] = 0.0;
        read[j] = b0 + threadIdx.x + j * kBlock < r1;
      }
    }
#pragma unroll
    for (int j = 0; j < RT; ++j)
      if (read[j]) {
        const int local = threadIdx.x + j * kBlock;
        const int at = atomicAdd(&s_n, 1);
        s_rows[at] = local;
        s_cur[local] = cur[j];
      }
    __syncthreads();
    const int n_read = s_n;
    n_rows += n_read;
    int n_ex = n_read;
    const int32_t* exact = s_rows;
    if (screen) {
      for (int p0 = 0; p0 < n_read; p0 += RS * W) {
        const int p = p0 + wave * RS + sslot;
        const bool live = p < n_read;
        const int local = live ? s_rows[p] : 0;
        const uint4* xb = reinterpret_cast<const uint4*>(items_b + (b0 + local) * ldb);
        uint4 w[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
          const int q = sgl + GS * j;
          w[j] = q < nb8 ? xb[q] : make_uint4(0u, 0u, 0u, 0u);
        }
        // FP32 sums of at most ld + 8 rounded terms each (differences, FMAs,
        // the butterfly): within 1e-5 relative of the exact sums for ld <= 256
        float sd = 0.f, sx = 0.f;
#pragma unroll
        for (int j = 0; j < SB; ++j) {
          const int q = sgl + GS * j;  // chunks past the row are zero on both sides
          const float4 c0 = s_ctr[2 * q], c1 = s_ctr[2 * q + 1];
          const float x0 = bf16_lo(w[j].x), x1 = bf16_hi(w[j].x), x2 = bf16_lo(w[j].y);
          const float x3 = bf16_hi(w[j].y), x4 = bf16_lo(w[j].z), x5 = bf16_hi(w[j].z);
          const float x6 = bf16_lo(w[j].w), x7 = bf16_hi(w[j].w);
          float e;
          e = x0 - c0.x; sd = fmaf(e, e, sd); sx = fmaf(x0, x0, sx);
          e = x1 - c0.y; sd = fmaf(e, e, sd); sx = fmaf(x1, x1, sx);
          e = x2 - c0.z; sd = fmaf(e, e, sd); sx = fmaf(x2, x2, sx);
          e = x3 - c0.w; sd = fmaf(e, e, sd); sx = fmaf(x3, x3, sx);
          e = x4 - c1.x; sd = fmaf(e, e, sd); sx = fmaf(x4, x4, sx);
          e = x5 - c1.y; sd = fmaf(e, e, sd); sx = fmaf(x5, x5, sx);
          e = x6 - c1.z; sd = fmaf(e, e, sd); sx = fmaf(x6, x6, sx);
          e = x7 - c1.w; sd = fmaf(e, e, sd); sx = fmaf(x7, x7, sx);
        }
#pragma unroll
        for (int o = GS / 2; o >= 1; o >>= 1) {
          sd += __shfl_xor(sd, o);
          sx += __shfl_xor(sx, o);
        }
        if (live && sgl == 0) {
          const double lb = sqrt((double)sd * (1.0 - 1e-5)) -
                            sqrt((double)sx * (1.0 + 1e-5)) * kBf16RelErr - 1e-30;
          const double old = s_cur[local];
          // an FP32 sum that overflowed settles nothing
          if (sd <= FLT_MAX && lb > 0.0 && lb * lb > old * (1.0 + 1e-12))
            s_val[local] = old;  // settled
          else s_exact[atomicAdd(&s_ne, 1)] = local;
        }
      }
      __syncthreads();
      n_ex = s_ne;
      exact = s_exact;
    }
    n_exact += n_ex;
    for (int p0 = 0; p0 < n_ex; p0 += R * W) {
      const int p = p0 + wave * R + slot;
      const bool live = p < n_ex;
      const int local = live ? exact[p] : 0;
      const int64_t row = b0 + local;
      const double acc = row_d2<G, U>(reinterpret_cast<const float4*>(items + row * ld), ctr,
                                      ld4, gl);
      if (live && gl == 0) {
        const double old = t > 0 ? s_cur[local] : acc;
        const bool lower = t == 0 || acc < old;
        s_val[local] = lower ? acc : old;
        if (lower) {
          d2[row] = acc;
          near[row] = t;
          if (tile_cnt) atomicAdd(&s_low, 1);
        }
      }
    }
    __syncthreads();  // s_val complete
#pragma unroll
    for (int j = 0; j < RT; ++j)
      if (b0 + threadIdx.x + j * kBlock < r1) own += read[j] ? s_val[threadIdx.x + j * kBlock] : cur[j];
    __syncthreads();  // s_val, s_cur and the row lists are reused
  }
  own = wave_sum(own);
  if (lane == 0) s_wave[wave] = own;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) sum += s_wave[w];
    tsum[tile] = sum;
    if (tile_cnt) {  // the tile's own slots: no other workgroup writes them
      tile_cnt[3 * tile] += n_rows;
      tile_cnt[3 * tile + 1] += n_exact;
      tile_cnt[3 * tile + 2] += (unsigned long long)s_low;
    }
  }
}

// Adds the per-tile counts (rows not ruled out by the triangle inequality,
// rows read exactly, rows whose D^2 fell) into the three timing counters
// (one workgroup).
__global__ __launch_bounds__(kBlock) void k_pp_count(const unsigned long long* __restrict__ tile_cnt,
                                                     int64_t n_tiles,
                                                     unsigned long long* __restrict__ out) {
  __shared__ unsigned long long s_sum[3][kBlock];
  unsigned long long a[3] = {0, 0, 0};
  for (int64_t i = threadIdx.x; i < n_tiles; i += kBlock)
    for (int c = 0; c < 3; ++c) a[c] += tile_cnt[3 * i + c];
  for (int c = 0; c < 3; ++c) s_sum[c][threadIdx.x] = a[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < kBlock; ++j)
      for (int c = 0; c < 3; ++c) a[c] += s_sum[c][j];
    for (int c = 0; c < 3; ++c) out[c] += a[c];
  }
}

// Timing scope of one level's seeding, "kmeanspp_level<l>" (update = false),
// or of each of its update launches, "kmeanspp_update_level<l>".
const char* seed_scope_name(int slot, bool update = false) {
  static const std::vector<std::string> names = [] {
    std::vector<std::string> v;
    for (int l = 0; l < kSeedSlots; ++l) v.push_back("kmeanspp_level" + std::to_string(l));
    for (int l = 0; l < kSeedSlots; ++l) v.push_back("kmeanspp_update_level" + std::to_string(l));
    return v;
  }();
  return names[slot + (update ? kSeedSlots : 0)].c_str();
}

struct SeedBuffers {
  const float* items;
  int ld;
  const uint16_t* items_b;  // BF16 copy of the rows (stride ldb)
  int ldb;
  const ChunkPlan* plan;
  const int64_t* tile_base;
  const int64_t* tile_row;
  const int32_t* tile_grp;
  int tmin;
  int64_t n_tiles;
  float* protos;
  double* d2;
  double* tsum;
  double* cc;
  int32_t* near;
  unsigned long long* tile_cnt;  // null unless timing is on
  int64_t max_tiles;             // tiles of the largest group
  const char* update_scope;      // timing scope of each update launch, or null
};

// Draw t: the pick (with the distances the update needs, unless it is the
// last draw) and the D^2 update.
template <int G, int U, int SB>
void launch_draw(const SeedBuffers& b, int t, uint64_t seed, uint64_t tag, int32_t* chosen,
                 hipStream_t s) {
  const ChunkPlan& p = *b.plan;
  const bool last = t + 1 == p.k;
  constexpr int per_pass = (kBlock / kWave) * (kWave / G);
  // about 2,048 distance workgroups at most (each repeats the pick, and more
  // would not be resident at once): several passes each when groups are many
  const int need = (!last && t > 0) ? (t + per_pass - 1) / per_pass : 0;
  const int cap = std::max(1, 2048 / std::max(1, p.n_chunks));
  const int passes = need > cap ? (need + cap - 1) / cap : 1;
  const int rows = (need + passes - 1) / passes;
  const dim3 grid((unsigned)p.n_chunks, (unsigned)(1 + rows));
  // registers for the tile sums: the level's largest group (fewer registers,
  // more workgroups resident)
#define MASK_PICK(NR)                                                                       \
  k_pp_pick<G, U, NR><<<grid, kBlock, 0, s>>>(b.items, b.ld, p.d_off, b.tile_base, b.tmin, \
                                              p.k, t, seed, tag, b.d2, b.tsum, b.protos,   \
                                              chosen, b.cc, passes)
  if (b.max_tiles <= 8 * kWave) MASK_PICK(8);
  else if (b.max_tiles <= 16 * kWave) MASK_PICK(16);
  else MASK_PICK(kMaxTiles / kWave);
#undef MASK_PICK
  if (last) return;
  // levels of at least 2^20 rows time every update launch (each reads
  // megabytes, so the two event records cost little beside it)
  ScopedTiming timing(b.update_scope, s, b.update_scope != nullptr);
  k_pp_update<G, U, SB><<<(unsigned)b.n_tiles, kBlock, 0, s>>>(
      b.items, b.ld, b.items_b, b.ldb, b.tile_row, b.tile_grp, p.k, t, b.protos, b.cc, b.d2,
      b.near, b.tsum, b.tile_cnt);
}

}  // namespace

void kmeanspp_init(const float* items, int ld, int dim, const ChunkPlan& plan, uint64_t seed,
                   int level, float* protos, int32_t* chosen, Arena& scratch, hipStream_t s) {
  (void)dim;  // rows are zero-padded to ld
  MASK_CHECK(ld <= kMaxDenseDim, "k-means++ seeding: dim above 256");
  const int tmin =
      (int64_t)plan.n_items * ld * (int64_t)sizeof(float) >= kLongTileBytes ? 256 : 128;
  std::vector<int64_t> base(plan.n_chunks + 1, 0), row;
  std::vector<int32_t> grp;
  for (int c = 0; c < plan.n_chunks; ++c) {
    const int64_t c0 = plan.off[c], m = plan.off[c + 1] - c0, T = tile_len(m, tmin);
    for (int64_t r = c0; r < c0 + m; r += T) {
      row.push_back(r);
      grp.push_back(c);
    }
    base[c + 1] = (int64_t)row.size();
  }
  row.push_back(plan.n_items);
  SeedBuffers b{};
  b.items = items;
  b.ld = ld;
  b.plan = &plan;
  b.n_tiles = base[plan.n_chunks];
  for (int c = 0; c < plan.n_chunks; ++c) b.max_tiles = std::max(b.max_tiles, base[c + 1] - base[c]);
  b.protos = protos;
  b.tmin = tmin;
  int64_t* tile_base = scratch.alloc<int64_t>(base.size());
  int64_t* tile_row = scratch.alloc<int64_t>(row.size());
  int32_t* tile_grp = scratch.alloc<int32_t>(std::max<size_t>(grp.size(), 1));
  MASK_HIP(hipMemcpyAsync(tile_base, base.data(), base.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  MASK_HIP(hipMemcpyAsync(tile_row, row.data(), row.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  if (!grp.empty())
    MASK_HIP(hipMemcpyAsync(tile_grp, grp.data(), grp.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
  b.tile_base = tile_base;
  b.tile_row = tile_row;
  b.tile_grp = tile_grp;
  b.d2 = scratch.alloc<double>(plan.n_items);
  b.tsum = scratch.alloc<double>(b.n_tiles);
  b.cc = scratch.alloc<double>((size_t)plan.n_chunks * plan.k);
  b.near = scratch.alloc<int32_t>(plan.n_items);
  // BF16 copy of the rows for the update's screen
  b.ldb = (ld + 7) & ~7;
  uint16_t* items_b = scratch.alloc<uint16_t>(plan.n_items * (int64_t)b.ldb);
  quantize_bf16(items, ld, plan.n_items, items_b, b.ldb, nullptr, s);
  b.items_b = items_b;
  const int slot = std::min(std::max(level, 0), kSeedSlots - 1);
  unsigned long long* counters = timing_seed_counter(slot);
  if (counters) {
    b.tile_cnt = scratch.alloc<unsigned long long>(3 * b.n_tiles);
    MASK_HIP(hipMemsetAsync(b.tile_cnt, 0, 3 * b.n_tiles * sizeof(unsigned long long), s));
  }
  b.update_scope = plan.n_items >= ((int64_t)1 << 20) ? seed_scope_name(slot, true) : nullptr;
  ScopedTiming timing(seed_scope_name(slot), s);
  const uint64_t tag = ((uint64_t)level << 40);
  const int f4 = ld / 4;
  for (int t = 0; t < plan.k; ++t) {
    // (G, U) of the exact distances; SB = the screen's chunks per lane,
    // ceil(ldb / 8 / 4)
    if (f4 <= 1) launch_draw<1, 1, 1>(b, t, seed, tag, chosen, s);
    else if (f4 <= 2) launch_draw<2, 1, 1>(b, t, seed, tag, chosen, s);
    else if (f4 <= 4) launch_draw<4, 1, 1>(b, t, seed, tag, chosen, s);
    else if (f4 <= 8) launch_draw<8, 1, 1>(b, t, seed, tag, chosen, s);
    else if (f4 <= 16) launch_draw<8, 2, 2>(b, t, seed, tag, chosen, s);
    else if (f4 <= 24) launch_draw<8, 2, 3>(b, t, seed, tag, chosen, s);  // measured: 8 lanes beat 16 at d = 96
    else if (f4 <= 32) launch_draw<16, 2, 4>(b, t, seed, tag, chosen, s);
    else launch_draw<16, 4, 8>(b, t, seed, tag, chosen, s);
  }
  if (counters) k_pp_count<<<1, kBlock, 0, s>>>(b.tile_cnt, b.n_tiles, counters);
  check_launch("kmeanspp");
}

}  // namespace mask

// k-means++ seeding (Arthur and Vassilvitskii 2007; Section 3.1 names it as
// the remedy for initial prototypes placed badly) for every group of a level
// at once.  The k draws are sequential; each is two launches: a pick (one
// wave per group) and a D^2 update over every row (one workgroup per tile of
// consecutive members) that also sums D^2 per tile.
//
// Draw t of group c uses u = the top 53 bits of the SplitMix64 output at
// counter tag + c * k + t.  Draw 0 picks member floor(u * m); draw t > 0 picks
// the first member whose running sum of D^2 (in group order) exceeds
// u * sum D^2, where D^2 is the squared distance (FP64, direct form) to the
// nearest prototype chosen so far.  With sum D^2 = 0 the pick is uniform as
// for draw 0.  The sums are taken in a fixed tree order (wave sums and
// scans), so a pick can differ from a sequential running sum only when the
// target lies within rounding of a member boundary.
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

// The members of group c are cut into tiles of T_c consecutive members (T_c a
// multiple of 64, at most kMaxTiles tiles per group); tiles of all groups are
// numbered consecutively from tile_base[c].
constexpr int kMaxTiles = 2048;

__device__ inline int64_t tile_len(int64_t m) {
  return (int64_t)kWave * ((m + (int64_t)kWave * kMaxTiles - 1) / ((int64_t)kWave * kMaxTiles));
}

// Draw t of every group: one wave per group.  It totals the group's tile
// sums, finds the first tile whose running sum passes the target and, inside
// it, the first member, with wave scans.  The chosen row becomes prototype
// c * k + t.  If rounding leaves the target unreached, the last member with
// D^2 > 0 of the tile (or of the group) is taken.
__global__ __launch_bounds__(kWave) void k_pp_pick(
    const float* __restrict__ items, int ld, const int64_t* __restrict__ chunk_off,
    const int64_t* __restrict__ tile_base, int k, int t, uint64_t seed, uint64_t tag,
    const double* __restrict__ d2, const double* __restrict__ tsum,
    float* __restrict__ protos, int32_t* __restrict__ chosen) {
  const int c = blockIdx.x, lane = threadIdx.x;
  const int64_t c0 = chunk_off[c], c1 = chunk_off[c + 1], m = c1 - c0;
  const double u = uniform01(seed, tag + (uint64_t)c * (uint64_t)k + (uint64_t)t);
  const int64_t T = tile_len(m);
  const int64_t tb = tile_base[c];
  const int nt = (int)(tile_base[c + 1] - tb);
  int64_t pick = -1;
  if (t > 0) {
    // every tile sum of the group in registers: lane l holds tiles j * 64 + l
    constexpr int kRegs = kMaxTiles / kWave;
    double v[kRegs];
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {
      const int b = j * kWave + lane;
      v[j] = b < nt ? tsum[tb + b] : 0.0;
    }
    double total = 0.0;
#pragma unroll
    for (int j = 0; j < kRegs; ++j) total += wave_sum(v[j]);
    if (total > 0.0) {
      const double target = u * total;
      double run = 0.0;
      int tile = -1;
#pragma unroll
      for (int j = 0; j < kRegs; ++j) {
        const double incl = wave_incl_scan(v[j], lane);
        const unsigned long long hit = __ballot(tile < 0 && run + incl > target);
        const double excl = __shfl(incl - v[j], hit ? __ffsll((long long)hit) - 1 : 0);
        const double last = __shfl(incl, kWave - 1);
        if (tile < 0) {
          if (hit) {
            tile = j * kWave + __ffsll((long long)hit) - 1;
            run += excl;
          } else {
            run += last;
          }
        }
      }
      int64_t lo = c0, hi = c1;  // where the fallback looks
      if (tile >= 0) {
        lo = c0 + (int64_t)tile * T;
        hi = min(c1, lo + T);
        for (int64_t i0 = lo; i0 < hi && pick < 0; i0 += kWave) {
          const bool in = i0 + lane < hi;
          const double dv = in ? d2[i0 + lane] : 0.0;
          const double incl = wave_incl_scan(dv, lane);
          const unsigned long long hit = __ballot(in && run + incl > target);
          if (hit) pick = i0 + (__ffsll((long long)hit) - 1) - c0;
          else run += __shfl(incl, kWave - 1);
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
  const int64_t pi = c0 + pick;
  const int64_t slot = (int64_t)c * k + t;
  for (int q = lane; q < ld; q += kWave) protos[slot * ld + q] = items[pi * ld + q];
  if (lane == 0 && chosen) chosen[slot] = (int32_t)pi;
}

// D^2 after draw t, one workgroup per tile: G lanes per row (each with U
// float4 columns in flight, FP64 accumulation, butterfly over the lane
// group), 64 / G rows per wave and pass, the four waves on interleaved rows.
// The tile's sum of D^2 is added in a fixed order: per row slot over the
// passes, across the slots of a wave, then across the waves.
template <int G, int U>
__global__ __launch_bounds__(kBlock) void k_pp_update(
    const float* __restrict__ items, int ld, const int64_t* __restrict__ chunk_off,
    const int64_t* __restrict__ tile_base, int n_chunks, int k, int t,
    const float* __restrict__ protos, double* __restrict__ d2, double* __restrict__ tsum) {
  constexpr int R = kWave / G;                 // rows per wave and pass
  constexpr int W = kBlock / kWave;            // waves per tile
  __shared__ double s_wave[W];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = n_chunks - 1;  // group of the tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_base[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  const int64_t c0 = chunk_off[lo], c1 = chunk_off[lo + 1];
  const int64_t T = tile_len(c1 - c0);
  const int64_t r0 = c0 + (tile - tile_base[lo]) * T, r1 = min(c1, r0 + T);
  const float4* ctr = reinterpret_cast<const float4*>(protos + ((int64_t)lo * k + t) * ld);
  const int ld4 = ld / 4, slot = lane / G, gl = lane % G;
  double tile_acc = 0.0;
  const int64_t first = r0 + wave * R + slot;
  for (int64_t i = first; i - slot - wave * R < r1; i += (int64_t)R * W) {
    const bool live = i < r1;
    const float4* x = reinterpret_cast<const float4*>(items + (live ? i : r0) * ld);
    double acc = 0.0;
    for (int q0 = gl; q0 < ld4; q0 += G * U) {
      float4 a[U], b[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int q = q0 + j * G;
        a[j] = q < ld4 ? x[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        b[j] = q < ld4 ? ctr[q] : make_float4(0.f, 0.f, 0.f, 0.f);
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
    if (live) {
      double v = acc;
      if (t > 0) v = fmin(d2[i], acc);
      if (gl == 0) d2[i] = v;
      tile_acc += v;
    }
  }
#pragma unroll
  for (int o = kWave / 2; o >= G; o >>= 1) tile_acc += __shfl_xor(tile_acc, o);
  if (lane == 0) s_wave[wave] = tile_acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) sum += s_wave[w];
    tsum[tile] = sum;
  }
}

template <int G, int U>
void launch_update(const float* items, int ld, const ChunkPlan& plan, const int64_t* tile_base,
                   int64_t n_tiles, int t, const float* protos, double* d2, double* tsum,
                   hipStream_t s) {
  k_pp_update<G, U><<<(unsigned)n_tiles, kBlock, 0, s>>>(items, ld, plan.d_off, tile_base,
                                                         plan.n_chunks, plan.k, t, protos, d2,
                                                         tsum);
}

}  // namespace

void kmeanspp_init(const float* items, int ld, int dim, const ChunkPlan& plan, uint64_t seed,
                   int level, float* protos, int32_t* chosen, Arena& scratch, hipStream_t s) {
  (void)dim;  // rows are zero-padded to ld
  MASK_CHECK(ld <= kMaxDenseDim, "k-means++ seeding: dim above 256");
  // tiles of every group (the same lengths as tile_len on the device)
  std::vector<int64_t> base(plan.n_chunks + 1, 0);
  for (int c = 0; c < plan.n_chunks; ++c) {
    const int64_t m = plan.off[c + 1] - plan.off[c];
    const int64_t T = (int64_t)kWave * ((m + (int64_t)kWave * kMaxTiles - 1) /
                                        ((int64_t)kWave * kMaxTiles));
    base[c + 1] = base[c] + (m + T - 1) / T;
  }
  const int64_t n_tiles = base[plan.n_chunks];
  int64_t* tile_base = scratch.alloc<int64_t>(plan.n_chunks + 1);
  MASK_HIP(hipMemcpyAsync(tile_base, base.data(), base.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  double* d2 = scratch.alloc<double>(plan.n_items);
  double* tsum = scratch.alloc<double>(n_tiles);
  ScopedTiming timing("kmeanspp", s);
  const uint64_t tag = ((uint64_t)level << 40);
  const int f4 = ld / 4;
  for (int t = 0; t < plan.k; ++t) {
    k_pp_pick<<<(unsigned)plan.n_chunks, kWave, 0, s>>>(items, ld, plan.d_off, tile_base, plan.k,
                                                       t, seed, tag, d2, tsum, protos, chosen);
    if (t + 1 == plan.k) break;  // the last draw needs no update
    if (f4 <= 1) launch_update<1, 1>(items, ld, plan, tile_base, n_tiles, t, protos, d2, tsum, s);
    else if (f4 <= 2) launch_update<2, 1>(items, ld, plan, tile_base, n_tiles, t, protos, d2, tsum, s);
    else if (f4 <= 4) launch_update<4, 1>(items, ld, plan, tile_base, n_tiles, t, protos, d2, tsum, s);
    else if (f4 <= 8) launch_update<8, 1>(items, ld, plan, tile_base, n_tiles, t, protos, d2, tsum, s);
    else if (f4 <= 16) launch_update<8, 2>(items, ld, plan, tile_base, n_tiles, t, protos, d2, tsum, s);
    else if (f4 <= 32) launch_update<8, 4>(items, ld, plan, tile_base, n_tiles, t, protos, d2, tsum, s);
    else launch_update<16, 4>(items, ld, plan, tile_base, n_tiles, t, protos, d2, tsum, s);
  }
  check_launch("kmeanspp");
}

}  // namespace mask

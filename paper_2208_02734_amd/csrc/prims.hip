// Data-movement primitives for the build: stable LSD radix sort with
// wavefront ballot ranking, device-wide exclusive scan, SplitMix64 keys for
// the level-0 permutation, row gathers and row norms.
#include "internal.hpp"

namespace mask {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

inline unsigned grid_for(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// ---------------------------------------------------------------- radix sort
// Each wavefront owns a contiguous tile of kRsTile keys.  Pass = (1) per-wave
// digit histogram, (2) exclusive scan of the digit-major histogram table,
// (3) per-wave stable scatter: lanes with equal digits find each other with
// one ballot per digit bit, the lowest such lane advances the wave's running
// offset for that digit.  Keys are processed in order inside a tile and tiles
// in order inside a digit, so each pass is stable.

constexpr int kRsItems = 16;
constexpr int kRsTile = kWave * kRsItems;

template <class K>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const K* __restrict__ keys, int64_t n,
                                                       int shift, int bits,
                                                       uint32_t* __restrict__ hist,
                                                       int64_t n_waves) {
  __shared__ uint32_t h[kWavesPerBlock][256];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nbins = 1 << bits;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  for (int i = lane; i < nbins; i += kWave) h[wave][i] = 0;
  __syncthreads();
  if (gw < n_waves) {
    const int64_t base = gw * kRsTile;
    const uint32_t mask = (uint32_t)nbins - 1;
#pragma unroll 4
    for (int it = 0; it < kRsItems; ++it) {
      int64_t i = base + it * kWave + lane;
      if (i < n) atomicAdd(&h[wave][(uint32_t)(keys[i] >> shift) & mask], 1u);
    }
  }
  __syncthreads();
  if (gw < n_waves)
    for (int d = lane; d < nbins; d += kWave) hist[(int64_t)d * n_waves + gw] = h[wave][d];
}

template <class K>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    K* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t n, int shift, int bits,
    const uint32_t* __restrict__ offsets, int64_t n_waves) {
  __shared__ uint32_t cnt[kWavesPerBlock][256];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nbins = 1 << bits;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const bool wave_active = gw < n_waves;
  if (wave_active)
    for (int d = lane; d < nbins; d += kWave) cnt[wave][d] = offsets[(int64_t)d * n_waves + gw];
  __syncthreads();
  const uint32_t mask = (uint32_t)nbins - 1;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = gw * kRsTile;
  for (int it = 0; it < kRsItems; ++it) {
    const int64_t i = base + it * kWave + lane;
    const bool valid = wave_active && i < n;
    K key = valid ? keys_in[i] : K(0);
    uint32_t val = valid ? vals_in[i] : 0u;
    uint32_t d = (uint32_t)(key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt_mask);
    uint32_t pos = 0;
    if (valid) pos = cnt[wave][d];
    __syncthreads();
    if (valid && rank == 0) cnt[wave][d] = pos + (uint32_t)__popcll(peers);
    if (valid) {
      keys_out[pos + rank] = key;
      vals_out[pos + rank] = val;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------- scan
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

// Exclusive block scan of one value per thread; returns the block total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave, uint32_t& total) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) s_wave[wave] = x;
  __syncthreads();
  uint32_t wave_base = 0, tot = 0;
  for (int w = 0; w < kWavesPerBlock; ++w) {
    if (w < wave) wave_base += s_wave[w];
    tot += s_wave[w];
  }
  __syncthreads();
  total = tot;
  return wave_base + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ data,
                                                        int64_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t s_wave[kWavesPerBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) acc += data[base + j];
  uint32_t total;
  block_exclusive_scan(acc, s_wave, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Single-block exclusive scan of the per-tile sums (any length).
__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t* __restrict__ sums, int64_t n,
                                                      uint32_t* __restrict__ out_total) {
  __shared__ uint32_t s_wave[kWavesPerBlock];
  uint32_t carry = 0;
  for (int64_t t = 0; t < n; t += kScanTile) {
    const int64_t base = t + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = (base + j < n) ? sums[base + j] : 0u;
      acc += v[j];
    }
    uint32_t total;
    uint32_t ex = block_exclusive_scan(acc, s_wave, total) + carry;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      if (base + j < n) sums[base + j] = ex;
      ex += v[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && out_total) *out_total = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(uint32_t* __restrict__ data, int64_t n,
                                                       const uint32_t* __restrict__ sums) {
  __shared__ uint32_t s_wave[kWavesPerBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (base + j < n) ? data[base + j] : 0u;
    acc += v[j];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan(acc, s_wave, total) + sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) data[base + j] = ex;
    ex += v[j];
  }
}

// ---------------------------------------------------------------- small ops
__global__ void k_splitmix(uint64_t seed, int64_t n, uint64_t* __restrict__ keys,
                           uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  keys[i] = z ^ (z >> 31);
  vals[i] = (uint32_t)i;
}

template <class I>
__global__ void k_gather_rows_vec(const float* __restrict__ src, int ld_src,
                                  const I* __restrict__ idx, int64_t n, int dim,
                                  float* __restrict__ dst, int ld_dst) {
  // one thread per float4 of the destination
  const int q4 = ld_dst / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * q4) return;
  const int64_t i = t / q4;
  const int c = (int)(t % q4) * 4;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (c < dim) {
    const int64_t row = idx ? (int64_t)idx[i] : i;
    v = *reinterpret_cast<const float4*>(src + row * ld_src + c);
  }
  *reinterpret_cast<float4*>(dst + i * ld_dst + c) = v;
}

template <class I>
__global__ void k_gather_rows_scalar(const float* __restrict__ src, int ld_src,
                                     const I* __restrict__ idx, int64_t n, int dim,
                                     float* __restrict__ dst, int ld_dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ld_dst) return;
  const int64_t i = t / ld_dst;
  const int c = (int)(t % ld_dst);
  float v = 0.f;
  if (c < dim) {
    const int64_t row = idx ? (int64_t)idx[i] : i;
    v = src[row * ld_src + c];
  }
  dst[i * ld_dst + c] = v;
}

template <class I>
void gather_rows_t(const float* src, int ld_src, const I* idx, int64_t n, int dim, float* dst,
                   int ld_dst, hipStream_t s) {
  if (n <= 0) return;
  const bool vec = (ld_src % 4 == 0) && (dim % 4 == 0) && (ld_dst % 4 == 0) &&
                   ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
  if (vec) {
    const int64_t work = n * (ld_dst / 4);
    k_gather_rows_vec<I><<<grid_for(work, kBlock), kBlock, 0, s>>>(src, ld_src, idx, n, dim, dst,
                                                                  ld_dst);
  } else {
    const int64_t work = n * ld_dst;
    k_gather_rows_scalar<I><<<grid_for(work, kBlock), kBlock, 0, s>>>(src, ld_src, idx, n, dim,
                                                                     dst, ld_dst);
  }
  check_launch("gather_rows");
}

// One thread per row: float32 sum of squares with four interleaved partial
// sums over the float4 lanes, combined as (s0+s1)+(s2+s3).
// G lanes per row, each summing its float4s (columns 4*(gl + G*i)) in four
// partials, then a butterfly over the group: coalesced and in a fixed order.
template <int G>
__global__ void k_row_norms(const float* __restrict__ x, int ld, int64_t n,
                            float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / G;
  const int gl = (int)(t % G);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (i < n) {
    const float4* r = reinterpret_cast<const float4*>(x + i * ld);
    for (int c = gl; c < ld / 4; c += G) {
      const float4 v = r[c];
      s0 = fmaf(v.x, v.x, s0);
      s1 = fmaf(v.y, v.y, s1);
      s2 = fmaf(v.z, v.z, s2);
      s3 = fmaf(v.w, v.w, s3);
    }
  }
  float a = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if (i < n && gl == 0) out[i] = a;
}

__global__ void k_offsets_from_sorted(const uint32_t* __restrict__ keys, int64_t n,
                                      int64_t n_bins, uint32_t* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int64_t lo = (i == 0) ? 0 : (int64_t)keys[i - 1] + 1;
  const int64_t hi = (i == n) ? n_bins : (int64_t)keys[i];
  for (int64_t p = lo; p <= hi; ++p) off[p] = (uint32_t)i;
}

__global__ void k_map_u32(const uint32_t* __restrict__ map, const uint32_t* __restrict__ in,
                          int64_t n, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = map[in[i]];
}
__global__ void k_scatter_iota(const uint32_t* __restrict__ idx, int64_t n,
                               uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[idx[i]] = (uint32_t)i;
}
__global__ void k_iota(uint32_t* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint32_t)i;
}
__global__ void k_fill(uint32_t* __restrict__ out, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

template <class K>
void radix_sort_t(K* keys, uint32_t* vals, int64_t n, int key_bits, SortWork& w,
                  hipStream_t s) {
  if (n <= 1 || key_bits <= 0) return;
  if (n > w.cap_n) throw Error{MASK_ERR_DEVICE, "radix sort workspace too small"};
  if (sizeof(K) == 8 && !w.wide) throw Error{MASK_ERR_DEVICE, "radix sort workspace is 32-bit"};
  const int64_t n_waves = (n + kRsTile - 1) / kRsTile;
  const unsigned blocks = grid_for(n_waves, kWavesPerBlock);
  K* kin = keys;
  uint32_t* vin = vals;
  K* kout = static_cast<K*>(w.keys2);
  uint32_t* vout = w.vals2;
  for (int shift = 0; shift < key_bits; shift += 8) {
    const int bits = (key_bits - shift) < 8 ? (key_bits - shift) : 8;
    k_radix_hist<K><<<blocks, kBlock, 0, s>>>(kin, n, shift, bits, w.hist, n_waves);
    check_launch("radix_hist");
    exclusive_scan_u32(w.hist, (int64_t)(1 << bits) * n_waves, nullptr, w.sums, s);
    k_radix_scatter<K><<<blocks, kBlock, 0, s>>>(kin, vin, kout, vout, n, shift, bits, w.hist,
                                                 n_waves);
    check_launch("radix_scatter");
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  if (kin != keys) {
    MASK_HIP(hipMemcpyAsync(keys, kin, n * sizeof(K), hipMemcpyDeviceToDevice, s));
    MASK_HIP(hipMemcpyAsync(vals, vin, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace

int64_t scan_sums_needed(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* out_total, uint32_t* sums,
                        hipStream_t s) {
  if (n <= 0) return;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  k_scan_reduce<<<(unsigned)tiles, kBlock, 0, s>>>(data, n, sums);
  check_launch("scan_reduce");
  k_scan_sums<<<1, kBlock, 0, s>>>(sums, tiles, out_total);
  check_launch("scan_sums");
  k_scan_apply<<<(unsigned)tiles, kBlock, 0, s>>>(data, n, sums);
  check_launch("scan_apply");
}

void sort_work_alloc(SortWork& w, int64_t n, bool wide, Arena& a) {
  const int64_t n_waves = (n + kRsTile - 1) / kRsTile;
  w.cap_n = n;
  w.wide = wide;
  w.keys2 = a.alloc_bytes((size_t)n * (wide ? 8 : 4));
  w.vals2 = a.alloc<uint32_t>(n);
  w.hist = a.alloc<uint32_t>(256 * n_waves);
  w.sums = a.alloc<uint32_t>(scan_sums_needed(256 * n_waves));
}

int64_t sort_work_carve(SortWork& w, void* base, int64_t n, bool wide) {
  const int64_t n_waves = (n + kRsTile - 1) / kRsTile;
  char* b = static_cast<char*>(base);
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    void* p = b ? b + off : nullptr;
    off += (bytes + 255) & ~int64_t(255);
    return p;
  };
  w.cap_n = n;
  w.wide = wide;
  w.keys2 = take(n * (wide ? 8 : 4));
  w.vals2 = static_cast<uint32_t*>(take(n * 4));
  w.hist = static_cast<uint32_t*>(take(256 * n_waves * 4));
  w.sums = static_cast<uint32_t*>(take(scan_sums_needed(256 * n_waves) * 4));
  return off;
}

void radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int key_bits, SortWork& w,
                    hipStream_t s) {
  radix_sort_t<uint32_t>(keys, vals, n, key_bits, w, s);
}
void radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int key_bits, SortWork& w,
                    hipStream_t s) {
  radix_sort_t<uint64_t>(keys, vals, n, key_bits, w, s);
}

void splitmix_keys(uint64_t seed, int64_t n, uint64_t* keys, uint32_t* vals, hipStream_t s) {
  if (n <= 0) return;
  k_splitmix<<<grid_for(n, kBlock), kBlock, 0, s>>>(seed, n, keys, vals);
  check_launch("splitmix");
}

void gather_rows(const float* src, int ld_src, const uint32_t* idx, int64_t n, int dim,
                 float* dst, int ld_dst, hipStream_t s) {
  gather_rows_t<uint32_t>(src, ld_src, idx, n, dim, dst, ld_dst, s);
}
void gather_rows_i32(const float* src, int ld_src, const int32_t* idx, int64_t n, int dim,
                     float* dst, int ld_dst, hipStream_t s) {
  gather_rows_t<int32_t>(src, ld_src, idx, n, dim, dst, ld_dst, s);
}
void copy_rows(const float* src, int ld_src, int64_t n, int dim, float* dst, int ld_dst,
               hipStream_t s) {
  gather_rows_t<uint32_t>(src, ld_src, nullptr, n, dim, dst, ld_dst, s);
}

void row_norms(const float* x, int ld, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return;
  const int f4 = ld / 4;
  if (f4 <= 4) k_row_norms<4><<<grid_for(n * 4, kBlock), kBlock, 0, s>>>(x, ld, n, out);
  else if (f4 <= 8) k_row_norms<8><<<grid_for(n * 8, kBlock), kBlock, 0, s>>>(x, ld, n, out);
  else k_row_norms<16><<<grid_for(n * 16, kBlock), kBlock, 0, s>>>(x, ld, n, out);
  check_launch("row_norms");
}

void offsets_from_sorted(const uint32_t* keys, int64_t n, int64_t n_bins, uint32_t* off,
                         hipStream_t s) {
  k_offsets_from_sorted<<<grid_for(n + 1, kBlock), kBlock, 0, s>>>(keys, n, n_bins, off);
  check_launch("offsets_from_sorted");
}

namespace {
__global__ void k_check_range_i32(const int32_t* __restrict__ a, int64_t n, int64_t bound,
                                  uint32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (a[i] < 0 || a[i] >= bound)) atomicOr(flag, 1u);
}
}  // namespace

void check_range_i32(const int32_t* a, int64_t n, int64_t bound, uint32_t* flag,
                     hipStream_t s) {
  MASK_HIP(hipMemsetAsync(flag, 0, sizeof(uint32_t), s));
  if (n <= 0) return;
  k_check_range_i32<<<grid_for(n, kBlock), kBlock, 0, s>>>(a, n, bound, flag);
  check_launch("check_range");
}

namespace {
__global__ __launch_bounds__(kBlock) void k_count_changed(const int32_t* __restrict__ a,
                                                          const int32_t* __restrict__ b,
                                                          int64_t n, uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int c = __syncthreads_count(i < n && a[i] != b[i]);
  if (threadIdx.x == 0 && c > 0) atomicAdd(count, (uint32_t)c);
}
}  // namespace

void count_changed(const int32_t* a, const int32_t* b, int64_t n, uint32_t* count,
                   hipStream_t s) {
  MASK_HIP(hipMemsetAsync(count, 0, sizeof(uint32_t), s));
  if (n <= 0) return;
  k_count_changed<<<grid_for(n, kBlock), kBlock, 0, s>>>(a, b, n, count);
  check_launch("count_changed");
}

void map_u32(const uint32_t* map, const uint32_t* in, int64_t n, uint32_t* out, hipStream_t s) {
  if (n <= 0) return;
  k_map_u32<<<grid_for(n, kBlock), kBlock, 0, s>>>(map, in, n, out);
  check_launch("map_u32");
}
void scatter_iota(const uint32_t* idx, int64_t n, uint32_t* out, hipStream_t s) {
  if (n <= 0) return;
  k_scatter_iota<<<grid_for(n, kBlock), kBlock, 0, s>>>(idx, n, out);
  check_launch("scatter_iota");
}
void gather_u32(const uint32_t* src, const uint32_t* idx, int64_t n, uint32_t* out,
                hipStream_t s) {
  map_u32(src, idx, n, out, s);
}
void iota_u32(uint32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_iota<<<grid_for(n, kBlock), kBlock, 0, s>>>(out, n);
  check_launch("iota");
}
void fill_u32(uint32_t* out, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill<<<grid_for(n, kBlock), kBlock, 0, s>>>(out, n, v);
  check_launch("fill");
}

}  // namespace mask

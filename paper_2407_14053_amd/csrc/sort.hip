// Device exclusive scan and stable LSD radix sort (64-wide wavefronts, LDS ranking) for gfx950.
//
// The sort orders each of n_seg equal-length segments independently: block histograms are laid out
// [segment][digit][block-in-segment], so one exclusive scan of the whole histogram array yields, for every
// block and digit, the output position of that block's first item with that digit -- the segment stays
// the most significant key.  Ranking within a block is stable: items are taken in 256-item chunks in
// order, and inside a wavefront the lanes holding the same digit are found with one ballot per digit bit.
#include "dl_internal.h"

namespace dl {
namespace {

constexpr int kThreads = 256;
constexpr int kScanIPT = 16;
constexpr int kScanTile = kThreads * kScanIPT;  // items per scan block
constexpr int kSortIPT = 16;
constexpr int kSortTile = kThreads * kSortIPT;  // items per sort block

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread across a 256-thread block; returns the block total in *total.
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x, lane);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) {
    if (i < w) before += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return before + inc - x;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                                 uint32_t* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t total;
  block_excl_scan(s, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Single block: exclusive scan of the block totals in place; partial[np] receives the grand total.
__global__ __launch_bounds__(kThreads) void scan_partials_kernel(uint32_t* __restrict__ partial, int64_t np) {
  uint32_t carry = 0;
  for (int64_t base = 0; base < np; base += kThreads) {
    const int64_t i = base + threadIdx.x;
    const uint32_t x = i < np ? partial[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan(x, &total);
    if (i < np) partial[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) partial[np] = carry;
}

__global__ __launch_bounds__(kThreads) void scan_down_kernel(const uint32_t* in, uint32_t* out, int64_t n,
                                                               const uint32_t* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
  uint32_t v[kScanIPT];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t run = block_excl_scan(s, &total) + partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

template <typename K>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const K* __restrict__ keys, int64_t seg_len,
                                                                int blocks_per_seg, int shift, int bits,
                                                                uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int radix = 1 << bits;
  const uint32_t dmask = (uint32_t)radix - 1;
  for (int d = threadIdx.x; d < radix; d += kThreads) h[d] = 0;
  __syncthreads();
  const int seg = blockIdx.x / blocks_per_seg;
  const int bis = blockIdx.x - seg * blocks_per_seg;
  const int64_t seg_base = (int64_t)seg * seg_len;
  const int64_t lo = seg_base + (int64_t)bis * kSortTile;
  const int64_t hi = min(lo + (int64_t)kSortTile, seg_base + seg_len);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const uint32_t d = (uint32_t)(keys[i] >> shift) & dmask;
    atomicAdd(&h[d], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += kThreads)
    hist[((int64_t)seg * radix + d) * blocks_per_seg + bis] = h[d];
}

template <typename K>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(const K* __restrict__ kin,
                                                                   const uint32_t* __restrict__ vin,
                                                                   K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                                   int64_t seg_len, int blocks_per_seg, int shift,
                                                                   int bits, const uint32_t* __restrict__ hist) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kThreads / 64][256];
  const int radix = 1 << bits;
  const uint32_t dmask = (uint32_t)radix - 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int seg = blockIdx.x / blocks_per_seg;
  const int bis = blockIdx.x - seg * blocks_per_seg;
  const int64_t seg_base = (int64_t)seg * seg_len;
  const int64_t lo = seg_base + (int64_t)bis * kSortTile;
  const int64_t hi = min(lo + (int64_t)kSortTile, seg_base + seg_len);
  for (int d = threadIdx.x; d < radix; d += kThreads) {
    run[d] = hist[((int64_t)seg * radix + d) * blocks_per_seg + bis];
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) wcnt[i][d] = 0;
  }
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t c = lo; c < hi; c += kThreads) {
    const int64_t idx = c + threadIdx.x;
    const bool valid = idx < hi;
    K key = 0;
    uint32_t val = 0, d = 0;
    if (valid) {
      key = kin[idx];
      val = vin[idx];
      d = (uint32_t)(key >> shift) & dmask;
    }
    uint64_t m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      m &= bit ? bal : ~bal;
    }
    const uint32_t lrank = (uint32_t)__popcll(m & below);
    if (valid && lrank == 0) wcnt[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + lrank;
      for (int i = 0; i < w; ++i) pos += wcnt[i][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    for (int dd = threadIdx.x; dd < radix; dd += kThreads) {
      uint32_t add = 0;
#pragma unroll
      for (int i = 0; i < kThreads / 64; ++i) {
        add += wcnt[i][dd];
        wcnt[i][dd] = 0;
      }
      run[dd] += add;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void lower_bounds_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                                  uint32_t* __restrict__ start, int64_t n_keys) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k > n_keys) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  start[k] = (uint32_t)lo;
}

template <typename K>
bool radix_sort_impl(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t seg_len, int n_seg, int bit_lo, int bit_hi,
                     uint32_t* hist, uint32_t* partial, hipStream_t s, hipError_t* err) {
  *err = hipSuccess;
  const int blocks_per_seg = (int)((seg_len + kSortTile - 1) / kSortTile);
  const int64_t nblocks = (int64_t)blocks_per_seg * n_seg;
  bool flipped = false;
  if (seg_len == 0 || n_seg == 0) return false;
  for (int shift = bit_lo; shift < bit_hi; shift += 8) {
    const int bits = (bit_hi - shift) < 8 ? (bit_hi - shift) : 8;
    const int64_t hsize = (int64_t)n_seg * (1 << bits) * blocks_per_seg;
    K* ki = flipped ? k1 : k0;
    uint32_t* vi = flipped ? v1 : v0;
    K* ko = flipped ? k0 : k1;
    uint32_t* vo = flipped ? v0 : v1;
    hipLaunchKernelGGL(radix_hist_kernel<K>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, ki, seg_len,
                       blocks_per_seg, shift, bits, hist);
    if ((*err = hipGetLastError()) != hipSuccess) return flipped;
    if ((*err = exclusive_scan_u32(hist, hist, hsize, partial, s)) != hipSuccess) return flipped;
    hipLaunchKernelGGL(radix_scatter_kernel<K>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, ki, vi, ko, vo,
                       seg_len, blocks_per_seg, shift, bits, hist);
    if ((*err = hipGetLastError()) != hipSuccess) return flipped;
    flipped = !flipped;
  }
  return flipped;
}

}  // namespace

int64_t scan_partial_count(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partial, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t np = scan_partial_count(n);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)np), dim3(kThreads), 0, s, in, n, partial);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kThreads), 0, s, partial, np);
  hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)np), dim3(kThreads), 0, s, in, out, n, partial);
  return hipGetLastError();
}

int64_t radix_hist_size(int64_t seg_len, int n_seg, int digit_bits) {
  const int64_t bps = (seg_len + kSortTile - 1) / kSortTile;
  return bps * n_seg * (1 << digit_bits);
}

bool radix_sort_u64(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t seg_len, int n_seg, int bit_lo,
                    int bit_hi, uint32_t* hist, uint32_t* partial, hipStream_t s, hipError_t* err) {
  return radix_sort_impl<uint64_t>(k0, v0, k1, v1, seg_len, n_seg, bit_lo, bit_hi, hist, partial, s, err);
}

bool radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t seg_len, int n_seg, int bit_lo,
                    int bit_hi, uint32_t* hist, uint32_t* partial, hipStream_t s, hipError_t* err) {
  return radix_sort_impl<uint32_t>(k0, v0, k1, v1, seg_len, n_seg, bit_lo, bit_hi, hist, partial, s, err);
}

hipError_t launch_lower_bounds(const uint32_t* keys, int64_t n, uint32_t* start, int64_t n_keys, hipStream_t s) {
  hipLaunchKernelGGL(lower_bounds_kernel, dim3((unsigned)((n_keys + 1 + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, s, keys, n, start, n_keys);
  return hipGetLastError();
}

}  // namespace dl

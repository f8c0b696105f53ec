// Device exclusive scan and stable LSD radix sort for gfx950 (64-wide wavefronts, LDS ranking).
//
// Sort structure: n_seg segments of static length seg_len, each sorted independently; the live length of a
// segment may be given on the device (seg_n), so that launches have static grids (graph capture) while the
// work follows the data.  The first pass may also leave out every item with one given key (culled items):
// the kept items of each segment are compacted to its front, their count written on the device, and later
// passes only touch them.  A fixed number of blocks per segment each own one contiguous range of the segment.
// Per pass:
//   hist    : per block, counts of each digit (per-wavefront LDS counters, then summed)
//   scan    : one exclusive scan over hist laid out [segment][digit][block] gives every block's first output
//             position for every digit (the segment stays the most significant key)
//   scatter : per block, 4096-item tiles; each wavefront ranks its quarter of the tile with one ballot per
//             digit bit (stable: lane order, then row order, then wavefront order), the tile is reordered by
//             digit in LDS, and written out as contiguous runs per digit.
#include "dl_internal.h"

namespace dl {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kScanIPT = 16;
constexpr int kScanTile = kThreads * kScanIPT;
constexpr int kRows = 16;                        // rows of 64 items per wavefront per tile
constexpr int kTile = kThreads * kRows;          // 4096 items per tile
// The depth-order range sorts work on views' fronts of a few thousand items: smaller tiles give them more
// workgroups (and less LDS each).
constexpr int kDepthRows = 4;
constexpr int kDepthTile = kThreads * kDepthRows;
constexpr int kMaxBits = 9;    // digit width of the general sorts
constexpr int kPartBits = 10;  // digit width of the tile partition (one pass for up to 1024 tiles per view)
constexpr int kMaxRadix = 1 << kPartBits;

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x, lane);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    if (i < w) before += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return before + inc - x;
}

// The scans take a static length n, or a device length n_mul * *n_dev (<= n; grids are sized for n).  Each
// workgroup owns a tile of kScanTile items, read and written with consecutive lanes on consecutive items.
// BYTES: each input word stands for the sum of its four bytes.
__device__ inline uint32_t scan_item(uint32_t x, bool bytes) {
  return bytes ? (x & 255u) + ((x >> 8) & 255u) + ((x >> 16) & 255u) + (x >> 24) : x;
}

template <bool BYTES>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                                 const uint32_t* __restrict__ n_dev, int n_mul,
                                                                 uint32_t* __restrict__ partial) {
  if (n_dev) n = min(n, (int64_t)n_mul * *n_dev);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n) {  // beyond a device length: nothing to sum
    if (threadIdx.x == 0) partial[blockIdx.x] = 0;
    return;
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const int64_t k = base + i * kThreads + threadIdx.x;
    if (k < n) s += scan_item(in[k], BYTES);
  }
  uint32_t total;
  block_excl_scan(s, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Second half of the scan: each tile adds the totals of the tiles before it (at most a few thousand, summed by
// the workgroup) and scans its own items, staged in LDS so that thread j scans items [16 j, 16 j + 16) of the
// tile (one padding word every 16 keeps those reads free of bank conflicts); the last tile writes the grand
// total to *grand.
template <bool BYTES>
__global__ __launch_bounds__(kThreads) void scan_down_kernel(const uint32_t* in, uint32_t* out, int64_t n,
                                                               const uint32_t* __restrict__ n_dev, int n_mul,
                                                               const uint32_t* __restrict__ partial_in,
                                                               uint32_t* __restrict__ grand) {
  __shared__ uint32_t st[kScanTile + kScanTile / kScanIPT];
  if (n_dev) n = min(n, (int64_t)n_mul * *n_dev);
  const int64_t np = (n + kScanTile - 1) / kScanTile;
  if ((int64_t)blockIdx.x >= np) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *grand = 0;  // nothing to scan
    return;
  }
  uint32_t pre = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kThreads) pre += partial_in[i];
  uint32_t prefix;
  block_excl_scan(pre, &prefix);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  auto pad = [](int j) { return j + (j >> 4); };
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const int j = i * kThreads + threadIdx.x;
    st[pad(j)] = base + j < n ? scan_item(in[base + j], BYTES) : 0u;
  }
  __syncthreads();
  uint32_t v[kScanIPT];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    v[i] = st[pad(threadIdx.x * kScanIPT + i)];
    s += v[i];
  }
  uint32_t total;
  uint32_t run = block_excl_scan(s, &total) + prefix;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    st[pad(threadIdx.x * kScanIPT + i)] = run;
    run += v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const int j = i * kThreads + threadIdx.x;
    if (base + j < n) out[base + j] = st[pad(j)];
  }
  if ((int64_t)blockIdx.x == np - 1 && threadIdx.x == 0) *grand = prefix + total;
}

// Range [lo, hi) of block `bis` within a segment whose live length is n (ranges are whole tiles).
__device__ inline void block_range(int64_t n, int bps, int bis, int64_t& lo, int64_t& hi, int tile) {
  int64_t per = (n + bps - 1) / bps;
  per = (per + tile - 1) / tile * tile;
  lo = min((int64_t)bis * per, n);
  hi = min(lo + per, n);
}

template <typename K>
struct SortArgs {
  const K* kin;
  const uint32_t* vin;
  K* kout;                // nullptr: keys are not written (the last pass of a partition)
  uint32_t* vout;
  int64_t seg_len;
  const uint32_t* seg_n;  // device live lengths (nullptr: seg_len)
  uint32_t cap;           // clamp of device lengths and range ends
  int bps;                // blocks per segment (the maximum, with device ranges)
  int shift, bits;
  uint32_t* hist;
  int drop;               // this pass leaves out items whose key equals drop_key
  K drop_key;
  const K* split;         // one-bit digit: key >= split[seg] (instead of a bit field of the key)
  // device ranges: segment s is [seg_lo[s], seg_hi[s]) (clamped to cap) of one array, sorted in place; the
  // histogram is laid out [segment][digit < ndig][block < bpse[s]] from ndig * pb[s] (pb = exclusive prefix of
  // bpse), so empty segments take no entries and no blocks.  nullptr: segment s is
  // [s * seg_len, s * seg_len + live length).
  const uint32_t* seg_lo;
  const uint32_t* seg_hi;
  const uint32_t* pb;
  const uint32_t* bpse;
  int ndig;
  int iota;  // the values are the items' positions in their segment (vin is not read)
};

template <typename K>
__device__ inline int64_t hist_at(const SortArgs<K>& a, int seg, int d, int bis, int bps, int radix) {
  return a.seg_lo ? (int64_t)a.ndig * a.pb[seg] + (int64_t)d * bps + bis : ((int64_t)seg * radix + d) * a.bps + bis;
}

template <typename K>
__device__ inline int64_t live_len(const SortArgs<K>& a, int seg) {
  if (!a.seg_n) return a.seg_len;
  return min((int64_t)min(a.seg_n[seg], a.cap), a.seg_len);
}

// Input range [base, base + n) of segment `seg`; output goes to the same range.
template <typename K>
__device__ inline void seg_range(const SortArgs<K>& a, int seg, int64_t& base, int64_t& n) {
  if (a.seg_lo) {
    base = min(a.seg_lo[seg], a.cap);
    n = max((int64_t)0, (int64_t)min(a.seg_hi[seg], a.cap) - base);
  } else {
    base = (int64_t)seg * a.seg_len;
    n = live_len(a, seg);
  }
}

template <typename K>
__device__ inline uint32_t digit_of(const SortArgs<K>& a, int seg, K k, uint32_t dmask) {
  return a.split ? (uint32_t)(k >= a.split[seg]) : (uint32_t)(k >> a.shift) & dmask;
}

template <typename K, int RB, int ROWS>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(SortArgs<K> a) {
  __shared__ uint32_t h[kWaves][1 << RB];
  const int radix = 1 << a.bits;
  const uint32_t dmask = (uint32_t)radix - 1;
  const int w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < radix; d += kThreads)
#pragma unroll
    for (int i = 0; i < kWaves; ++i) h[i][d] = 0;
  __syncthreads();
  const int seg = blockIdx.x / a.bps;
  const int bis = blockIdx.x - seg * a.bps;
  const int bps = a.seg_lo ? (int)a.bpse[seg] : a.bps;
  if (bis >= bps) return;
  const int ndig = a.seg_lo ? a.ndig : radix;
  int64_t base, n, lo, hi;
  seg_range(a, seg, base, n);
  block_range(n, bps, bis, lo, hi, kThreads * ROWS);
  const K* kin = a.kin + base;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const K k = kin[i];
    if (a.drop && k == a.drop_key) continue;
    atomicAdd(&h[w][digit_of(a, seg, k, dmask)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < ndig; d += kThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s += h[i][d];
    a.hist[hist_at(a, seg, d, bis, bps, radix)] = s;
  }
}

// ROWS rows of 64 items per wavefront make a tile of kThreads * ROWS items (the unit of the block ranges).
template <typename K, int RB, int ROWS>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(SortArgs<K> a) {
  constexpr int kTile = kThreads * ROWS;
  constexpr int kRows = ROWS;
  constexpr int DPT = (1 << RB) / kThreads;     // digits owned by each thread in the tile-local scan
  __shared__ uint32_t run[1 << RB];             // next output position per digit
  __shared__ uint32_t wc[kWaves][1 << RB];      // per-wavefront digit counts within the tile
  __shared__ uint32_t loff[1 << RB];            // tile-local start per digit
  __shared__ K skey[kTile];
  __shared__ uint32_t sval[kTile];
  const int radix = 1 << a.bits;
  const uint32_t dmask = (uint32_t)radix - 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int seg = blockIdx.x / a.bps;
  const int bis = blockIdx.x - seg * a.bps;
  const int bps = a.seg_lo ? (int)a.bpse[seg] : a.bps;
  if (bis >= bps) return;
  const int ndig = a.seg_lo ? a.ndig : radix;
  int64_t base, n, lo, hi;
  seg_range(a, seg, base, n);
  block_range(n, bps, bis, lo, hi, kTile);
  const K* kin = a.kin + base;
  const uint32_t* vin = a.vin + base;
  K* kout = a.kout ? a.kout + base : nullptr;
  uint32_t* vout = a.vout + base;
  // the scan runs over all segments; subtract the segment's first offset so positions are segment-relative
  const uint32_t seg0 = a.hist[a.seg_lo ? (int64_t)a.ndig * a.pb[seg] : (int64_t)seg * radix * a.bps];
  for (int d = threadIdx.x; d < radix; d += kThreads)
    run[d] = d < ndig ? a.hist[hist_at(a, seg, d, bis, bps, radix)] - seg0 : 0u;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  for (int64_t t0 = lo; t0 < hi; t0 += kTile) {
    const int tn = (int)min((int64_t)kTile, hi - t0);
    for (int d = threadIdx.x; d < radix; d += kThreads)
#pragma unroll
      for (int i = 0; i < kWaves; ++i) wc[i][d] = 0;
    __syncthreads();
    // wavefront w ranks items [w * 1024, (w + 1) * 1024) of the tile, 64 at a time, in order
    K key[kRows];
    uint32_t val[kRows], dig[kRows], rnk[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int li = w * (kRows * 64) + r * 64 + lane;
      bool valid = li < tn;
      key[r] = valid ? kin[t0 + li] : (K)0;
      val[r] = valid ? (a.iota ? (uint32_t)(t0 + li) : vin[t0 + li]) : 0u;
      if (a.drop && key[r] == a.drop_key) valid = false;
      const uint32_t d = digit_of(a, seg, key[r], dmask);
      dig[r] = d;
      uint64_t m = __ballot(valid);
      for (int b = 0; b < a.bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
      }
      const uint32_t lr = (uint32_t)__popcll(m & below);
      const uint32_t base = valid ? wc[w][d] : 0u;
      rnk[r] = valid ? base + lr : 0xffffffffu;
      if (valid && lr == 0) wc[w][d] = base + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // tile-local digit offsets (exclusive scan over digits; thread t owns digits [DPT t, DPT t + DPT)) and
    // per-wavefront bases
    uint32_t tot[DPT];
    uint32_t mysum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int d = DPT * threadIdx.x + q;
      tot[q] = 0;
      if (d < radix) {
#pragma unroll
        for (int i = 0; i < kWaves; ++i) tot[q] += wc[i][d];
      }
      mysum += tot[q];
    }
    uint32_t total;
    uint32_t acc_d = block_excl_scan(mysum, &total);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int d = DPT * threadIdx.x + q;
      if (d < radix) {
        loff[d] = acc_d;
        uint32_t acc = acc_d;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) {
          const uint32_t c = wc[i][d];
          wc[i][d] = acc;  // becomes the tile-local base of wavefront i for this digit
          acc += c;
        }
      }
      acc_d += tot[q];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      if (rnk[r] != 0xffffffffu) {
        const uint32_t p = wc[w][dig[r]] + rnk[r];
        skey[p] = key[r];
        sval[p] = val[r];
      }
    }
    __syncthreads();
    // contiguous runs per digit: consecutive lanes write consecutive addresses (`total` = kept items)
    for (int p = threadIdx.x; p < (int)total; p += kThreads) {
      const K k = skey[p];
      const uint32_t d = digit_of(a, seg, k, dmask);
      const uint32_t g = run[d] + (uint32_t)p - loff[d];
      if (kout) kout[g] = k;
      vout[g] = sval[p];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int d = DPT * threadIdx.x + q;
      if (d < radix) run[d] += tot[q];
    }
    __syncthreads();
  }
}

// List starts of a one-pass partition: the first output position of digit t in segment v is the segment's
// start plus the scanned histogram at [v][t][block 0] less the segment's first entry (an empty segment has no
// entries: its lists start at its range); start[n_seg * n_dig] = end of the last segment.
__global__ __launch_bounds__(kThreads) void hist_starts_kernel(const uint32_t* __restrict__ hist,
                                                                 const uint32_t* __restrict__ pb,
                                                                 const uint32_t* __restrict__ bpse, int n_dig,
                                                                 int n_seg, const uint32_t* __restrict__ seg_lo,
                                                                 const uint32_t* __restrict__ seg_hi, uint32_t cap,
                                                                 uint32_t* __restrict__ start) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t n = (int64_t)n_seg * n_dig;
  if (i > n) return;
  if (i == n) {
    start[i] = min(seg_hi[n_seg - 1], cap);
    return;
  }
  const int v = (int)(i / n_dig);
  const int t = (int)(i - (int64_t)v * n_dig);
  const uint32_t b = bpse[v];
  const uint32_t lo = min(seg_lo[v], cap);
  const int64_t h0 = (int64_t)n_dig * pb[v];
  start[i] = b ? lo + (hist[h0 + (int64_t)t * b] - hist[h0]) : lo;
}

// Histogram layout over device ranges (one workgroup, n_seg <= kThreads): blocks per segment = its tiles of kTile
// items (at most bps_max, none for an empty segment) and their exclusive prefix pb (pb[n_seg] = total blocks).
__device__ inline void range_layout(const uint32_t* __restrict__ seg_lo, const uint32_t* __restrict__ seg_hi,
                                    uint32_t cap, int n_seg, int bps_max, uint32_t* __restrict__ bpse,
                                    uint32_t* __restrict__ pb, int tile = kTile) {
  const int v = threadIdx.x;
  uint32_t b = 0;
  if (v < n_seg) {
    const uint32_t lo = min(seg_lo[v], cap), hi = min(seg_hi[v], cap);
    const uint32_t n = hi > lo ? hi - lo : 0u;
    b = (uint32_t)min((int64_t)bps_max, ((int64_t)n + tile - 1) / tile);
    bpse[v] = b;
  }
  uint32_t total;
  const uint32_t off = block_excl_scan(b, &total);
  if (v < n_seg) pb[v] = off;
  if (v == 0) pb[n_seg] = total;
}

__global__ __launch_bounds__(kThreads) void part_layout_kernel(const uint32_t* __restrict__ seg_lo,
                                                                 const uint32_t* __restrict__ seg_hi, uint32_t cap,
                                                                 int n_seg, int bps_max, uint32_t* __restrict__ bpse,
                                                                 uint32_t* __restrict__ pb, int tile) {
  range_layout(seg_lo, seg_hi, cap, n_seg, bps_max, bpse, pb, tile);
}

// List starts after a multi-pass partition: first position in segment v whose key is >= t.
__global__ __launch_bounds__(kThreads) void segment_bounds_kernel(const uint32_t* __restrict__ keys, int n_dig,
                                                                    int n_seg, const uint32_t* __restrict__ seg_lo,
                                                                    const uint32_t* __restrict__ seg_hi, uint32_t cap,
                                                                    uint32_t* __restrict__ start) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t n = (int64_t)n_seg * n_dig;
  if (i > n) return;
  if (i == n) {
    start[i] = min(seg_hi[n_seg - 1], cap);
    return;
  }
  const int v = (int)(i / n_dig);
  const uint32_t t = (uint32_t)(i - (int64_t)v * n_dig);
  uint32_t lo = min(seg_lo[v], cap), hi = max(lo, min(seg_hi[v], cap));
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  start[i] = lo;
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per depth chunk, one workgroup (N <= kThreads): the start of each view's key range (the scanned wavefront counts
// at the view's first slot; the end of the last view is the chunk's total), the largest total seen (overflow
// check), and the tile partition's histogram layout over these ranges.
__global__ __launch_bounds__(kThreads) void chunk_setup_kernel(const uint32_t* __restrict__ scanned, int64_t wstride,
                                                                 int N, const unsigned long long* __restrict__ total,
                                                                 unsigned long long* __restrict__ max_total,
                                                                 uint32_t cap, int bps_max,
                                                                 uint32_t* __restrict__ start,
                                                                 uint32_t* __restrict__ bpse,
                                                                 uint32_t* __restrict__ pb) {
  const int v = threadIdx.x;
  const unsigned long long t = *total;
  if (v < N) start[v] = scanned[(int64_t)v * wstride];
  if (v == 0) {
    start[N] = (uint32_t)(t < 0xffffffffull ? t : 0xffffffffull);
    if (t > *max_total) *max_total = t;
  }
  __syncthreads();
  range_layout(start, start + 1, cap, N, bps_max, bpse, pb);
}

// ---- the front of each view's depth order ----
// The projection counts a sample of each view's visible keys (Gaussians i with i mod kFrontSamplePeriod <
// kFrontSampleRun) on their top kFrontBits bits.  The threshold only steers how much goes into the first chunk;
// the exact front sizes come from the gather (or split) pass.
constexpr int kFrontBins = 1 << kFrontBits;

// The threshold of one view (a whole workgroup of kThreads calls it): the smallest bin b whose cumulative sample
// count reaches ceil(n_s num / den) of the n_s sampled keys; the front is every key below
// thr = (b + 1) << (key_bits - kFrontBits) (0: none).
__device__ uint64_t front_threshold(const uint32_t* __restrict__ h, int key_bits, int64_t num, int64_t den) {
  constexpr int kPer = kFrontBins / kThreads;
  __shared__ unsigned long long th_s;
  uint32_t c[kPer];
  uint32_t mine = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    c[i] = h[threadIdx.x * kPer + i];
    mine += c[i];
  }
  if (threadIdx.x == 0) th_s = 0;
  uint32_t n;
  uint32_t run = block_excl_scan(mine, &n);  // its barriers order the reset before the store below
  const uint32_t target = (uint32_t)(((int64_t)n * num + den - 1) / den);
  if (target > 0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t before = run;
      run += c[i];
      if (before < target && run >= target)  // one thread: the count is monotone
        th_s = (unsigned long long)(threadIdx.x * kPer + i + 1) << (key_bits - kFrontBits);
    }
  }
  __syncthreads();
  const uint64_t th = th_s;
  __syncthreads();  // every thread has read it before a later call resets it
  return th;
}

// Per view (one workgroup each): thr[v] = front_threshold of its histogram.
__global__ __launch_bounds__(kThreads) void front_select_kernel(const uint32_t* __restrict__ hist, int key_bits,
                                                                  int64_t num, int64_t den,
                                                                  uint64_t* __restrict__ thr) {
  const int v = blockIdx.x;
  const uint64_t th = front_threshold(hist + (int64_t)v * kFrontBins, key_bits, num, den);
  if (threadIdx.x == 0) thr[v] = th;
}

// Exact sizes after the split pass, from its scanned histogram ([segment][digit 0, 1][block], exclusive) and the
// scan's grand total: n_vis = kept items, n_front = items of digit 0.
// ---- the depth split ----
// One stable pass drops each view's culled items and puts its front (keys below the view's threshold) before
// its back.  Each wavefront owns a contiguous run of its view's items, runs in view order; the histogram holds,
// per view, the kept fronts of every wavefront, then the kept backs ([view][2][wavefront]), so that after one
// scan each wavefront streams its items straight into the two output runs, ranked by ballots: stable, with no
// LDS staging.  The values are the items' positions in their view (Gaussian indices).
__device__ inline void split_range(int64_t G, int wps, int k, int64_t& lo, int64_t& hi) {
  int64_t per = (G + wps - 1) / wps;
  per = (per + 63) / 64 * 64;
  lo = min((int64_t)k * per, G);
  hi = min(lo + per, G);
}

__device__ inline uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__global__ __launch_bounds__(kThreads) void split_hist_kernel(const uint64_t* __restrict__ keys, int64_t G, int wps,
                                                                const uint64_t* __restrict__ thr, uint64_t drop,
                                                                const uint32_t* __restrict__ live,
                                                                uint32_t* __restrict__ hist) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int v = (int)(gw / wps), k = (int)(gw - (int64_t)v * wps);
  int64_t lo, hi;
  split_range(G, wps, k, lo, hi);
  if (live && !live[v]) hi = lo;  // a view left out: no items
  const uint64_t* kin = keys + (int64_t)v * G;
  const uint64_t th = thr[v];
  uint32_t c0 = 0, c1 = 0;
  int64_t i = lo + lane;
  for (; i + 192 < hi; i += 256) {  // four independent loads in flight
    const uint64_t k0 = kin[i], k1 = kin[i + 64], k2 = kin[i + 128], k3 = kin[i + 192];
    c0 += (k0 != drop && k0 < th) + (k1 != drop && k1 < th) + (k2 != drop && k2 < th) + (k3 != drop && k3 < th);
    c1 += (k0 != drop && k0 >= th) + (k1 != drop && k1 >= th) + (k2 != drop && k2 >= th) + (k3 != drop && k3 >= th);
  }
  for (; i < hi; i += 64) {
    const uint64_t k0 = kin[i];
    c0 += k0 != drop && k0 < th;
    c1 += k0 != drop && k0 >= th;
  }
  c0 = wave_sum_u32(c0);
  c1 = wave_sum_u32(c1);
  if (lane == 0) {
    hist[(int64_t)v * 2 * wps + k] = c0;
    hist[((int64_t)v * 2 + 1) * wps + k] = c1;
  }
}

__global__ __launch_bounds__(kThreads) void split_scatter_kernel(const uint64_t* __restrict__ keys, int64_t G,
                                                                   int wps, const uint64_t* __restrict__ thr,
                                                                   uint64_t drop, const uint32_t* __restrict__ live,
                                                                   bool back_only, const uint32_t* __restrict__ hist,
                                                                   uint64_t* __restrict__ kout,
                                                                   uint32_t* __restrict__ vout) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int v = (int)(gw / wps), k = (int)(gw - (int64_t)v * wps);
  if (live && !live[v]) return;
  int64_t lo, hi;
  split_range(G, wps, k, lo, hi);
  const uint64_t* kin = keys + (int64_t)v * G;
  uint64_t* ko = kout + (int64_t)v * G;
  uint32_t* vo = vout + (int64_t)v * G;
  const uint64_t th = thr[v];
  // the scan runs over all views: positions are relative to the view's first entry
  const uint32_t seg0 = hist[(int64_t)v * 2 * wps];
  uint32_t p0 = hist[(int64_t)v * 2 * wps + k] - seg0;        // next front slot
  uint32_t p1 = hist[((int64_t)v * 2 + 1) * wps + k] - seg0;  // next back slot
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int64_t i0 = lo; i0 < hi; i0 += 128) {
    // two rows of 64 items side by side, written in order
    const int64_t ia = i0 + lane, ib = i0 + 64 + lane;
    const uint64_t ka = ia < hi ? kin[ia] : drop, kb = ib < hi ? kin[ib] : drop;
    const bool fa = ka != drop && ka < th, ba = ka != drop && ka >= th;
    const bool fb = kb != drop && kb < th, bb = kb != drop && kb >= th;
    const uint64_t mfa = __ballot(fa), mba = __ballot(ba), mfb = __ballot(fb), mbb = __ballot(bb);
    if ((fa && !back_only) || ba) {
      const uint32_t at = fa ? p0 + (uint32_t)__popcll(mfa & below) : p1 + (uint32_t)__popcll(mba & below);
      ko[at] = ka;
      vo[at] = (uint32_t)ia;
    }
    p0 += (uint32_t)__popcll(mfa);
    p1 += (uint32_t)__popcll(mba);
    if ((fb && !back_only) || bb) {
      const uint32_t at = fb ? p0 + (uint32_t)__popcll(mfb & below) : p1 + (uint32_t)__popcll(mbb & below);
      ko[at] = kb;
      vo[at] = (uint32_t)ib;
    }
    p0 += (uint32_t)__popcll(mfb);
    p1 += (uint32_t)__popcll(mbb);
  }
}

__global__ void split_counts_kernel(const uint32_t* __restrict__ hist, const uint32_t* __restrict__ grand, int n_seg,
                                    int bps, const uint32_t* __restrict__ live, uint32_t* __restrict__ n_vis,
                                    uint32_t* __restrict__ n_front) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_seg || (live && !live[v])) return;
  const uint32_t a = hist[(int64_t)v * 2 * bps];
  const uint32_t b = hist[((int64_t)v * 2 + 1) * bps];
  const uint32_t c = v + 1 < n_seg ? hist[(int64_t)(v + 1) * 2 * bps] : *grand;
  n_vis[v] = c - a;
  n_front[v] = b - a;
}

// The first chunk's part of the split: each wavefront keeps its run's front items (not dropped, key below the
// view's threshold), in order, at the start of that run in `kout`, each packed as key << 24 | position in the view
// (36 + 24 bits), and counts them and its kept items: cnt[2 v wps + k] = fronts, cnt[(2 v + 1) wps + k] = kept,
// for run k of view v.  Every workgroup (four runs of one view, wps a multiple of four) picks the view's
// threshold from its sampled histogram itself, and the view's first writes it to thr[v].  The front sort gathers
// the runs; the backs are split only when a later chunk needs them.
__global__ __launch_bounds__(kThreads) void front_gather_kernel(const uint64_t* __restrict__ keys, int64_t G, int wps,
                                                                  const uint32_t* __restrict__ hist, int key_bits,
                                                                  int64_t num, int64_t den,
                                                                  uint64_t* __restrict__ thr, uint64_t drop,
                                                                  uint64_t* __restrict__ kout,
                                                                  uint32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int v = (int)(gw / wps), k = (int)(gw - (int64_t)v * wps);
  const uint64_t th = front_threshold(hist + (int64_t)v * kFrontBins, key_bits, num, den);
  if (k == 0 && lane == 0) thr[v] = th;
  int64_t lo, hi;
  split_range(G, wps, k, lo, hi);
  const uint64_t* kin = keys + (int64_t)v * G;
  uint64_t* ko = kout + (int64_t)v * G + lo;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t p = 0, kept = 0;
  for (int64_t i0 = lo; i0 < hi; i0 += 256) {
    uint64_t kk[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // four independent loads in flight
      const int64_t i = i0 + 64 * r + lane;
      kk[r] = i < hi ? kin[i] : drop;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool in = kk[r] != drop, fr = in && kk[r] < th;
      const uint64_t m = __ballot(fr);
      if (fr) ko[p + (uint32_t)__popcll(m & below)] = (kk[r] << 24) | (uint64_t)(i0 + 64 * r + lane);
      p += (uint32_t)__popcll(m);
      kept += (uint32_t)__popcll(__ballot(in));
    }
  }
  if (lane == 0) {
    cnt[(int64_t)v * 2 * wps + k] = p;
    cnt[((int64_t)v * 2 + 1) * wps + k] = kept;
  }
}

// Device ranges of the depth sorts (one workgroup, N <= kThreads): front [v G, v G + f_v); back
// [v G + f_v, v G + n_v) for views with a live tile, empty otherwise; rank_hi = end rank of the range; and the
// sort's histogram layout over these ranges.
__global__ __launch_bounds__(kThreads) void depth_ranges_kernel(int N, int64_t G, const uint32_t* __restrict__ n_vis,
                                                                  const uint32_t* __restrict__ n_front,
                                                                  const uint32_t* __restrict__ live,
                                                                  uint32_t* __restrict__ lo, uint32_t* __restrict__ hi,
                                                                  uint32_t* __restrict__ rank_hi, int bps_max,
                                                                  uint32_t* __restrict__ bpse,
                                                                  uint32_t* __restrict__ pb) {
  const int v = threadIdx.x;
  if (v < N) {
    const uint32_t base = (uint32_t)((int64_t)v * G);
    if (!live) {
      lo[v] = base;
      hi[v] = base + n_front[v];
      rank_hi[v] = n_front[v];
    } else {
      const uint32_t e = live[v] ? n_vis[v] : n_front[v];
      lo[v] = base + n_front[v];
      hi[v] = base + e;
      rank_hi[v] = e;
    }
  }
  __syncthreads();
  range_layout(lo, hi, 0xffffffffu, N, bps_max, bpse, pb, kDepthTile);
}

__global__ __launch_bounds__(kThreads) void lower_bounds_kernel(const uint32_t* __restrict__ keys,
                                                                  const uint32_t* __restrict__ n_dev, uint32_t cap,
                                                                  int64_t n_static, uint32_t* __restrict__ start,
                                                                  int64_t n_keys, int shift) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k > n_keys) return;
  const int64_t n = n_dev ? (int64_t)min(*n_dev, cap) : n_static;
  const int64_t ks = k << shift;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < ks) lo = mid + 1;
    else hi = mid;
  }
  start[k] = (uint32_t)lo;
}

// ---- depth order of small fronts: a few workgroups per view sort the view's front in LDS ----
// The front of a view (its nearest visible Gaussians, left by the gather pass at the starts of the view's runs as
// key << 24 | index, each run in Gaussian index order) is split into `parts` ranges of the key's top 12 bits at
// quantiles of the projection's sampled histogram; each part's workgroup loads the front in index order, keeps its
// range's items (also in index order) in LDS, sorts them by four stable LSD passes of 9 bits over the key bits,
// and writes them after the items of the lower ranges, which gives the order by (depth key, index) of the device
// passes.  Wavefront w owns the contiguous items [w R, (w + 1) R) (R a multiple of 64), visited in slots of 64
// consecutive items; a lane's rank among the equal digits of its slot comes from a match mask of nine ballots, its
// rank in the wavefront from a running count per (digit, wavefront), and the scatter position from the exclusive
// scan of those counts in (digit, wavefront) order.  A front larger than the LDS holds is sorted by its first
// part alone, after a cut at a bin of the key's top 12 bits (an exact histogram of the front): only the items
// below that bin are collected, the view's threshold is lowered to the bin's start, and the others belong to the
// back, which a later split pass takes from the projection's keys with that threshold.
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kFsThreads = 1024;
constexpr int kFsWaves = kFsThreads / 64;
constexpr int kFsSlots = 12;
constexpr int kFsCap = kFsThreads * kFsSlots;  // 12288 items
static_assert(kFsCap == kFrontSortCap, "the declared front capacity");
constexpr int kFsBits = 9;
constexpr int kFsBins = 1 << kFsBits;
constexpr int kFsCutBins = 4096;  // the top 12 bits of the 36-bit key
// The pass counters of (digit d, wavefront w) live at d kFsStride + w: rows padded to an odd stride, so that the
// leaders of different digits and the scan's threads reach different LDS banks (a stride of 16 put every digit
// on two banks).
constexpr int kFsStride = kFsWaves + 1;
constexpr int kFsCntSize = kFsBins * kFsStride;
constexpr int kFsMaxRuns = kFsBins * kFsWaves;  // gather runs per view (their offsets live in the count array)
constexpr int kFsRunsPerThread = kFsMaxRuns / kFsThreads;
static_assert(kFsBins * kFsWaves >= kFsCutBins, "the cut histogram shares the count array");
static_assert(kFsWaves == 16 && kFsThreads * 8 == kFsBins * kFsWaves, "eight (digit, wavefront) counters per thread");
static_assert(kFsCutBins == 4 * kFsThreads, "four cut bins per thread");
static_assert(kFsCutBins == kFrontBins, "the parts' bins are the sampled histogram's");
static_assert(kDepthKeyBits == 4 * kFsBits, "four passes cover the depth key");

struct FrontSortSmem {
  unsigned long long items[kFsCap];
  uint32_t cnt[kFsCntSize];
  uint32_t wsum[kFsWaves];
  uint32_t misc[2];
};

// Exclusive prefix over the workgroup of one value per thread, in thread order (all threads must call it);
// *total (if given) receives the workgroup's sum.
__device__ inline uint32_t fs_block_scan(uint32_t x, uint32_t* wsum, uint32_t* total = nullptr) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t base = 0, all = 0;
  for (int k = 0; k < kFsWaves; ++k) {
    base += k < w ? wsum[k] : 0u;
    all += wsum[k];
  }
  __syncthreads();
  if (total) *total = all;
  return base + inc - x;
}

// The runs of a view: run k starts at item min(k per, G) (as split_range has it); the gather pass left the run's
// fronts there.
__device__ inline int64_t fs_run_len(int64_t G, int wps) {
  int64_t lo, hi;
  split_range(G, wps, 1, lo, hi);
  return lo;  // min(per, G): either way min(k lo, G) is run k's start
}
__device__ inline int64_t fs_run_start(int64_t G, int64_t per, int k) { return min((int64_t)k * per, G); }


// The bin of a packed item (key << 24 | index): the key's top 12 bits.
__device__ inline uint32_t fs_bin(uint64_t it) { return (uint32_t)(it >> 48) & (kFsCutBins - 1); }

// A front of f > kFsCap items (runs of cf[k] items): the largest bin `cut` of the top 12 key bits such that the
// items of the bins below it fit; those are written to sm.items in index order and their count returned, and
// *thr_v becomes cut << 24.
__device__ uint32_t fs_cut_runs(FrontSortSmem& sm, const uint64_t* items, int64_t base, int64_t G, int wps,
                                int64_t per, const uint32_t* cf, uint64_t* thr_v) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int b = t; b < kFsCutBins; b += kFsThreads) sm.cnt[b] = 0;
  if (t == 0) sm.misc[0] = sm.misc[1] = 0;
  __syncthreads();
  for (int k = w; k < wps; k += kFsWaves) {
    const int64_t r0 = base + fs_run_start(G, per, k);
    const uint32_t c = cf[k];
    for (uint32_t i = lane; i < c; i += 64) atomicAdd(&sm.cnt[fs_bin(items[r0 + i])], 1u);
  }
  __syncthreads();
  // bin b holds cnt[b]; thread t owns bins 4t .. 4t + 3; `below` = items in the bins below the current one
  uint32_t c4[4], loc = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c4[k] = sm.cnt[4 * t + k];
    loc += c4[k];
  }
  uint32_t below = fs_block_scan(loc, sm.wsum);
  uint32_t best = 0, best_n = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (below <= (uint32_t)kFsCap) {  // keeping the bins below 4t + k keeps `below` items
      best = 4 * t + k;
      best_n = below;
    }
    below += c4[k];
  }
  // the largest such bin (the item counts below are non-decreasing in the bin)
  atomicMax(&sm.misc[0], best);
  __syncthreads();
  const uint32_t cut = sm.misc[0];
  if (best == cut && best_n <= (uint32_t)kFsCap) sm.misc[1] = best_n;  // the owner of bin `cut` (one thread)
  __syncthreads();
  const uint32_t kept_total = sm.misc[1];
  // kept items per run (the histogram is no longer read), then their offsets in run order
  for (int k = w; k < wps; k += kFsWaves) {
    const int64_t r0 = base + fs_run_start(G, per, k);
    const uint32_t c = cf[k];
    uint32_t n = 0;
    for (uint32_t i0 = 0; i0 < c; i0 += 64) {
      const uint32_t i = i0 + lane;
      n += (uint32_t)__popcll(__ballot(i < c && fs_bin(items[r0 + i]) < cut));
    }
    if (lane == 0) sm.cnt[k] = n;
  }
  __syncthreads();
  uint32_t e[kFsRunsPerThread], mine = 0;
#pragma unroll
  for (int q = 0; q < kFsRunsPerThread; ++q) {
    const int k = t * kFsRunsPerThread + q;
    e[q] = k < wps ? sm.cnt[k] : 0u;
    mine += e[q];
  }
  uint32_t run = fs_block_scan(mine, sm.wsum);
#pragma unroll
  for (int q = 0; q < kFsRunsPerThread; ++q) {
    const int k = t * kFsRunsPerThread + q;
    if (k < wps) sm.cnt[k] = run;
    run += e[q];
  }
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int k = w; k < wps; k += kFsWaves) {
    const int64_t r0 = base + fs_run_start(G, per, k);
    const uint32_t c = cf[k];
    uint32_t o = sm.cnt[k];
    for (uint32_t i0 = 0; i0 < c; i0 += 64) {
      const uint32_t i = i0 + lane;
      const uint64_t it = i < c ? items[r0 + i] : 0ull;
      const bool keep = i < c && fs_bin(it) < cut;
      const uint64_t m = __ballot(keep);
      if (keep) sm.items[o + (uint32_t)__popcll(m & lt)] = it;
      o += (uint32_t)__popcll(m);
    }
  }
  if (t == 0) *thr_v = (uint64_t)cut << 24;
  __syncthreads();
  return kept_total;
}

__global__ __launch_bounds__(kFsThreads) void front_sort_kernel(const uint64_t* __restrict__ items,
                                                                 uint32_t* __restrict__ vals, int64_t G, int wps,
                                                                 int N, int parts, const uint32_t* __restrict__ cnt,
                                                                 const uint32_t* __restrict__ fhist,
                                                                 uint64_t* __restrict__ thr,
                                                                 uint32_t* __restrict__ n_vis,
                                                                 uint32_t* __restrict__ n_front,
                                                                 uint32_t* __restrict__ rank_hi) {
  __shared__ FrontSortSmem sm;
  // the parts of a view run on one XCD (workgroups are dealt to the 8 XCDs in turn), whose L2 holds its runs
  const int kk = (int)(blockIdx.x >> 3);
  const int v = (kk / parts) * 8 + (int)(blockIdx.x & 7u), q = kk % parts;
  if (v >= N) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t base = (int64_t)v * G;
  const int64_t per = fs_run_len(G, wps);
  const uint32_t* cf = cnt + (int64_t)v * 2 * wps;  // fronts per run
  const uint32_t* cv = cf + wps;                    // kept items per run
  // the runs' offsets in the front (thread t owns runs t R', ..., t R' + R' - 1), the front and visible counts
  uint32_t e[kFsRunsPerThread], mine = 0, vis = 0;
#pragma unroll
  for (int qq = 0; qq < kFsRunsPerThread; ++qq) {
    const int k = t * kFsRunsPerThread + qq;
    e[qq] = k < wps ? cf[k] : 0u;
    mine += e[qq];
    vis += k < wps ? cv[k] : 0u;
  }
  uint32_t f = 0, nv = 0;
  uint32_t run = fs_block_scan(mine, sm.wsum, &f);
  fs_block_scan(vis, sm.wsum, &nv);
  const bool cut = f > (uint32_t)kFsCap;
  if (cut && q != 0) return;  // a cut front is sorted by its first part alone
  const bool split = parts > 1 && !cut;
  uint32_t lo_bin = 0, hi_bin = kFsCutBins;  // this part's bins of the key's top 12 bits
  if (!cut) {
#pragma unroll
    for (int qq = 0; qq < kFsRunsPerThread; ++qq) {
      const int k = t * kFsRunsPerThread + qq;
      if (k < wps) sm.cnt[k] = run;
      run += e[qq];
    }
    if (split) {
      // boundary j of the parts: the bin after the one where the sampled count of the front's bins (those below
      // the threshold's) reaches ceil(j S / parts), S the samples in the front; 4096 when no bin does (S = 0)
      const uint32_t tb = (uint32_t)(thr[v] >> (kDepthKeyBits - kFrontBits));
      const uint32_t* h = fhist + (int64_t)v * kFrontBins;
      uint32_t c4[4], loc = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t b = 4 * t + k;
        c4[k] = b < tb ? h[b] : 0u;
        loc += c4[k];
      }
      uint32_t S = 0;
      uint32_t before = fs_block_scan(loc, sm.wsum, &S);
      if (t == 0) sm.misc[0] = sm.misc[1] = kFsCutBins;
      __syncthreads();
      const uint32_t t0 = (uint32_t)(((uint64_t)S * q + parts - 1) / parts);
      const uint32_t t1 = (uint32_t)(((uint64_t)S * (q + 1) + parts - 1) / parts);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t b0 = before;
        before += c4[k];
        if (b0 < t0 && before >= t0) sm.misc[0] = 4 * t + k + 1;  // one thread each (the count is monotone)
        if (b0 < t1 && before >= t1) sm.misc[1] = 4 * t + k + 1;
      }
    }
    __syncthreads();
    if (split) {
      lo_bin = q > 0 ? sm.misc[0] : 0u;
      hi_bin = q + 1 < parts ? sm.misc[1] : (uint32_t)kFsCutBins;
    }
  } else {
    f = fs_cut_runs(sm, items, base, G, wps, per, cf, thr + v);
  }
  const uint32_t f_all = f;
  uint32_t R = (f + kFsThreads - 1) / kFsThreads * 64;  // items per wavefront, a multiple of 64
  int nslot = (int)(R / 64);                             // <= kFsSlots
  unsigned long long it[kFsSlots];
  uint32_t rank[kFsSlots];
#pragma unroll
  for (int j = 0; j < kFsSlots; ++j) {
    it[j] = 0ull;
    rank[j] = 0;
  }
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t out0 = 0;  // the part's first rank in the view's front
  if (cut) {
#pragma unroll
    for (int j = 0; j < kFsSlots; ++j) {
      const uint32_t i = w * R + j * 64 + lane;
      if (j < nslot && i < f) it[j] = sm.items[i];
    }
  } else {
    // each lane finds its items' runs (the last run whose offset is at most the item; empty runs share their
    // successor's offset), the searches of all slots in step, then loads them, all loads in flight together
    int k[kFsSlots];
#pragma unroll
    for (int j = 0; j < kFsSlots; ++j) k[j] = 0;
    for (int step = 1 << (31 - __clz(wps)); step > 0; step >>= 1) {
#pragma unroll
      for (int j = 0; j < kFsSlots; ++j) {
        const uint32_t i = w * R + j * 64 + lane;
        const int kk2 = min(k[j] + step, wps - 1);
        k[j] = (k[j] + step < wps && sm.cnt[kk2] <= i) ? k[j] + step : k[j];
      }
    }
#pragma unroll
    for (int j = 0; j < kFsSlots; ++j) {
      const uint32_t i = w * R + j * 64 + lane;
      if (j < nslot && i < f) it[j] = items[base + fs_run_start(G, per, k[j]) + (i - sm.cnt[k[j]])];
    }
    if (split) {
      // keep the part's items, in front order, at the start of the LDS array; count the items of the lower parts
      uint64_t m[kFsSlots];
      uint32_t own = 0, low = 0;
#pragma unroll
      for (int j = 0; j < kFsSlots; ++j) {
        const bool valid = j < nslot && w * R + j * 64 + lane < f;
        const uint32_t b = fs_bin(it[j]);
        m[j] = __ballot(valid && b >= lo_bin && b < hi_bin);
        own += (uint32_t)__popcll(m[j]);
        low += (uint32_t)__popcll(__ballot(valid && b < lo_bin));
      }
      uint32_t fq = 0;
      uint32_t o = __shfl(fs_block_scan(lane == 0 ? own : 0u, sm.wsum, &fq), 0, 64);
      fs_block_scan(lane == 0 ? low : 0u, sm.wsum, &out0);
#pragma unroll
      for (int j = 0; j < kFsSlots; ++j) {
        if ((m[j] >> lane) & 1ull) sm.items[o + (uint32_t)__popcll(m[j] & lt)] = it[j];
        o += (uint32_t)__popcll(m[j]);
      }
      __syncthreads();
      f = fq;
      R = (f + kFsThreads - 1) / kFsThreads * 64;
      nslot = (int)(R / 64);
#pragma unroll
      for (int j = 0; j < kFsSlots; ++j) {
        const uint32_t i = w * R + j * 64 + lane;
        it[j] = (j < nslot && i < f) ? sm.items[i] : 0ull;
      }
    }
  }
  __syncthreads();  // the run offsets (and the kept items) are read before the first pass clears the counts
  for (int p = 0; p < 4; ++p) {
    const int sh = 24 + kFsBits * p;
    for (int b = t; b < kFsCntSize; b += kFsThreads) sm.cnt[b] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kFsSlots; ++j) {
      if (j >= nslot) break;
      const bool valid = w * R + j * 64 + lane < f;
      const uint32_t d = (uint32_t)(it[j] >> sh) & (kFsBins - 1);
      uint64_t m = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kFsBits; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bb : ~bb;
      }
      const int leader = valid ? __ffsll((long long)m) - 1 : lane;
      uint32_t before = 0;
      if (valid && lane == leader) {
        before = sm.cnt[d * kFsStride + w];
        sm.cnt[d * kFsStride + w] = before + (uint32_t)__popcll(m);
      }
      before = __shfl(before, leader, 64);
      rank[j] = before + (uint32_t)__popcll(m & lt);
      wave_lds_fence();
    }
    __syncthreads();
    // exclusive scan of the counts in (digit, wavefront) order: thread t owns the 8 entries 8t .. 8t + 7 of that
    // order, which are digit t / 2's counters of wavefronts 8 (t % 2) .. 8 (t % 2) + 7
    uint32_t e[8], loc = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      e[k] = sm.cnt[(t >> 1) * kFsStride + 8 * (t & 1) + k];  // digit t / 2, wavefronts 8 (t % 2) + k
      loc += e[k];
    }
    uint32_t run = fs_block_scan(loc, sm.wsum);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      sm.cnt[(t >> 1) * kFsStride + 8 * (t & 1) + k] = run;
      run += e[k];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kFsSlots; ++j) {
      if (j >= nslot) break;
      if (w * R + j * 64 + lane < f) {
        const uint32_t d = (uint32_t)(it[j] >> sh) & (kFsBins - 1);
        sm.items[sm.cnt[d * kFsStride + w] + rank[j]] = it[j];
      }
    }
    __syncthreads();
    if (p < 3) {
#pragma unroll
      for (int j = 0; j < kFsSlots; ++j) {
        if (j >= nslot) break;
        const uint32_t i = w * R + j * 64 + lane;
        if (i < f) it[j] = sm.items[i];
      }
      __syncthreads();
    }
  }
  for (uint32_t i = t; i < f; i += kFsThreads) vals[base + out0 + i] = (uint32_t)(sm.items[i] & 0xffffffull);
  if (t == 0 && q == 0) {
    n_vis[v] = nv;
    n_front[v] = f_all;
    rank_hi[v] = f_all;
  }
}

int blocks_per_seg(int64_t seg_len, int n_seg) {
  // enough blocks to fill the chip (~2048 in flight), never more than one per tile of the segment
  int64_t tiles = (seg_len + kTile - 1) / kTile;
  int64_t want = (2048 + n_seg - 1) / n_seg;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, want));
}

int depth_blocks_per_seg(int64_t seg_len, int n_seg) {
  int64_t tiles = (seg_len + kDepthTile - 1) / kDepthTile;
  int64_t want = (4096 + n_seg - 1) / n_seg;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, want));
}

template <typename K>
SortArgs<K> base_args(const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, uint32_t* hist) {
  SortArgs<K> a{};
  a.kin = kin;
  a.vin = vin;
  a.kout = kout;
  a.vout = vout;
  a.hist = hist;
  a.cap = 0xffffffffu;
  return a;
}

// One pass: histogram, scan (of hsize entries, or of n_mul * *hsize_dev on the device), scatter.
template <typename K, int RB, int ROWS = kRows>
hipError_t launch_pass(const SortArgs<K>& a, int64_t nblocks, int64_t hsize, uint32_t* partial,
                       const uint32_t* hsize_dev, int n_mul, hipStream_t s) {
  hipLaunchKernelGGL((radix_hist_kernel<K, RB, ROWS>), dim3((unsigned)nblocks), dim3(kThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = exclusive_scan_u32(a.hist, a.hist, hsize, partial, s, hsize_dev, n_mul)) != hipSuccess) return e;
  hipLaunchKernelGGL((radix_scatter_kernel<K, RB, ROWS>), dim3((unsigned)nblocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename K>
bool radix_sort_impl(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t seg_len, int n_seg, const uint32_t* seg_n,
                     uint32_t cap, int bit_lo, int bit_hi, uint32_t* hist, uint32_t* partial, hipStream_t s,
                     hipError_t* err) {
  *err = hipSuccess;
  if (seg_len == 0 || n_seg == 0 || bit_hi <= bit_lo) return false;
  const int bps = blocks_per_seg(seg_len, n_seg);
  const int64_t nblocks = (int64_t)bps * n_seg;
  // split the bit range into the fewest passes of at most kMaxBits bits, as even as possible
  const int nbits = bit_hi - bit_lo;
  const int passes = (nbits + kMaxBits - 1) / kMaxBits;
  bool flipped = false;
  int shift = bit_lo;
  for (int p = 0; p < passes; ++p) {
    const int bits = (nbits - (shift - bit_lo) + (passes - p) - 1) / (passes - p);
    SortArgs<K> a = base_args<K>(flipped ? k1 : k0, flipped ? v1 : v0, flipped ? k0 : k1, flipped ? v0 : v1, hist);
    a.seg_len = seg_len;
    a.seg_n = seg_n;
    a.cap = cap;
    a.bps = bps;
    a.shift = shift;
    a.bits = bits;
    a.ndig = 1 << bits;
    if ((*err = launch_pass<K, kMaxBits>(a, nblocks, (int64_t)n_seg * (1 << bits) * bps, partial, nullptr, 1, s)))
      return flipped;
    flipped = !flipped;
    shift += bits;
  }
  return flipped;
}

int part_blocks_per_seg(int n_seg) { return std::max(1, (2048 + n_seg - 1) / n_seg); }

// LSD passes over device ranges [lo[s], hi[s]) (clamped to cap) with the adaptive histogram layout (bpse, pb),
// computed here unless the caller has (layout_ready).  n_dig_one_pass > 0 makes a single pass use only that many
// digits (a partition whose keys are below it); the keys of the last pass may be dropped.  Returns whether the
// result is in (k1, v1).
template <typename K, int RB, int ROWS = kRows>
bool ranges_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int n_seg, const uint32_t* lo, const uint32_t* hi,
                 uint32_t cap, int bps, int bits_total, int n_dig_one_pass, bool keep_last_keys, uint32_t* hist,
                 uint32_t* partial, uint32_t* bpse, uint32_t* pb, bool layout_ready, hipStream_t s, hipError_t* err) {
  *err = hipSuccess;
  if (!layout_ready) {
    hipLaunchKernelGGL(part_layout_kernel, dim3(1), dim3(kThreads), 0, s, lo, hi, cap, n_seg, bps, bpse, pb,
                       kThreads * ROWS);
    if ((*err = hipGetLastError()) != hipSuccess) return false;
  }
  const int64_t nblocks = (int64_t)bps * n_seg;
  const int passes = (bits_total + RB - 1) / RB;
  bool flipped = false;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int pbits = (bits_total - shift + (passes - p) - 1) / (passes - p);
    const bool last = p == passes - 1;
    SortArgs<K> a = base_args<K>(flipped ? k1 : k0, flipped ? v1 : v0,
                                 (last && !keep_last_keys) ? nullptr : (flipped ? k0 : k1), flipped ? v0 : v1, hist);
    a.cap = cap;
    a.bps = bps;
    a.shift = shift;
    a.bits = pbits;
    a.seg_lo = lo;
    a.seg_hi = hi;
    a.pb = pb;
    a.bpse = bpse;
    a.ndig = (passes == 1 && n_dig_one_pass > 0) ? n_dig_one_pass : (1 << pbits);
    if ((*err = launch_pass<K, RB, ROWS>(a, nblocks, (int64_t)n_seg * a.ndig * bps, partial, pb + n_seg, a.ndig,
                                         s)))
      return flipped;
    flipped = !flipped;
    shift += pbits;
  }
  return flipped;
}

}  // namespace

int64_t scan_partial_count(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partial, hipStream_t s,
                              const uint32_t* n_dev, int n_mul, bool byte_sums) {
  if (n <= 0) return hipSuccess;
  const int64_t np = scan_partial_count(n);
  if (byte_sums) {
    hipLaunchKernelGGL(scan_reduce_kernel<true>, dim3((unsigned)np), dim3(kThreads), 0, s, in, n, n_dev, n_mul,
                       partial);
    hipLaunchKernelGGL(scan_down_kernel<true>, dim3((unsigned)np), dim3(kThreads), 0, s, in, out, n, n_dev, n_mul,
                       partial, partial + np);
  } else {
    hipLaunchKernelGGL(scan_reduce_kernel<false>, dim3((unsigned)np), dim3(kThreads), 0, s, in, n, n_dev, n_mul,
                       partial);
    hipLaunchKernelGGL(scan_down_kernel<false>, dim3((unsigned)np), dim3(kThreads), 0, s, in, out, n, n_dev, n_mul,
                       partial, partial + np);
  }
  return hipGetLastError();
}

int64_t radix_hist_size(int64_t seg_len, int n_seg) {
  return (int64_t)blocks_per_seg(seg_len, n_seg) * n_seg * kMaxRadix;
}

bool radix_sort_u64(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t seg_len, int n_seg,
                    const uint32_t* seg_n, uint32_t cap, int bit_lo, int bit_hi, uint32_t* hist, uint32_t* partial,
                    hipStream_t s, hipError_t* err) {
  return radix_sort_impl<uint64_t>(k0, v0, k1, v1, seg_len, n_seg, seg_n, cap, bit_lo, bit_hi, hist, partial, s,
                                   err);
}

int split_waves_per_seg(int64_t seg_len, int n_seg) {
  // about 8192 wavefronts in all, a multiple of the wavefronts of a workgroup, at most one per 64 items
  int64_t w = std::max<int64_t>(1, std::min<int64_t>((8192 + n_seg - 1) / n_seg, (seg_len + 63) / 64));
  return (int)((w + kWaves - 1) / kWaves * kWaves);
}

int64_t split_hist_size(int64_t seg_len, int n_seg) { return (int64_t)n_seg * 2 * split_waves_per_seg(seg_len, n_seg); }

bool radix_split_u64(uint64_t* k0, uint64_t* k1, uint32_t* v1, int64_t seg_len, int n_seg, const uint64_t* thr,
                     uint64_t drop_key, uint32_t* n_vis, uint32_t* n_front, uint32_t* hist, uint32_t* partial,
                     hipStream_t s, hipError_t* err, const uint32_t* live, bool back_only) {
  const int wps = split_waves_per_seg(seg_len, n_seg);
  const int64_t hsize = split_hist_size(seg_len, n_seg);
  const unsigned blocks = (unsigned)((int64_t)n_seg * wps / kWaves);
  hipLaunchKernelGGL(split_hist_kernel, dim3(blocks), dim3(kThreads), 0, s, k0, seg_len, wps, thr, drop_key, live,
                     hist);
  if ((*err = hipGetLastError()) != hipSuccess) return true;
  if ((*err = exclusive_scan_u32(hist, hist, hsize, partial, s)) != hipSuccess) return true;
  hipLaunchKernelGGL(split_scatter_kernel, dim3(blocks), dim3(kThreads), 0, s, k0, seg_len, wps, thr, drop_key, live,
                     back_only, hist, k1, v1);
  if ((*err = hipGetLastError()) != hipSuccess) return true;
  hipLaunchKernelGGL(split_counts_kernel, dim3((unsigned)((n_seg + 63) / 64)), dim3(64), 0, s, hist,
                     partial + scan_partial_count(hsize), n_seg, wps, live, n_vis, n_front);
  *err = hipGetLastError();
  return true;
}

hipError_t launch_front_gather(const uint64_t* keys, uint64_t* kout, int64_t G, int N, const uint32_t* hist,
                               int key_bits, int64_t num, int64_t den, uint64_t* thr, uint64_t drop_key,
                               uint32_t* cnt, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  // positions must fit the packed item's 24 bits
  if (G > kFrontSortMaxG) return hipErrorInvalidValue;
  const int wps = split_waves_per_seg(G, N);
  hipLaunchKernelGGL(front_gather_kernel, dim3((unsigned)((int64_t)N * wps / kWaves)), dim3(kThreads), 0, s, keys, G,
                     wps, hist, key_bits, num, den, thr, drop_key, kout, cnt);
  return hipGetLastError();
}

int64_t depth_ranges_hist_size(int64_t seg_len, int n_seg) {
  return (int64_t)depth_blocks_per_seg(seg_len, n_seg) * n_seg * kMaxRadix;
}

bool depth_ranges_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t seg_len, int n_seg,
                       const uint32_t* lo, const uint32_t* hi, int key_bits, uint32_t* hist, uint32_t* partial,
                       uint32_t* layout, hipStream_t s, hipError_t* err) {
  if (n_seg > kThreads) {
    *err = hipErrorInvalidValue;
    return false;
  }
  // the layout comes with the ranges; the keys of the last pass are not needed, only the values (Gaussian
  // indices) in depth order
  return ranges_sort<uint64_t, kMaxBits, kDepthRows>(k0, v0, k1, v1, n_seg, lo, hi, 0xffffffffu,
                                                     depth_blocks_per_seg(seg_len, n_seg), key_bits, 0, false, hist,
                                                     partial, layout, layout + n_seg, true, s, err);
}

int depth_sort_blocks(int64_t seg_len, int n_seg) { return blocks_per_seg(seg_len, n_seg); }

hipError_t launch_front_select(int N, int key_bits, int64_t num, int64_t den, const uint32_t* hist, uint64_t* thr,
                               hipStream_t s) {
  hipLaunchKernelGGL(front_select_kernel, dim3((unsigned)N), dim3(kThreads), 0, s, hist, key_bits, num, den, thr);
  return hipGetLastError();
}

int64_t front_hist_size(int N) { return (int64_t)N * kFrontBins; }

hipError_t launch_depth_ranges(int N, int64_t G, const uint32_t* n_vis, const uint32_t* n_front,
                               const uint32_t* live, uint32_t* lo, uint32_t* hi, uint32_t* rank_hi, uint32_t* layout,
                               hipStream_t s) {
  if (N > kThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL(depth_ranges_kernel, dim3(1), dim3(kThreads), 0, s, N, G, n_vis, n_front, live, lo, hi, rank_hi,
                     depth_blocks_per_seg(G, N), layout, layout + N);
  return hipGetLastError();
}

bool front_sort_fits(int64_t G, int N) { return G <= kFrontSortMaxG && split_waves_per_seg(G, N) <= kFsMaxRuns; }

int front_sort_parts(int N) { return (int)std::max(1, std::min(8, 256 / std::max(N, 1))); }

hipError_t launch_front_sort(const uint64_t* items, uint32_t* vals, int64_t G, int N, const uint32_t* cnt,
                             const uint32_t* fhist, uint64_t* thr, uint32_t* n_vis, uint32_t* n_front,
                             uint32_t* rank_hi, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  // indices must fit the packed item's 24 bits, and the runs' offsets the count array
  if (!front_sort_fits(G, N)) return hipErrorInvalidValue;
  // one workgroup per (view, part) in enough groups of 8 for the views, the parts of a view 8 apart
  const int parts = front_sort_parts(N);
  const int64_t nb = (int64_t)8 * parts * ((N + 7) / 8);
  hipLaunchKernelGGL(front_sort_kernel, dim3((unsigned)nb), dim3(kFsThreads), 0, s, items, vals, G,
                     split_waves_per_seg(G, N), N, parts, cnt, fhist, thr, n_vis, n_front, rank_hi);
  return hipGetLastError();
}

bool radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t seg_len, int n_seg,
                    const uint32_t* seg_n, uint32_t cap, int bit_lo, int bit_hi, uint32_t* hist, uint32_t* partial,
                    hipStream_t s, hipError_t* err) {
  return radix_sort_impl<uint32_t>(k0, v0, k1, v1, seg_len, n_seg, seg_n, cap, bit_lo, bit_hi, hist, partial, s,
                                   err);
}

int64_t tile_partition_hist_size(int n_seg) { return (int64_t)part_blocks_per_seg(n_seg) * n_seg * kMaxRadix; }

int tile_partition_blocks(int n_seg) { return part_blocks_per_seg(n_seg); }

const uint32_t* tile_partition(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int n_seg,
                               const uint32_t* seg_start, uint32_t cap, int n_dig, uint32_t* hist, uint32_t* partial,
                               uint32_t* layout, uint32_t* start, hipStream_t s, hipError_t* err) {
  *err = hipSuccess;
  if (n_seg > kThreads) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  int bits = 1;
  while ((1 << bits) < n_dig) ++bits;
  const int bps = part_blocks_per_seg(n_seg);
  const uint32_t* lo = seg_start;
  const uint32_t* hi = seg_start + 1;  // consecutive ranges of one array
  uint32_t* bpse = layout;
  uint32_t* pb = layout + n_seg;
  const int passes = (bits + kPartBits - 1) / kPartBits;
  bool fl;
  if (bits > kMaxBits)
    fl = ranges_sort<uint32_t, kPartBits>(k0, v0, k1, v1, n_seg, lo, hi, cap, bps, bits, n_dig, passes > 1, hist,
                                          partial, bpse, pb, true, s, err);
  else
    fl = ranges_sort<uint32_t, kMaxBits>(k0, v0, k1, v1, n_seg, lo, hi, cap, bps, bits, n_dig, false, hist, partial,
                                         bpse, pb, true, s, err);
  if (*err != hipSuccess) return nullptr;
  const int64_t ns = (int64_t)n_seg * n_dig + 1;
  const unsigned g = (unsigned)((ns + kThreads - 1) / kThreads);
  if (passes == 1)
    hipLaunchKernelGGL(hist_starts_kernel, dim3(g), dim3(kThreads), 0, s, hist, pb, bpse, n_dig, n_seg, lo, hi, cap,
                       start);
  else
    hipLaunchKernelGGL(segment_bounds_kernel, dim3(g), dim3(kThreads), 0, s, fl ? k1 : k0, n_dig, n_seg, lo, hi, cap,
                       start);
  if ((*err = hipGetLastError()) != hipSuccess) return nullptr;
  return fl ? v1 : v0;
}

hipError_t launch_chunk_setup(const uint32_t* scanned, int64_t wstride, int N, const unsigned long long* total,
                              unsigned long long* max_total, uint32_t cap, uint32_t* start, uint32_t* layout,
                              hipStream_t s) {
  if (N > kThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chunk_setup_kernel, dim3(1), dim3(kThreads), 0, s, scanned, wstride, N, total, max_total, cap,
                     part_blocks_per_seg(N), start, layout, layout + N);
  return hipGetLastError();
}

hipError_t launch_lower_bounds(const uint32_t* keys, const uint32_t* n_dev, uint32_t cap, int64_t n_static,
                               uint32_t* start, int64_t n_keys, hipStream_t s, int shift) {
  hipLaunchKernelGGL(lower_bounds_kernel, dim3((unsigned)((n_keys + 1 + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, s, keys, n_dev, cap, n_static, start, n_keys, shift);
  return hipGetLastError();
}

}  // namespace dl

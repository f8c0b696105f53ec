// Tile binning of the depth-sorted projected Gaussians of each view, one depth chunk at a time (gfx950).
//
// Input order is (view, depth rank), so emitting (key = view * T + tile, value = Gaussian) pairs in that
// order and then partitioning them by key with a stable radix sort yields every (view, tile) list already in
// front-to-back order: the depth digits were sorted before the Gaussians were duplicated into tiles.
//
// Depth chunks: chunk c of view v holds the visible Gaussians of depth rank [n_v lo_c, n_v hi_c) / den.
// Chunks are binned and blended front to back; a tile whose rays have all terminated is marked dead by the
// blend and receives no keys from later chunks, so keys behind opaque regions are never produced.
//
// A Gaussian is listed in a tile when its cutoff ellipse (q <= q_limit) reaches at least one pixel centre of
// the tile.  The test is conservative (margins above FP32 error), so that the per-pixel rule in the blend
// alone decides what each ray composites and the image does not depend on the tile size or the chunks.
#include "dl_internal.h"

namespace dl {
namespace {

struct TileRange {
  int tx0, tx1, ty0, ty1;
};

__device__ inline bool tile_range(const float* r, const BlendConst& bc, TileRange& tr) {
  // columns y whose centre y + 0.5 lies within [u - ext_x, u + ext_x], widened by one pixel
  const float u = r[0], v = r[1], ex = r[10], ey = r[11];
  int y0 = (int)ceilf(u - ex - 0.5f), y1 = (int)floorf(u + ex - 0.5f);
  int x0 = (int)ceilf(v - ey - 0.5f), x1 = (int)floorf(v + ey - 0.5f);
  y0 = max(y0 - 1, 0); y1 = min(y1 + 1, bc.W - 1);
  x0 = max(x0 - 1, 0); x1 = min(x1 + 1, bc.H - 1);
  if (y0 > y1 || x0 > x1) return false;
  tr.tx0 = y0 / bc.tw; tr.tx1 = y1 / bc.tw;
  tr.ty0 = x0 / bc.th; tr.ty1 = x1 / bc.th;
  return true;
}

// Minimum over the tile's pixel centres (a rectangle) of q = a dx^2 + 2 b dx dy + c dy^2 about (u, v).
// Zero when the centre lies inside; otherwise the minimum of the convex quadratic sits on an edge, where
// it is a 1D quadratic minimised at the clamped stationary point (-b dx / c along a vertical edge,
// -b dy / a along a horizontal one).  ia = 1 / a and ic = 1 / c are precomputed per Gaussian.
__device__ inline bool tile_touch(const float* r, float ia, float ic, float xlo, float xhi, float ylo, float yhi) {
  const float u = r[0], v = r[1], a = r[2], b = r[3], c = r[4], qlim = r[9];
  const float dxl = xlo - u, dxh = xhi - u, dyl = ylo - v, dyh = yhi - v;
  if (dxl <= 0.0f && dxh >= 0.0f && dyl <= 0.0f && dyh >= 0.0f) return true;
  float qmin = 3.0e38f;
  {
    float dx = dxl;
    float dy = fminf(fmaxf(-b * dx * ic, dyl), dyh);
    qmin = fminf(qmin, a * dx * dx + 2.0f * b * dx * dy + c * dy * dy);
    dx = dxh;
    dy = fminf(fmaxf(-b * dx * ic, dyl), dyh);
    qmin = fminf(qmin, a * dx * dx + 2.0f * b * dx * dy + c * dy * dy);
  }
  {
    float dy = dyl;
    float dx = fminf(fmaxf(-b * dy * ia, dxl), dxh);
    qmin = fminf(qmin, a * dx * dx + 2.0f * b * dx * dy + c * dy * dy);
    dy = dyh;
    dx = fminf(fmaxf(-b * dy * ia, dxl), dxh);
    qmin = fminf(qmin, a * dx * dx + 2.0f * b * dx * dy + c * dy * dy);
  }
  return qmin <= qlim * 1.001f + 1e-3f;
}

__device__ inline void load_rec(const float4* rec, float* r) {
  const float4 A = rec[0], B = rec[1], C = rec[2];
  r[0] = A.x; r[1] = A.y; r[2] = A.z; r[3] = A.w;
  r[4] = B.x; r[5] = B.y; r[6] = B.z; r[7] = B.w;
  r[8] = C.x; r[9] = C.y; r[10] = C.z; r[11] = C.w;
}

template <bool EMIT>
__global__ __launch_bounds__(256) void bin_kernel(const float4* __restrict__ rec, const uint32_t* __restrict__ sorted_idx,
                                                  const uint32_t* __restrict__ vis_count, BlendConst bc, ChunkArgs ch,
                                                  const uint8_t* __restrict__ alive, uint32_t* __restrict__ counts,
                                                  unsigned long long* __restrict__ total,
                                                  const uint32_t* __restrict__ offsets, uint32_t* __restrict__ keys,
                                                  uint32_t* __restrict__ vals) {
  const int v = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = vis_count[v];
  const int64_t lo = nv * ch.num_lo / ch.den, hi = nv * ch.num_hi / ch.den;
  const int64_t r = lo + idx;
  const int64_t slot = (int64_t)v * ch.stride + idx;
  uint32_t cnt = 0;
  if (idx < ch.stride && r < hi) {
    const uint32_t g = sorted_idx[(int64_t)v * bc.G + r];
    float rr[12];
    load_rec(rec + ((int64_t)v * bc.G + g) * kRecF4, rr);
    TileRange tr;
    if (tile_range(rr, bc, tr)) {
      const float ia = 1.0f / rr[2], ic = 1.0f / rr[4];
      uint32_t pos = 0, end = 0;
      if (EMIT) {
        // this Gaussian's keys end where the next slot's begin; nothing is written past the capacity
        pos = offsets[slot];
        const uint32_t nxt = slot + 1 < (int64_t)bc.N * ch.stride ? offsets[slot + 1] : 0xffffffffu;
        end = min(min(nxt, ch.cap), pos + (uint32_t)((tr.tx1 - tr.tx0 + 1) * (tr.ty1 - tr.ty0 + 1)));
      }
      const uint8_t* al = alive ? alive + (int64_t)v * bc.T : nullptr;
      for (int ty = tr.ty0; ty <= tr.ty1; ++ty) {
        const float ylo = ty * bc.th + 0.5f, yhi = min((ty + 1) * bc.th, bc.H) - 0.5f;
        for (int tx = tr.tx0; tx <= tr.tx1; ++tx) {
          const int t = ty * bc.ntx + tx;
          if (al && !al[t]) continue;
          const float xlo = tx * bc.tw + 0.5f, xhi = min((tx + 1) * bc.tw, bc.W) - 0.5f;
          if (!tile_touch(rr, ia, ic, xlo, xhi, ylo, yhi)) continue;
          if (EMIT) {
            if (pos < end) {
              keys[pos] = (uint32_t)v * (uint32_t)bc.T + (uint32_t)t;
              vals[pos] = g;
            }
            ++pos;
          } else {
            ++cnt;
          }
        }
      }
    }
  }
  if (!EMIT) {
    if (idx < ch.stride) counts[slot] = cnt;
    __shared__ unsigned long long part[4];
    unsigned long long x = cnt;
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long s = part[0] + part[1] + part[2] + part[3];
      if (s) atomicAdd(total, s);
    }
  }
}

// n = min(total, cap); record the largest total seen and whether any chunk overflowed.
__global__ void finalize_count_kernel(const unsigned long long* __restrict__ total, uint32_t cap,
                                      uint32_t* __restrict__ n_out, unsigned long long* __restrict__ max_total) {
  const unsigned long long t = *total;
  *n_out = (uint32_t)(t < cap ? t : cap);
  if (t > *max_total) *max_total = t;
}

__global__ __launch_bounds__(256) void init_alive_kernel(uint8_t* __restrict__ alive, const uint32_t* __restrict__ ray_off,
                                                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  alive[i] = ray_off ? (uint8_t)(ray_off[i + 1] > ray_off[i]) : (uint8_t)1;
}

__global__ void fill_u64_kernel(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_bin_count(const float4* rec, const uint32_t* sorted_idx, const uint32_t* vis_count,
                            const BlendConst& bc, const ChunkArgs& ch, const uint8_t* alive, uint32_t* counts,
                            unsigned long long* total, hipStream_t s) {
  const dim3 grid((unsigned)((ch.stride + 255) / 256), (unsigned)bc.N);
  hipLaunchKernelGGL(bin_kernel<false>, grid, dim3(256), 0, s, rec, sorted_idx, vis_count, bc, ch, alive, counts,
                     total, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_bin_emit(const float4* rec, const uint32_t* sorted_idx, const uint32_t* vis_count,
                           const BlendConst& bc, const ChunkArgs& ch, const uint8_t* alive, const uint32_t* offsets,
                           uint32_t* keys, uint32_t* vals, hipStream_t s) {
  const dim3 grid((unsigned)((ch.stride + 255) / 256), (unsigned)bc.N);
  hipLaunchKernelGGL(bin_kernel<true>, grid, dim3(256), 0, s, rec, sorted_idx, vis_count, bc, ch, alive, nullptr,
                     nullptr, offsets, keys, vals);
  return hipGetLastError();
}

hipError_t launch_finalize_count(const unsigned long long* total, uint32_t cap, uint32_t* n_out,
                                 unsigned long long* max_total, hipStream_t s) {
  hipLaunchKernelGGL(finalize_count_kernel, dim3(1), dim3(1), 0, s, total, cap, n_out, max_total);
  return hipGetLastError();
}

hipError_t launch_init_alive(uint8_t* alive, const uint32_t* ray_off, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(init_alive_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, alive, ray_off, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace dl

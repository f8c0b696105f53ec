// View map (Eq. (1)-(3)), per-(view, tile) ray lists (Sec. 5) and interlacing (Alg. 1) on gfx950.
#include "dl_internal.h"

namespace dl {
namespace {

// (a b) mod m for 0 <= a < 2^20 and 0 <= b < m < 2^61, by binary expansion of a: no intermediate value reaches 2m,
// so the product never leaves 64-bit integers whatever the size of b.
__device__ inline int64_t mul_mod(int64_t a, int64_t b, int64_t m) {
  int64_t r = 0;
#pragma unroll
  for (int i = 19; i >= 0; --i) {
    r += r;
    if (r >= m) r -= m;
    if ((a >> i) & 1) {
      r += b;
      if (r >= m) r -= m;
    }
  }
  return r;
}

// V[x][s], s = 3y + k.  With tan(alpha) = a/b, L_x = p/q, K_offset = r/c the view is
// v = floor(N * frac(d_offset / L_x)), and d_offset / L_x = (s b c + 3 x a c - r b) q / (b c p).  The host
// reduces the three integer coefficients modulo Q = b c p, so that rho = (s As + x Ax + C) mod Q is the
// numerator of frac(d_offset / L_x) exactly (the floored modulo of Eq. (2) since every term is >= 0), and
// v = N rho / Q with integer division (the floor of Eq. (3)).  When Q (3W + H + 1) fits 63 bits the sum is
// formed directly; otherwise each product is reduced modulo Q on its own (mul_mod).
__global__ __launch_bounds__(256) void view_map_kernel(uint8_t* __restrict__ V, int W3, int H, int N,
                                                       int64_t As, int64_t Ax, int64_t C, int64_t Q, int wide) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)W3 * H) return;
  const int64_t x = idx / W3;
  const int64_t s = idx - x * W3;
  int64_t rho;
  if (wide) {
    rho = mul_mod(s, As, Q) + mul_mod(x, Ax, Q);
    if (rho >= Q) rho -= Q;
    rho += C;
    if (rho >= Q) rho -= Q;
  } else {
    rho = (s * As + x * Ax + C) % Q;
  }
  V[idx] = (uint8_t)((N * rho) / Q);
}

// One thread per pixel: the distinct views among its three subpixels, each with the mask of channels it
// serves.  Entry j of pixel p goes to slot 3p + j; unused slots get key 0xffffffff (sorted last).
// key = v * T + tile, value = local column | local row << 12 | mask << 24.
__global__ __launch_bounds__(256) void rays_emit_kernel(const uint8_t* __restrict__ V, int W, int H, int tw, int th,
                                                        int ntx, int T, uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)W * H) return;
  const int x = (int)(p / W), y = (int)(p - (int64_t)x * W);
  const uint8_t* row = V + (int64_t)x * 3 * W + 3 * y;
  const uint32_t v[3] = {row[0], row[1], row[2]};
  const uint32_t tile = (uint32_t)((x / th) * ntx + (y / tw));
  const uint32_t loc = (uint32_t)(y % tw) | ((uint32_t)(x % th) << 12);
  for (int j = 0; j < 3; ++j) {
    bool first = true;
    for (int i = 0; i < j; ++i) first &= v[i] != v[j];
    uint32_t key = 0xffffffffu, val = 0;
    if (first) {
      uint32_t mask = 0;
      for (int i = 0; i < 3; ++i) mask |= (v[i] == v[j]) ? (1u << i) : 0u;
      key = v[j] * (uint32_t)T + tile;
      val = loc | (mask << 24);
    }
    keys[3 * p + j] = key;
    vals[3 * p + j] = val;
  }
}

// Ray-list keys widened by the ray's 4 x 4 sub-block of its tile (see launch_ray_key_blocks); one thread per entry.
__global__ __launch_bounds__(256) void ray_key_blocks_kernel(uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ vals, int64_t n, int tw,
                                                             int th) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  if (k == 0xffffffffu) return;
  const uint32_t e = vals[i];
  const uint32_t bx = (4u * (e & 0xfffu)) / (uint32_t)tw, by = (4u * ((e >> 12) & 0xfffu)) / (uint32_t)th;
  keys[i] = (k << 4) | (by * 4u + bx);
}

// *count += entries whose channel mask (bits 24-26) has more than one channel; one thread per entry.
__global__ __launch_bounds__(256) void count_multichannel_kernel(const uint32_t* __restrict__ ent, int64_t n,
                                                                 uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t m = i < n ? (ent[i] >> 24) & 7u : 0u;
  const bool multi = (m & (m - 1u)) != 0u;
  const unsigned long long b = __ballot(multi);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (uint32_t)__popcll(b));
}

// Alg. 1: out[x][y][k] = views[V[x][3y + k]][x][y][k]; one thread per subpixel.
__global__ __launch_bounds__(256) void interleave_kernel(const uint8_t* __restrict__ V,
                                                         const float* __restrict__ views, float* __restrict__ out,
                                                         int W, int H) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)3 * W * H;
  if (idx >= n) return;
  const int64_t v = V[idx];
  out[idx] = views[v * n + idx];
}

// Alg. 1 with its Resize: out[s] = view V[s] at panel pixel (x, y) of subpixel s (or its source pixel on a
// repurposed panel), upsampled from vh x vw by bilinear interpolation with half-pixel centres (source
// coordinate (i + 1/2) in / out - 1/2, clamped at 0, neighbours clamped to the last row / column).
__global__ __launch_bounds__(256) void interleave_resize_kernel(const uint8_t* __restrict__ V,
                                                                const int32_t* __restrict__ src,
                                                                const float* __restrict__ views,
                                                                float* __restrict__ out, int W, int H, int vw, int vh) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)3 * W * H;
  if (s >= n) return;
  const int k = (int)(s % 3);
  const int64_t p = src ? (int64_t)src[s] : s / 3;
  const int x = (int)(p / W), y = (int)(p - (int64_t)x * W);
  const float fy = fmaxf(((float)x + 0.5f) * ((float)vh / (float)H) - 0.5f, 0.0f);
  const float fx = fmaxf(((float)y + 0.5f) * ((float)vw / (float)W) - 0.5f, 0.0f);
  const int r0 = min((int)fy, vh - 1), c0 = min((int)fx, vw - 1);
  const int r1 = min(r0 + 1, vh - 1), c1 = min(c0 + 1, vw - 1);
  const float ly = fy - (float)r0, lx = fx - (float)c0;
  const float* img = views + (int64_t)V[s] * vh * vw * 3;
  const float a = img[((int64_t)r0 * vw + c0) * 3 + k], b = img[((int64_t)r0 * vw + c1) * 3 + k];
  const float c = img[((int64_t)r1 * vw + c0) * 3 + k], d = img[((int64_t)r1 * vw + c1) * 3 + k];
  out[s] = (1.0f - ly) * ((1.0f - lx) * a + lx * b) + ly * ((1.0f - lx) * c + lx * d);
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_view_map(uint8_t* V, int W, int H, int N, int64_t As, int64_t Ax, int64_t C, int64_t Q, int wide,
                           hipStream_t s) {
  const int64_t n = (int64_t)3 * W * H;
  hipLaunchKernelGGL(view_map_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, V, 3 * W, H, N, As, Ax, C, Q, wide);
  return hipGetLastError();
}

hipError_t launch_rays_emit(const uint8_t* V, int W, int H, int tw, int th, int ntx, int T, uint32_t* keys,
                            uint32_t* vals, hipStream_t s) {
  const int64_t n = (int64_t)W * H;
  hipLaunchKernelGGL(rays_emit_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, V, W, H, tw, th, ntx, T, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_ray_key_blocks(uint32_t* keys, const uint32_t* vals, int64_t n, int tw, int th, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ray_key_blocks_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, keys, vals, n, tw, th);
  return hipGetLastError();
}

hipError_t launch_count_multichannel(const uint32_t* ent, int64_t n, uint32_t* count, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(count_multichannel_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, ent, n, count);
  return hipGetLastError();
}

hipError_t launch_interleave_resize(const uint8_t* V, const int32_t* src, const float* views, float* out, int W,
                                   int H, int vw, int vh, hipStream_t s) {
  const int64_t n = (int64_t)3 * W * H;
  hipLaunchKernelGGL(interleave_resize_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, V, src, views, out, W, H, vw,
                     vh);
  return hipGetLastError();
}

hipError_t launch_interleave(const uint8_t* V, const float* views, float* out, int W, int H, hipStream_t s) {
  const int64_t n = (int64_t)3 * W * H;
  hipLaunchKernelGGL(interleave_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, V, views, out, W, H);
  return hipGetLastError();
}

}  // namespace dl

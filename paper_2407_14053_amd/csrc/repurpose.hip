// Subpixel repurposing (Sec. "Subpixel Repurposing", Alg. 2, Eq. (11)-(16)): which ray each subpixel shows.
//
// Host part (per display, offline): a walk over the panel in areas of P_w grating units that gives every
// subpixel (x, y, k) of view v = V(x, 3y + k) a source pixel (x', y') of that view: the subpixel shows channel k
// of the ray (v, x', y').  A pixel rendered for one of its channels lends its two other channels to later
// subpixels of the same view found along the lens direction (Eq. (14) search window), so fewer distinct rays
// are rendered.  The heuristic's open points are resolved as follows:
//   - area of a subpixel: that of its pixel, floor(d_offset(x, y, 0) / (P_w L_x)) with d_offset of Eq. (1) at the
//     pixel's left edge (slanted strips of P_w grating units); areas in increasing order, each area's subpixels
//     in row-major order (x, y, k);
//   - one waiting pixel per (view, channel), empty at the start of an area; sampling a subpixel anew (Eq. (11))
//     lends its pixel to the view's two other channels (Eq. (12)), overwriting; repurposing (Eq. (13)) takes
//     and empties the slot of (view, channel);
//   - search window (Eq. (14), parentheses unbalanced in print): rows min(x + 2, h - 1) .. min(x +
//     floor(5 N / (2 L_x)), h - 1), columns max(y - floor(N / (3 L_x)), 0) .. y;
//   - next subpixel: unassigned, same view, inside the window; one whose channel has a waiting pixel if any,
//     else any; first in row-major order (row, column, channel).  The search does not look at areas: the chain
//     goes on only while the subpixel found lies in the chain's area.  None, or one outside the area: the chain
//     ends and the view's slots are emptied.
// Device part: the (view, pixel) rays and, per ray and channel, the subpixel it fills (at most one, since
// each (v, x', y', k) is used once), so the blend writes every ray's channels where they belong.
#include "dl_internal.h"

#include <vector>

namespace dl {
namespace {

int64_t floor_div(__int128 a, __int128 b) {  // b > 0
  __int128 q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return (int64_t)q;
}

// tgt[(3 p + j) * 3 + k] = the subpixel filled by channel k of the ray (view V[3p + j], pixel p), where j is
// the first of the pixel's subpixels with that view; -1 where none.  err: a subpixel whose source pixel does
// not show its view (cannot happen for a map built here).
__global__ __launch_bounds__(256) void tgt_build_kernel(const uint8_t* __restrict__ V, const int32_t* __restrict__ src,
                                                        int64_t n, int32_t* __restrict__ tgt, int32_t* __restrict__ err) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t p = src[s];
  const uint8_t v = V[s];
  const int k = (int)(s % 3);
  int j = -1;
  for (int i = 2; i >= 0; --i)
    if (V[3 * p + i] == v) j = i;
  if (j < 0) {
    *err = 1;
    return;
  }
  tgt[(3 * p + j) * 3 + k] = (int32_t)s;
}

// Ray entries of a repurposed panel, one thread per pixel: for each distinct view among its subpixels that
// fills at least one subpixel, key = v * T + tile, value = local column | local row << 12 | channel mask << 24
// | j << 27 (the slot of the ray's targets).
__global__ __launch_bounds__(256) void rays_emit_sr_kernel(const uint8_t* __restrict__ V,
                                                           const int32_t* __restrict__ tgt, int W, int H, int tw,
                                                           int th, int ntx, int T, uint32_t* __restrict__ keys,
                                                           uint32_t* __restrict__ vals) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)W * H) return;
  const int x = (int)(p / W), y = (int)(p - (int64_t)x * W);
  const uint8_t* row = V + 3 * p;
  const uint32_t tile = (uint32_t)((x / th) * ntx + (y / tw));
  const uint32_t loc = (uint32_t)(y % tw) | ((uint32_t)(x % th) << 12);
  for (int j = 0; j < 3; ++j) {
    bool first = true;
    for (int i = 0; i < j; ++i) first &= row[i] != row[j];
    uint32_t mask = 0;
    if (first)
      for (int k = 0; k < 3; ++k) mask |= tgt[(3 * p + j) * 3 + k] >= 0 ? (1u << k) : 0u;
    keys[3 * p + j] = mask ? (uint32_t)row[j] * (uint32_t)T + tile : 0xffffffffu;
    vals[3 * p + j] = loc | (mask << 24) | ((uint32_t)j << 27);
  }
}

// Standard paradigm through the repurposed map: out[s] = views[V[s]][src[s]][s mod 3].
__global__ __launch_bounds__(256) void interleave_sr_kernel(const uint8_t* __restrict__ V,
                                                            const int32_t* __restrict__ src,
                                                            const float* __restrict__ views, float* __restrict__ out,
                                                            int64_t n) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  out[s] = views[(int64_t)V[s] * n + 3 * (int64_t)src[s] + s % 3];
}

__global__ __launch_bounds__(256) void own_pixel_kernel(int32_t* __restrict__ out, int64_t n) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) out[s] = (int32_t)(s / 3);
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int repurpose_sources(const dl_display_desc& d, int pw, const uint8_t* V, int32_t* src, std::string* why) {
  const int W = d.width, H = d.height, N = d.n_views, W3 = 3 * d.width;
  const __int128 a = d.tan_slant.num, b = d.tan_slant.den, p = d.pitch.num, q = d.pitch.den, r = d.offset.num,
                 c = d.offset.den;
  if (pw < 1) {
    *why = "repurpose_pw must be >= 1";
    return DL_EINVAL;
  }
  // area(x, s) = floor(d_offset(x, y, 0) / (pw L)) = floor(D q / (b c pw p)), D = 3 y b c + 3 x a c - r b for
  // the subpixel s = 3 y + k (all three subpixels of a pixel share its area)
  const __int128 den = b * c * (__int128)pw * p;
  std::vector<int32_t> area((size_t)H * W3);
  int64_t amin = INT64_MAX, amax = INT64_MIN;
  for (int x = 0; x < H; ++x)
    for (int s = 0; s < W3; ++s) {
      const __int128 D = (__int128)(s - s % 3) * b * c + (__int128)3 * x * a * c - r * b;
      const int64_t A = floor_div(D * q, den);
      if (A < INT32_MIN || A > INT32_MAX) {
        *why = "repurposing area index out of range";
        return DL_ERANGE;
      }
      area[(size_t)x * W3 + s] = (int32_t)A;
      amin = std::min(amin, A);
      amax = std::max(amax, A);
    }
  const int drow = (int)floor_div((__int128)5 * N * q, (__int128)2 * p);  // 2 N / L + N / (2 L)
  const int dcol = (int)floor_div((__int128)N * q, (__int128)3 * p);      // N / (3 L)
  std::fill(src, src + (size_t)H * W3, -1);
  std::vector<int32_t> slot((size_t)N * 3, -1);  // waiting pixel per (view, channel)
  std::vector<int> cur(H, 0);                    // per row: first subpixel not yet visited (areas grow with s)
  for (int64_t A = amin; A <= amax; ++A) {
    std::fill(slot.begin(), slot.end(), -1);
    for (int x0 = 0; x0 < H; ++x0) {
      int& c0 = cur[x0];
      for (; c0 < W3 && area[(size_t)x0 * W3 + c0] == A; ++c0) {
        const int v = V[(size_t)x0 * W3 + c0];
        int x = x0, y = c0 / 3, k = c0 % 3;
        while (src[(size_t)x * W3 + 3 * y + k] < 0 && area[(size_t)x * W3 + 3 * y + k] == A) {
          int32_t& sl = slot[(size_t)v * 3 + k];
          if (sl >= 0) {  // Eq. (13)
            src[(size_t)x * W3 + 3 * y + k] = sl;
            sl = -1;
          } else {        // Eq. (11)-(12)
            const int32_t pix = x * W + y;
            src[(size_t)x * W3 + 3 * y + k] = pix;
            slot[(size_t)v * 3 + (k + 1) % 3] = pix;
            slot[(size_t)v * 3 + (k + 2) % 3] = pix;
          }
          // Eq. (14) window; the next subpixel of view v in it
          const int xlo = std::min(x + 2, H - 1), xhi = std::min(x + drow, H - 1);
          const int ylo = std::max(y - dcol, 0), yhi = y;
          int fx = -1, fy = 0, fk = 0, px = -1, py = 0, pk = 0;
          for (int xx = xlo; xx <= xhi && px < 0; ++xx)
            for (int yy = ylo; yy <= yhi; ++yy)
              for (int kk = 0; kk < 3; ++kk) {
                const size_t sidx = (size_t)xx * W3 + 3 * yy + kk;
                if (V[sidx] != v || src[sidx] >= 0) continue;
                if (fx < 0) {
                  fx = xx; fy = yy; fk = kk;
                }
                if (px < 0 && slot[(size_t)v * 3 + kk] >= 0) {
                  px = xx; py = yy; pk = kk;
                }
              }
          if (px >= 0) {
            x = px; y = py; k = pk;
          } else if (fx >= 0) {
            x = fx; y = fy; k = fk;
          } else {
            break;
          }
        }
        for (int kk = 0; kk < 3; ++kk) slot[(size_t)v * 3 + kk] = -1;
      }
    }
  }
  for (size_t i = 0; i < (size_t)H * W3; ++i)
    if (src[i] < 0) {
      *why = "repurposing left a subpixel unassigned";
      return DL_EINVAL;
    }
  return DL_OK;
}

hipError_t launch_tgt_build(const uint8_t* V, const int32_t* src, int W, int H, int32_t* tgt, int32_t* err,
                            hipStream_t s) {
  const int64_t n = (int64_t)3 * W * H;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(3 * n)), dim3(256), 0, s, tgt, 3 * n, -1);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(256), 0, s, err, (int64_t)1, 0);
  hipLaunchKernelGGL(tgt_build_kernel, dim3(blocks_for(n)), dim3(256), 0, s, V, src, n, tgt, err);
  return hipGetLastError();
}

hipError_t launch_rays_emit_sr(const uint8_t* V, const int32_t* tgt, int W, int H, int tw, int th, int ntx, int T,
                               uint32_t* keys, uint32_t* vals, hipStream_t s) {
  const int64_t n = (int64_t)W * H;
  hipLaunchKernelGGL(rays_emit_sr_kernel, dim3(blocks_for(n)), dim3(256), 0, s, V, tgt, W, H, tw, th, ntx, T, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_interleave_sr(const uint8_t* V, const int32_t* src, const float* views, float* out, int W, int H,
                                hipStream_t s) {
  const int64_t n = (int64_t)3 * W * H;
  hipLaunchKernelGGL(interleave_sr_kernel, dim3(blocks_for(n)), dim3(256), 0, s, V, src, views, out, n);
  return hipGetLastError();
}

hipError_t launch_own_pixel(int32_t* out, int W, int H, hipStream_t s) {
  const int64_t n = (int64_t)3 * W * H;
  hipLaunchKernelGGL(own_pixel_kernel, dim3(blocks_for(n)), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

}  // namespace dl

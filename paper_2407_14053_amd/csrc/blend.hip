// Front-to-back alpha compositing of each (view, tile) list into the rays that need it (gfx950).
//
// Workgroup = one (view, tile) work item, 256 lanes (4 wavefronts of 64).  Each lane owns up to RPT rays of
// the tile: for DirectL the rays in the view's ray list (pixels whose subpixels that view owns, with the
// channel mask), for the standard paradigm every pixel of the tile.  The tile's depth-ordered list is
// staged through LDS 256 records at a time (one coalesced 48-byte record per lane); every lane then reads
// the records as LDS broadcasts and applies, per ray, the per-pixel rule and Eq. (5)/(10):
//   q = d^T Sigma'^{-1} d,  alpha = min(alpha_max, o exp(-q/2)),  blend iff q <= q_cut and alpha >= alpha_min,
//   stop (without blending) when T (1 - alpha) < t_min.
// A wavefront leaves the LDS chunk as soon as a ballot shows all its rays finished, and the workgroup
// leaves the list when none of its lanes has a live ray.  The epilogue writes C + T bg into the owned
// subpixels of the encoded image (DirectL) or into all three channels of the view image (standard).
// The arithmetic per (ray, record) is written with explicit FMAs and compiled without contraction, so
// both paths produce bit-identical colours for the same ray.
#include "dl_internal.h"

namespace dl {
namespace {

constexpr int kThreads = 256;

__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  // workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous range of work items so
  // that the tiles sharing a view's records share an L2
  const uint32_t q = nb / 8, rem = nb % 8;
  const uint32_t x = b % 8, k = b / 8;
  return x * q + min(x, rem) + k;
}

template <bool STD, int RPT>
__global__ __launch_bounds__(kThreads) void blend_kernel(const float4* __restrict__ rec,
                                                          const uint32_t* __restrict__ tile_start,
                                                          const uint32_t* __restrict__ gidx,
                                                          const uint32_t* __restrict__ ray_off,
                                                          const uint32_t* __restrict__ ray_ent, BlendConst bc,
                                                          float* __restrict__ out) {
  __shared__ float4 sm[kThreads * kRecF4];
  const uint32_t wi = xcd_remap(blockIdx.x, gridDim.x);
  const int vl = (int)(wi / (uint32_t)bc.T);
  const int t = (int)(wi - (uint32_t)vl * (uint32_t)bc.T);
  const int v = bc.v0 + vl;
  const int tx = t % bc.ntx, ty = t / bc.ntx;
  const int ox = tx * bc.tw, oy = ty * bc.th;
  int nr, r0 = 0, cw = 0;
  if (STD) {
    cw = min(bc.tw, bc.W - ox);
    nr = cw * min(bc.th, bc.H - oy);
  } else {
    r0 = (int)ray_off[(int64_t)v * bc.T + t];
    nr = (int)ray_off[(int64_t)v * bc.T + t + 1] - r0;
  }
  if (nr <= 0) return;

  float px[RPT], py[RPT], Tr[RPT], C0[RPT], C1[RPT], C2[RPT];
  uint32_t mask[RPT];
  bool live[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * kThreads;
    live[j] = idx < nr;
    int lx = 0, ly = 0;
    mask[j] = 0;
    if (live[j]) {
      if (STD) {
        ly = idx / cw;
        lx = idx - ly * cw;
        mask[j] = 7u;
      } else {
        const uint32_t e = ray_ent[r0 + idx];
        lx = (int)(e & 0xfffu);
        ly = (int)((e >> 12) & 0xfffu);
        mask[j] = e >> 24;
      }
    }
    px[j] = (float)(ox + lx) + 0.5f;
    py[j] = (float)(oy + ly) + 0.5f;
    Tr[j] = 1.0f;
    C0[j] = C1[j] = C2[j] = 0.0f;
  }
  const float q_cut = bc.q_cut, a_min = bc.alpha_min, a_max = bc.alpha_max, t_min = bc.t_min;
  const uint32_t ls = tile_start[(int64_t)vl * bc.T + t];
  const uint32_t le = tile_start[(int64_t)vl * bc.T + t + 1];
  const float4* vrec = rec + (int64_t)v * bc.G * kRecF4;

  for (uint32_t base = ls; base < le; base += kThreads) {
    const int n = (int)min((uint32_t)kThreads, le - base);
    if ((int)threadIdx.x < n) {
      const uint32_t g = gidx[base + threadIdx.x];
      const float4* src = vrec + (int64_t)g * kRecF4;
      sm[threadIdx.x * kRecF4 + 0] = src[0];
      sm[threadIdx.x * kRecF4 + 1] = src[1];
      sm[threadIdx.x * kRecF4 + 2] = src[2];
    }
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int j = 0; j < RPT; ++j) any |= live[j];
    if (__ballot(any) != 0ull) {
      for (int k = 0; k < n; ++k) {
        const float4 A = sm[k * kRecF4 + 0];  // u, v, conic a, conic b
        const float4 B = sm[k * kRecF4 + 1];  // conic c, opacity, r, g
        const float bb = sm[k * kRecF4 + 2].x;  // b (blue)
        bool any_live = false;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          if (!live[j]) continue;
          const float dx = px[j] - A.x, dy = py[j] - A.y;
          const float q = fmaf(A.z * dx, dx, fmaf(2.0f * A.w * dx, dy, B.x * dy * dy));
          if (q <= q_cut) {
            const float alpha = fminf(a_max, B.y * __expf(-0.5f * q));
            if (alpha >= a_min) {
              const float tn = Tr[j] * (1.0f - alpha);
              if (tn < t_min) {
                live[j] = false;
              } else {
                const float w = alpha * Tr[j];
                C0[j] = fmaf(w, B.z, C0[j]);
                C1[j] = fmaf(w, B.w, C1[j]);
                C2[j] = fmaf(w, bb, C2[j]);
                Tr[j] = tn;
              }
            }
          }
          any_live |= live[j];
        }
        if (__ballot(any_live) == 0ull) break;
      }
    }
    bool mine = false;
#pragma unroll
    for (int j = 0; j < RPT; ++j) mine |= live[j];
    if (!__syncthreads_or(mine)) break;
  }

#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * kThreads;
    if (idx >= nr) continue;
    const int xr = (int)(py[j] - 0.5f), yc = (int)(px[j] - 0.5f);
    const float c[3] = {fmaf(Tr[j], bc.bg[0], C0[j]), fmaf(Tr[j], bc.bg[1], C1[j]), fmaf(Tr[j], bc.bg[2], C2[j])};
    if (STD) {
      float* dst = out + (((int64_t)v * bc.H + xr) * bc.W + yc) * 3;
      dst[0] = c[0];
      dst[1] = c[1];
      dst[2] = c[2];
    } else {
      float* dst = out + ((int64_t)xr * bc.W + yc) * 3;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (mask[j] & (1u << k)) dst[k] = c[k];
    }
  }
}

template <bool STD>
hipError_t launch_rpt(int rpt, unsigned nblocks, const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                      const uint32_t* ray_off, const uint32_t* ray_ent, const BlendConst& bc, float* out,
                      hipStream_t s) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL((blend_kernel<STD, 1>), dim3(nblocks), dim3(kThreads), 0, s, rec, tile_start, gidx, ray_off, ray_ent, bc, out); break;
    case 2: hipLaunchKernelGGL((blend_kernel<STD, 2>), dim3(nblocks), dim3(kThreads), 0, s, rec, tile_start, gidx, ray_off, ray_ent, bc, out); break;
    case 4: hipLaunchKernelGGL((blend_kernel<STD, 4>), dim3(nblocks), dim3(kThreads), 0, s, rec, tile_start, gidx, ray_off, ray_ent, bc, out); break;
    case 8: hipLaunchKernelGGL((blend_kernel<STD, 8>), dim3(nblocks), dim3(kThreads), 0, s, rec, tile_start, gidx, ray_off, ray_ent, bc, out); break;
    case 16: hipLaunchKernelGGL((blend_kernel<STD, 16>), dim3(nblocks), dim3(kThreads), 0, s, rec, tile_start, gidx, ray_off, ray_ent, bc, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int rpt_for(int max_rays) {
  int r = 1;
  while (r * kThreads < max_rays) r *= 2;
  return r;
}

}  // namespace

hipError_t launch_blend_directl(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                const uint32_t* ray_off, const uint32_t* ray_ent, int max_rays,
                                const BlendConst& bc, float* out, hipStream_t s) {
  const unsigned nb = (unsigned)((int64_t)bc.nv * bc.T);
  if (nb == 0) return hipSuccess;
  return launch_rpt<false>(rpt_for(max_rays), nb, rec, tile_start, gidx, ray_off, ray_ent, bc, out, s);
}

hipError_t launch_blend_standard(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                 const BlendConst& bc, float* views, hipStream_t s) {
  const unsigned nb = (unsigned)((int64_t)bc.nv * bc.T);
  if (nb == 0) return hipSuccess;
  return launch_rpt<true>(rpt_for(bc.tw * bc.th), nb, rec, tile_start, gidx, nullptr, nullptr, bc, views, s);
}

}  // namespace dl

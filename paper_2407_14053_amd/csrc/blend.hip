// Front-to-back alpha compositing of each (view, tile) list into the rays that need it (gfx950).
//
// Workgroup = one (view, tile) work item, 256 lanes (4 wavefronts of 64).  Each lane owns up to RPT rays of
// the tile: for DirectL the rays in the view's ray list (pixels whose subpixels that view owns, with the
// channel mask), for the standard paradigm every pixel of the tile.  The tile's depth-ordered list is
// staged through LDS 256 records at a time (one coalesced 48-byte record per lane); every lane then reads
// the records as LDS broadcasts and applies, per ray, the per-pixel rule and Eq. (5)/(10):
//   q = d^T Sigma'^{-1} d,  alpha = min(alpha_max, o exp(-q/2)),  blend iff q <= q_cut and alpha >= alpha_min
//   (tested as one bound on q per record),
//   stop (without blending) when T (1 - alpha) < t_min,
// with q held as Q = q log2(e)/2 (the record's conic is pre-scaled) and o exp(-q/2) = 2^(log2(o) - Q): the
// staged record carries log2(o), so the exponent comes out of the quadratic form's FMAs and alpha costs one
// v_exp_f32 and a min.
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
  // workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous range of work items
  const uint32_t q = nb / 8, rem = nb % 8;
  const uint32_t x = b % 8, k = b / 8;
  return x * q + min(x, rem) + k;
}

template <bool STD, int RPT, bool STATS, int NT>
__global__ __launch_bounds__(NT) void blend_kernel(const float4* __restrict__ rec,
                                                          const uint32_t* __restrict__ tile_start,
                                                          const uint32_t* __restrict__ gidx,
                                                          const uint32_t* __restrict__ ray_off,
                                                          const uint32_t* __restrict__ ray_ent, BlendConst bc,
                                                          BlendChunk bk, uint8_t* __restrict__ alive,
                                                          float4* __restrict__ state, float* __restrict__ out) {
  __shared__ float4 sm[NT * kRecF4];
  // work items in tile-major order, a contiguous range of them per XCD: all views of a tile run on one XCD
  // at about the same time, so the partial writes of their interleaved subpixels meet in that XCD's L2
  const uint32_t wi = xcd_remap(blockIdx.x, gridDim.x);
  const int t = (int)(wi / (uint32_t)bc.N);
  const int v = (int)(wi - (uint32_t)t * (uint32_t)bc.N);
  const int64_t vt = (int64_t)v * bc.T + t;
  if (!alive[vt]) return;
  const int tx = t % bc.ntx, ty = t / bc.ntx;
  const int ox = tx * bc.tw, oy = ty * bc.th;
  int nr, r0 = 0, cw = 0;
  if (STD) {
    cw = min(bc.tw, bc.W - ox);
    nr = cw * min(bc.th, bc.H - oy);
  } else {
    r0 = (int)ray_off[vt];
    nr = (int)ray_off[vt + 1] - r0;
  }
  if (nr <= 0) return;

  // sT: the ray's transmittance, its sign carrying the ray's state (negative once terminated or absent)
  float px[RPT], py[RPT], sT[RPT], C0[RPT], C1[RPT], C2[RPT];
  uint32_t mask[RPT], nev[RPT], nbl[RPT];
  int64_t gid[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * NT;
    const bool valid = idx < nr;
    int lx = 0, ly = 0;
    mask[j] = 0;
    if (valid) {
      if (STD) {
        ly = idx / cw;
        lx = idx - ly * cw;
        mask[j] = 7u;
      } else {
        const uint32_t e = ray_ent[r0 + idx];
        lx = (int)(e & 0xfffu);
        ly = (int)((e >> 12) & 0xfffu);
        mask[j] = (e >> 24) & 7u;
      }
    }
    px[j] = (float)(ox + lx) + 0.5f;
    py[j] = (float)(oy + ly) + 0.5f;
    gid[j] = STD ? ((int64_t)v * bc.H + oy + ly) * bc.W + ox + lx : (int64_t)r0 + idx;
    sT[j] = valid ? 1.0f : -1.0f;
    C0[j] = C1[j] = C2[j] = 0.0f;
    if (valid && !bk.first) {
      const float4 st = state[gid[j]];
      sT[j] = st.x;
      C0[j] = st.y;
      C1[j] = st.z;
      C2[j] = st.w;
    }
    nev[j] = nbl[j] = 0;
  }
  const float a_max = bc.alpha_max, t_min = bc.t_min;
  const uint32_t ls = tile_start[vt];
  const uint32_t le = tile_start[vt + 1];
  const float4* vrec = rec + (int64_t)v * bc.G * kRecF4;

  for (uint32_t base = ls; base < le; base += NT) {
    const int n = (int)min((uint32_t)NT, le - base);
    if ((int)threadIdx.x < n) {
      const uint32_t g = gidx[base + threadIdx.x];
      const float4* src = vrec + (int64_t)g * kRecF4;
      const float4 r1 = src[1], r2 = src[2];
      const float lo = __builtin_amdgcn_logf(r2.x);  // log2(o)
      sm[threadIdx.x * kRecF4 + 0] = src[0];
      // the LDS copy carries log2(o) in place of o and, in place of the binning's Q limit, the blend's bound on
      // E = log2(o) - Q (see blend_elim)
      sm[threadIdx.x * kRecF4 + 1] = make_float4(r1.x, blend_elim(lo, bc), r1.z, r1.w);
      sm[threadIdx.x * kRecF4 + 2] = make_float4(lo, r2.y, r2.z, r2.w);
    }
    __syncthreads();
    bool any = false;
    bool slot[RPT];  // wavefront has a live ray in slot j (slots other than the first are often empty)
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      any |= sT[j] > 0.0f;
      slot[j] = __ballot(sT[j] > 0.0f) != 0ull;
    }
    if (__ballot(any) != 0ull) {
      for (int k = 0; k < n; ++k) {
        const float4 A = sm[k * kRecF4 + 0];    // u, v, conic A, B (scaled)
        const float2 CQ = *reinterpret_cast<const float2*>(&sm[k * kRecF4 + 1]);  // conic C (scaled), E limit
        const float cC = CQ.x;
        const float4 B = sm[k * kRecF4 + 2];    // log2(opacity), r, g, b
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          if (j > 0 && !slot[j]) continue;
          // per-pixel rule and front-to-back update, without branches:
          //   E = log2(o) - Q = log2(o) - C dy^2 - (A dx + B dy) dx, alpha = min(alpha_max, 2^E)
          //   T' = T (1 - alpha) as one FMA, the colour weight as T - T' (alpha T up to one rounding of T')
          // A finished ray keeps T < 0: then T' < 0 < t_min, so an accepted record only "stops" it again, and
          // the stop writes -|T|, which leaves it unchanged; no liveness test is needed per pair.
          const float dx = px[j] - A.x, dy = py[j] - A.y;
          const float E = fmaf(-fmaf(A.w, dy, A.z * dx), dx, fmaf(-(cC * dy), dy, B.x));
          const float alpha = fminf(a_max, __builtin_amdgcn_exp2f(E));
          const float T = sT[j];
          const float tn = fmaf(-alpha, T, T);
          const bool ok = E >= CQ.y;
          const bool stop = ok && (tn < t_min);
          const bool take = ok != stop;  // ok and not stop (stop implies ok): one scalar mask operation
          const float Tt = take ? tn : T;
          const float w = T - Tt;
          if (STATS) {
            nev[j] += T > 0.0f ? 1u : 0u;
            nbl[j] += take ? 1u : 0u;
          }
          C0[j] = fmaf(w, B.y, C0[j]);
          C1[j] = fmaf(w, B.z, C1[j]);
          C2[j] = fmaf(w, B.w, C2[j]);
          sT[j] = stop ? -fabsf(T) : Tt;
        }
        // leave the chunk once no ray of the wavefront is live (checked every 4 records)
        if ((k & 3) == 3) {
          bool any_live = false;
#pragma unroll
          for (int j = 0; j < RPT; ++j) any_live |= sT[j] > 0.0f;
          if (__ballot(any_live) == 0ull) break;
        }
      }
    }
    bool mine = false;
#pragma unroll
    for (int j = 0; j < RPT; ++j) mine |= sT[j] > 0.0f;
    if (!__syncthreads_or(mine)) break;
  }
  bool mine = false;
#pragma unroll
  for (int j = 0; j < RPT; ++j) mine |= sT[j] > 0.0f;
  const bool tile_live = __syncthreads_or(mine);
  if (!tile_live && threadIdx.x == 0) alive[vt] = 0;

  if (STATS) {
    unsigned long long e = 0, b = 0, r = 0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      e += nev[j];
      b += nbl[j];
      r += (bk.first && threadIdx.x + j * NT < nr) ? 1 : 0;
    }
    for (int d = 32; d >= 1; d >>= 1) {
      e += __shfl_xor(e, d, 64);
      b += __shfl_xor(b, d, 64);
      r += __shfl_xor(r, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      // spread over slots: same-address atomics from every wavefront would serialise
      unsigned long long* slot = bc.stats + 3 * ((blockIdx.x * 4 + (threadIdx.x >> 6)) % kStatSlots);
      atomicAdd(&slot[0], e);
      atomicAdd(&slot[1], b);
      atomicAdd(&slot[2], r);
    }
  }

#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * NT;
    if (idx >= nr) continue;
    if (!bk.last && tile_live) state[gid[j]] = make_float4(sT[j], C0[j], C1[j], C2[j]);
    if (bk.last || !tile_live) {
      const int xr = (int)(py[j] - 0.5f), yc = (int)(px[j] - 0.5f);
      const float Tf = fabsf(sT[j]);
      const float c[3] = {fmaf(Tf, bc.bg[0], C0[j]), fmaf(Tf, bc.bg[1], C1[j]), fmaf(Tf, bc.bg[2], C2[j])};
      if (STD) {
        float* dst = out + (((int64_t)v * bc.H + xr) * bc.W + yc) * 3;
        dst[0] = c[0];
        dst[1] = c[1];
        dst[2] = c[2];
      } else {
        if (bc.tgt) {
          // repurposed panel: channel k of the ray fills the subpixel listed for it
          const uint32_t slot = (ray_ent[r0 + idx] >> 27) & 3u;
          const int32_t* tg = bc.tgt + ((int64_t)3 * ((int64_t)xr * bc.W + yc) + slot) * 3;
#pragma unroll
          for (int k = 0; k < 3; ++k)
            if (mask[j] & (1u << k)) out[tg[k]] = c[k];
        } else {
          float* dst = out + ((int64_t)xr * bc.W + yc) * 3;
#pragma unroll
          for (int k = 0; k < 3; ++k)
            if (mask[j] & (1u << k)) dst[k] = c[k];
        }
      }
    }
  }
}

template <bool STD, int NT>
hipError_t launch_rpt(int rpt, unsigned nblocks, const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                      const uint32_t* ray_off, const uint32_t* ray_ent, const BlendConst& bc, BlendChunk bk,
                      uint8_t* alive, float4* state, float* out, hipStream_t s) {
#define DL_BLEND_CASE(R)                                                                                        \
  case R:                                                                                                      \
    if (bc.stats)                                                                                              \
      hipLaunchKernelGGL((blend_kernel<STD, R, true, NT>), dim3(nblocks), dim3(NT), 0, s, rec, tile_start,     \
                         gidx, ray_off, ray_ent, bc, bk, alive, state, out);                                   \
    else                                                                                                       \
      hipLaunchKernelGGL((blend_kernel<STD, R, false, NT>), dim3(nblocks), dim3(NT), 0, s, rec, tile_start,    \
                         gidx, ray_off, ray_ent, bc, bk, alive, state, out);                                   \
    break;
  switch (rpt) {
    DL_BLEND_CASE(1)
    DL_BLEND_CASE(2)
    DL_BLEND_CASE(3)
    DL_BLEND_CASE(4)
    DL_BLEND_CASE(5)
    DL_BLEND_CASE(6)
    DL_BLEND_CASE(7)
    DL_BLEND_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef DL_BLEND_CASE
  return hipGetLastError();
}

// Workgroup shape for a tile's largest ray list: 256 lanes with up to 4 rays each, else 512 lanes with up to 8
// (registers, and so occupancy, grow with the rays per lane; slots a whole wavefront leaves empty cost nothing).
template <bool STD>
hipError_t launch_blend(int max_rays, unsigned nblocks, const float4* rec, const uint32_t* tile_start,
                        const uint32_t* gidx, const uint32_t* ray_off, const uint32_t* ray_ent, const BlendConst& bc,
                        BlendChunk bk, uint8_t* alive, float4* state, float* out, hipStream_t s) {
  if (max_rays <= 4 * 256)
    return launch_rpt<STD, 256>(std::max(1, (max_rays + 255) / 256), nblocks, rec, tile_start, gidx, ray_off, ray_ent,
                                bc, bk, alive, state, out, s);
  if (max_rays > 8 * 512) return hipErrorInvalidValue;
  return launch_rpt<STD, 512>((max_rays + 511) / 512, nblocks, rec, tile_start, gidx, ray_off, ray_ent, bc, bk, alive,
                              state, out, s);
}

}  // namespace

hipError_t launch_blend_directl(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                const uint32_t* ray_off, const uint32_t* ray_ent, int max_rays,
                                const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state, float* out,
                                hipStream_t s) {
  const unsigned nb = (unsigned)((int64_t)bc.N * bc.T);
  if (nb == 0) return hipSuccess;
  return launch_blend<false>(max_rays, nb, rec, tile_start, gidx, ray_off, ray_ent, bc, bk, alive, state, out, s);
}

hipError_t launch_blend_standard(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                 const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state, float* views,
                                 hipStream_t s) {
  const unsigned nb = (unsigned)((int64_t)bc.N * bc.T);
  if (nb == 0) return hipSuccess;
  return launch_blend<true>(bc.tw * bc.th, nb, rec, tile_start, gidx, nullptr, nullptr, bc, bk, alive, state, views,
                            s);
}

}  // namespace dl

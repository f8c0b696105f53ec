// Front-to-back alpha compositing of each (view, tile) list into the rays that need it (gfx950).
//
// Workgroup = one (view, tile) work item, 256 or 512 lanes (wavefronts of 64).  Each lane owns up to RPT rays
// of the tile: for DirectL the rays in the view's ray list (pixels whose subpixels that view owns, with the
// channel mask), for the standard paradigm every pixel of the tile.  The tile's depth-ordered list is
// staged through LDS NT records at a time (one record per lane); every lane then
// reads the records as LDS broadcasts and applies, per ray, the per-pixel rule and Eq. (5)/(10):
//   q = d^T Sigma'^{-1} d,  alpha = min(alpha_max, o exp(-q/2)),  blend iff q <= q_cut and alpha >= alpha_min
//   (tested as one bound on q per record),
//   stop (without blending) when T (1 - alpha) < t_min,
// with q held as Q = q log2(e)/2 (the record's conic is pre-scaled) and o exp(-q/2) = 2^(log2(o) - Q): the
// staged record carries log2(o), so the exponent comes out of the quadratic form's FMAs and alpha costs one
// v_exp_f32.  The clamp at alpha_max can only bind for a Gaussian whose opacity is within 2^-10 of alpha_max
// (blend_cap); a staged chunk without such a record runs a loop without the clamp's v_min.
// When every ray of the panel fills one channel (the identity map with three views per pixel), the staged
// colours are three LDS rows and each ray reads and accumulates only its own channel (one FMA per pair instead
// of three); the record loop is unrolled by 4 so that one address add per ray serves four records.
// A wavefront leaves the LDS chunk as soon as a ballot shows all its rays finished, and the workgroup
// leaves the list when none of its lanes has a live ray.  The epilogue writes C + T bg into the owned
// subpixels of the encoded image (DirectL) or into all three channels of the view image (standard).
// The arithmetic per (ray, record) is written with explicit FMAs and compiled without contraction, so
// both paths produce bit-identical colours for the same ray.
#include "dl_internal.h"

namespace dl {
namespace {

constexpr int kUnroll = 4;   // records per step of the record loop (the staged count is padded to a multiple)
constexpr int kColPad = 17;  // LDS colour rows of single-channel rays: r, g and b of a record in three banks


// Staged record, 32 bytes: [u, v, conic A, B (scaled)] [conic C (scaled), bound on E = log2(o) - Q, log2(o), the
// clamp of alpha (blend_cap)]; the colours follow as float4 (RGB rays) or as three rows (single-channel rays).
template <int NT>
struct BlendSmem {
  float4 rec[NT][2];
  float4 rgb[NT];               // unused, r, g, b
  float col[3][NT + kColPad];  // single-channel rays: r, g, b rows
};

// One staged chunk's records [0, n4) for every ray of the lane (n4 a multiple of kUnroll; records past the
// chunk's end are neutral: their bound on E is +inf).
template <bool SC, bool CLAMP, int RPT, bool STATS, int NT>
__device__ __forceinline__ void blend_records(const BlendSmem<NT>& sm, int n4, uint32_t slots,
                                              const float (&px)[RPT], const float (&py)[RPT], float (&sT)[RPT],
                                              float (&C0)[RPT], float (&C1)[RPT], float (&C2)[RPT],
                                              const uint32_t (&ch)[RPT], uint32_t (&nev)[RPT],
                                              uint32_t (&nbl)[RPT], float t_min) {
  for (int k0 = 0; k0 < n4; k0 += kUnroll) {
    const float* colj[RPT];
    if (SC) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) colj[j] = &sm.col[ch[j]][k0];
    }
    const float4(*rp)[2] = &sm.rec[k0];
    const float4* cp = &sm.rgb[k0];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const float4 A = rp[u][0];   // u, v, conic A, B (scaled)
      const float4 CQ = rp[u][1];  // conic C (scaled), E bound, log2(o), clamp
      const float cC = CQ.x, lo = CQ.z, cap = CQ.w;
      float cr = 0.0f, cg = 0.0f, cb = 0.0f;
      if (!SC) {
        const float4 B = cp[u];
        cr = B.y;
        cg = B.z;
        cb = B.w;
      }
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        if (j == 0 || ((slots >> j) & 1u)) {
          // per-pixel rule and front-to-back update, without branches per lane:
          //   E = log2(o) - Q = log2(o) - C dy^2 - (A dx + B dy) dx, alpha = min(cap, 2^E)
          //   T' = T (1 - alpha) as one FMA, the colour weight as T - T' (alpha T up to one rounding of T')
          // A finished ray keeps T < 0: then T' < 0 < t_min, so an accepted record only "stops" it again, and
          // the stop writes -|T|, which leaves it unchanged; no liveness test is needed per pair.
          const float dx = px[j] - A.x, dy = py[j] - A.y;
          const float E = fmaf(-fmaf(A.w, dy, A.z * dx), dx, fmaf(-(cC * dy), dy, lo));
          const bool ok = E >= CQ.y;
          const float T = sT[j];
          if (STATS) nev[j] += T > 0.0f ? 1u : 0u;
          // a record that no lane of the wavefront accepts changes nothing (T' = T, weight 0): the rest is
          // skipped by a scalar branch on the compare's lane mask (about 12% of the (record, 64-ray slot) pairs
          // at 3840x2160, N = 45, by the count of exponentials)
          if (__ballot(ok) != 0ull) {
            const float ga = __builtin_amdgcn_exp2f(E);
            const float alpha = CLAMP ? fminf(cap, ga) : ga;
            const float tn = fmaf(-alpha, T, T);
            const bool stop = ok && (tn < t_min);
            const bool take = ok != stop;  // ok and not stop (stop implies ok): one scalar mask operation
            const float Tt = take ? tn : T;
            const float w = T - Tt;
            if (STATS) nbl[j] += take ? 1u : 0u;
            if (SC) {
              C0[j] = fmaf(w, colj[j][u], C0[j]);
            } else {
              C0[j] = fmaf(w, cr, C0[j]);
              C1[j] = fmaf(w, cg, C1[j]);
              C2[j] = fmaf(w, cb, C2[j]);
            }
            sT[j] = stop ? -fabsf(T) : Tt;
          }
        }
      }
    }
    // leave the chunk once no ray of the wavefront is live
    bool any_live = false;
#pragma unroll
    for (int j = 0; j < RPT; ++j) any_live |= sT[j] > 0.0f;
    if (__ballot(any_live) == 0ull) break;
  }
}

// Occupancy: a lane with up to 4 rays is held to the registers of 8 wavefronts per SIMD (64 VGPRs; the compiler
// spills a few values of the cold paths): the latency of the LDS broadcasts and of the exponential is hidden by more
// wavefronts, measured 8% faster per launch than the 112-VGPR form at 4 wavefronts (3840x2160, N = 45); more rays per
// lane get 6 or 4 wavefronts.  (The second argument of the launch bounds is the minimum of wavefronts per SIMD.)
template <int RPT>
constexpr int blend_min_waves() {
  return RPT <= 4 ? 8 : (RPT <= 6 ? 6 : 4);
}

template <bool STD, bool SC, int RPT, bool STATS, int NT>
__global__ __launch_bounds__(NT, (blend_min_waves<RPT>())) void blend_kernel(const float4* __restrict__ rec,
                                                   const uint32_t* __restrict__ tile_start,
                                                   const uint32_t* __restrict__ gidx,
                                                   const uint32_t* __restrict__ ray_off,
                                                   const uint32_t* __restrict__ ray_ent, BlendConst bc,
                                                   BlendChunk bk, uint8_t* __restrict__ alive,
                                                   float4* __restrict__ state, float* __restrict__ out) {
  __shared__ BlendSmem<NT> sm;
  // Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b mod 8).  XCD x takes tiles x, x + 8,
  // x + 16, ..., each with its N views in a row: all views of a tile run on one XCD at about the same time, so the
  // partial writes of their interleaved subpixels meet in that XCD's L2, and every XCD gets tiles from the whole
  // image (contiguous bands of tile rows left the XCDs with the dense middle rows last to finish: 8% slower).
  const uint32_t xcd = blockIdx.x & 7u, kk = blockIdx.x >> 3;
  const int t = (int)((kk / (uint32_t)bc.N) * 8u + xcd);
  const int v = (int)(kk % (uint32_t)bc.N);
  if (t >= bc.T) return;
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
  // (single-channel rays accumulate their one channel in C0; ch is that channel)
  // (the ray's state slot and channel mask are not kept across the record loop: they are recomputed from the pixel
  // position, the ray list and the thread index where needed, so that the loop's registers stay within the
  // occupancy bound without spilling)
  float px[RPT], py[RPT], sT[RPT], C0[RPT], C1[RPT], C2[RPT];
  uint32_t ch[RPT], nev[RPT], nbl[RPT];
  const auto state_slot = [&](int j) -> int64_t {
    if (STD)
      return ((int64_t)v * bc.H + (int)(py[j] - 0.5f)) * bc.W + (int)(px[j] - 0.5f);
    return (int64_t)r0 + threadIdx.x + j * NT;
  };
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * NT;
    const bool valid = idx < nr;
    int lx = 0, ly = 0;
    uint32_t mask = 0;
    if (valid) {
      if (STD) {
        ly = idx / cw;
        lx = idx - ly * cw;
        mask = 7u;
      } else {
        const uint32_t e = ray_ent[r0 + idx];
        lx = (int)(e & 0xfffu);
        ly = (int)((e >> 12) & 0xfffu);
        mask = (e >> 24) & 7u;
      }
    }
    ch[j] = min(mask >> 1, 2u);  // the channel of a one-channel mask (1, 2, 4 -> 0, 1, 2)
    px[j] = (float)(ox + lx) + 0.5f;
    py[j] = (float)(oy + ly) + 0.5f;
    sT[j] = valid ? 1.0f : -1.0f;
    C0[j] = C1[j] = C2[j] = 0.0f;
    if (valid && !bk.first) {
      const float4 st = state[state_slot(j)];
      sT[j] = st.x;
      if (SC) {
        C0[j] = ch[j] == 0 ? st.y : (ch[j] == 1 ? st.z : st.w);
      } else {
        C0[j] = st.y;
        C1[j] = st.z;
        C2[j] = st.w;
      }
    }
    nev[j] = nbl[j] = 0;
  }
  const float t_min = bc.t_min;
  const uint32_t ls = tile_start[vt];
  const uint32_t le = tile_start[vt + 1];
  const float4* vrec = rec + (int64_t)v * bc.G * kRecF4;

  for (uint32_t base = ls; base < le; base += NT) {
    const int n = (int)min((uint32_t)NT, le - base);
    const int n4 = (n + kUnroll - 1) / kUnroll * kUnroll;
    bool need_clamp = false;
    if ((int)threadIdx.x < n) {
      const uint32_t g = gidx[base + threadIdx.x];
      const float4* src = vrec + (int64_t)g * kRecF4;
      const float4 r0v = src[0], r1 = src[1], r2 = src[2];
      const float lo = __builtin_amdgcn_logf(r2.x);  // log2(o)
      const float cap = blend_cap(r2.x, bc);
      need_clamp = cap < __builtin_inff();
      // the LDS copy carries log2(o) in place of o and, in place of the binning's Q limit, the blend's bound on
      // E = log2(o) - Q (see blend_elim)
      sm.rec[threadIdx.x][0] = r0v;
      sm.rec[threadIdx.x][1] = make_float4(r1.x, blend_elim(lo, bc), lo, cap);
      if (SC) {
        sm.col[0][threadIdx.x] = r2.y;
        sm.col[1][threadIdx.x] = r2.z;
        sm.col[2][threadIdx.x] = r2.w;
      } else {
        sm.rgb[threadIdx.x] = r2;
      }
    } else if ((int)threadIdx.x < n4) {
      // padding to the unrolled step: a record no ray can accept
      sm.rec[threadIdx.x][0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      sm.rec[threadIdx.x][1] = make_float4(0.0f, __builtin_inff(), 0.0f, __builtin_inff());
      if (SC)
        sm.col[0][threadIdx.x] = sm.col[1][threadIdx.x] = sm.col[2][threadIdx.x] = 0.0f;
      else
        sm.rgb[threadIdx.x] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    const bool clamp = __syncthreads_or(need_clamp);
    // bit j: the wavefront has a live ray in slot j (slots other than the first are often empty); wave-uniform
    uint32_t slots = 0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) slots |= (__ballot(sT[j] > 0.0f) != 0ull ? 1u : 0u) << j;
    slots = __builtin_amdgcn_readfirstlane(slots);
    if (slots) {
      if (clamp)
        blend_records<SC, true, RPT, STATS, NT>(sm, n4, slots, px, py, sT, C0, C1, C2, ch, nev, nbl, t_min);
      else
        blend_records<SC, false, RPT, STATS, NT>(sm, n4, slots, px, py, sT, C0, C1, C2, ch, nev, nbl, t_min);
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
  if (tile_live && threadIdx.x == 0 && bk.later) *bk.later = 1ull;  // every writer stores the same value

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
      unsigned long long* sl = bc.stats + 3 * ((blockIdx.x * 4 + (threadIdx.x >> 6)) % kStatSlots);
      atomicAdd(&sl[0], e);
      atomicAdd(&sl[1], b);
      atomicAdd(&sl[2], r);
    }
  }

#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * NT;
    if (idx >= nr) continue;
    if (SC) {
      // the state and the image carry the ray's channel only
      const uint32_t k = ch[j];
      if (!bk.last && tile_live) {
        const float c[3] = {k == 0 ? C0[j] : 0.0f, k == 1 ? C0[j] : 0.0f, k == 2 ? C0[j] : 0.0f};
        state[state_slot(j)] = make_float4(sT[j], c[0], c[1], c[2]);
      }
      if (bk.last || !tile_live) {
        const int xr = (int)(py[j] - 0.5f), yc = (int)(px[j] - 0.5f);
        const float bgk = k == 0 ? bc.bg[0] : (k == 1 ? bc.bg[1] : bc.bg[2]);
        out[((int64_t)xr * bc.W + yc) * 3 + k] = fmaf(fabsf(sT[j]), bgk, C0[j]);
      }
      continue;
    }
    if (!bk.last && tile_live) state[state_slot(j)] = make_float4(sT[j], C0[j], C1[j], C2[j]);
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
        const uint32_t e = ray_ent[r0 + idx];
        const uint32_t mask = (e >> 24) & 7u;
        if (bc.tgt) {
          // repurposed panel: channel k of the ray fills the subpixel listed for it
          const uint32_t sl = (e >> 27) & 3u;
          const int32_t* tg = bc.tgt + ((int64_t)3 * ((int64_t)xr * bc.W + yc) + sl) * 3;
#pragma unroll
          for (int k = 0; k < 3; ++k)
            if (mask & (1u << k)) out[tg[k]] = c[k];
        } else {
          float* dst = out + ((int64_t)xr * bc.W + yc) * 3;
#pragma unroll
          for (int k = 0; k < 3; ++k)
            if (mask & (1u << k)) dst[k] = c[k];
        }
      }
    }
  }
}

template <bool STD, bool SC, int NT>
hipError_t launch_rpt(int rpt, unsigned nblocks, const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                      const uint32_t* ray_off, const uint32_t* ray_ent, const BlendConst& bc, BlendChunk bk,
                      uint8_t* alive, float4* state, float* out, hipStream_t s) {
#define DL_BLEND_CASE(R)                                                                                        \
  case R:                                                                                                      \
    if (bc.stats)                                                                                              \
      hipLaunchKernelGGL((blend_kernel<STD, SC, R, true, NT>), dim3(nblocks), dim3(NT), 0, s, rec, tile_start, \
                         gidx, ray_off, ray_ent, bc, bk, alive, state, out);                                   \
    else                                                                                                       \
      hipLaunchKernelGGL((blend_kernel<STD, SC, R, false, NT>), dim3(nblocks), dim3(NT), 0, s, rec,            \
                         tile_start, gidx, ray_off, ray_ent, bc, bk, alive, state, out);                       \
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
template <bool STD, bool SC>
hipError_t launch_blend(int max_rays, unsigned nblocks, const float4* rec, const uint32_t* tile_start,
                        const uint32_t* gidx, const uint32_t* ray_off, const uint32_t* ray_ent, const BlendConst& bc,
                        BlendChunk bk, uint8_t* alive, float4* state, float* out, hipStream_t s) {
  if (max_rays <= 4 * 256)
    return launch_rpt<STD, SC, 256>(std::max(1, (max_rays + 255) / 256), nblocks, rec, tile_start, gidx, ray_off,
                                    ray_ent, bc, bk, alive, state, out, s);
  if (max_rays > 8 * 512) return hipErrorInvalidValue;
  return launch_rpt<STD, SC, 512>((max_rays + 511) / 512, nblocks, rec, tile_start, gidx, ray_off, ray_ent, bc, bk,
                                  alive, state, out, s);
}

}  // namespace

hipError_t launch_blend_directl(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                const uint32_t* ray_off, const uint32_t* ray_ent, int max_rays,
                                const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state, float* out,
                                hipStream_t s) {
  const unsigned nb = (unsigned)((int64_t)bc.N * 8 * ((bc.T + 7) / 8));  // whole rounds of 8 tiles
  if (nb == 0) return hipSuccess;
  if (bc.single_channel && !bc.tgt)
    return launch_blend<false, true>(max_rays, nb, rec, tile_start, gidx, ray_off, ray_ent, bc, bk, alive, state,
                                     out, s);
  return launch_blend<false, false>(max_rays, nb, rec, tile_start, gidx, ray_off, ray_ent, bc, bk, alive, state, out,
                                    s);
}

hipError_t launch_blend_standard(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                 const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state, float* views,
                                 hipStream_t s) {
  const unsigned nb = (unsigned)((int64_t)bc.N * 8 * ((bc.T + 7) / 8));  // whole rounds of 8 tiles
  if (nb == 0) return hipSuccess;
  return launch_blend<true, false>(bc.tw * bc.th, nb, rec, tile_start, gidx, nullptr, nullptr, bc, bk, alive, state,
                                   views, s);
}

}  // namespace dl

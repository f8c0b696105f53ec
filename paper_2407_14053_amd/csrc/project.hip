// Per-view EWA projection and SH colour of every Gaussian (Eq. (7)-(9) and Sec. 3.3), gfx950.
//
// One thread per Gaussian reads its 59 parameters once (coalesced structure-of-arrays rows), builds
// Sigma = R S S^T R^T once, then loops over the N views of the rig: camera transform, Jacobian J of the
// perspective map, Sigma' = J W Sigma W^T J^T + h I, its inverse (the conic), the projected mean and the
// cutoff ellipse, the depth key and the view-dependent colour.  The render path keeps only the keys from that
// loop, plus one block of each Gaussian's view-independent terms; the records of the ranks the depth order
// keeps are then built from the blocks by the same device functions (most (view, Gaussian) records of a
// dense scene are never read).  Geometry runs in FP64 (the chip's vector
// FP64 rate makes this free next to the memory traffic) and the record is rounded to FP32 once, so the
// FP32 blend starts from correctly rounded inputs; depth keys keep 31 mantissa bits of the FP64 z and its
// exponent counted from that of z_near (36 bits: four radix passes of 9 bits).
// The conic is stored pre-multiplied by log2(e)/2 (A, C) and log2(e) (B), so that the blend evaluates
// alpha = o * 2^-(A dx^2 + B dx dy + C dy^2) with one hardware exp2.
#include "dl_internal.h"

namespace dl {
namespace {

// View-independent terms of one Gaussian (FP64 geometry from its FP32 parameters).
struct GaussTerms {
  double mx, my, mz;  // mean
  double Sg[6];       // Sigma = R diag(s^2) R^T (Eq. (8)), symmetric: xx xy xz yy yz zz
  double qlim;        // tile-test cutoff of the quadratic form
  float o32;          // opacity
};

template <int DEG>
__device__ __forceinline__ void gaussian_terms(const float* __restrict__ soa, int64_t np, int64_t ii, const ProjConst& pc,
                                      GaussTerms& g, float* shc) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  g.mx = soa[kRowMean * np + ii];
  g.my = soa[(kRowMean + 1) * np + ii];
  g.mz = soa[(kRowMean + 2) * np + ii];
  // quaternion (w, x, y, z) normalised
  double qw = soa[kRowQuat * np + ii], qx = soa[(kRowQuat + 1) * np + ii];
  double qy = soa[(kRowQuat + 2) * np + ii], qz = soa[(kRowQuat + 3) * np + ii];
  const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  const double Rq[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                        2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                        2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
  double s2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double sc = exp((double)soa[(kRowLogScale + k) * np + ii]);
    s2[k] = sc * sc;
  }
  {
    int o = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        g.Sg[o++] = Rq[a * 3 + 0] * s2[0] * Rq[b * 3 + 0] + Rq[a * 3 + 1] * s2[1] * Rq[b * 3 + 1] +
                    Rq[a * 3 + 2] * s2[2] * Rq[b * 3 + 2];
      }
  }
  const double opac = 1.0 / (1.0 + exp(-(double)soa[kRowLogit * np + ii]));
  g.o32 = (float)opac;
  // effective cutoff of the ellipse for tile tests: beyond q = 2 ln(o / alpha_min) alpha < alpha_min
  double qlim = pc.q_cut;
  if (opac > pc.alpha_min) qlim = fmin(qlim, 2.0 * log(opac / (double)pc.alpha_min));
  g.qlim = qlim * (1.0 + 1e-4) + 1e-3;
#pragma unroll
  for (int k = 0; k < NB * 3; ++k) shc[k] = soa[(kRowSH + k) * np + ii];
}

// One view: camera z, visibility (in front of z_near, opacity able to reach alpha_min, cutoff ellipse reaching
// a pixel centre), the depth key, and record words 0-8 when visible.
__device__ __forceinline__ bool view_geometry(const double* cam, const ProjConst& pc, const GaussTerms& g, float* r,
                                     uint64_t& key, double& Zo) {
  constexpr double ks = 0.72134752044448170368;  // log2(e) / 2
  // FP64 chain as explicit FMAs (one rounding per multiply-add)
  const double X = fma(cam[0], g.mx, fma(cam[1], g.my, fma(cam[2], g.mz, cam[9])));
  const double Y = fma(cam[3], g.mx, fma(cam[4], g.my, fma(cam[5], g.mz, cam[10])));
  const double Z = fma(cam[6], g.mx, fma(cam[7], g.my, fma(cam[8], g.mz, cam[11])));
  Zo = Z;
  key = kDepthCulled;
  bool vis = (Z > (double)pc.z_near) && (g.o32 >= pc.alpha_min);
  if (!vis) return false;
  // T = J W, rows of the 2x3 product
  const double iz = 1.0 / Z;
  const double f = pc.focal;
  const double fz = f * iz, xz = X * iz, yz = Y * iz;
  double T0[3], T1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T0[k] = fz * fma(-xz, cam[6 + k], cam[k]);
    T1[k] = fz * fma(-yz, cam[6 + k], cam[3 + k]);
  }
  // Sigma' = T Sigma T^T + h I
  const double* Sg = g.Sg;
  const double S0[3] = {fma(Sg[0], T0[0], fma(Sg[1], T0[1], Sg[2] * T0[2])),
                        fma(Sg[1], T0[0], fma(Sg[3], T0[1], Sg[4] * T0[2])),
                        fma(Sg[2], T0[0], fma(Sg[4], T0[1], Sg[5] * T0[2]))};
  const double S1[3] = {fma(Sg[0], T1[0], fma(Sg[1], T1[1], Sg[2] * T1[2])),
                        fma(Sg[1], T1[0], fma(Sg[3], T1[1], Sg[4] * T1[2])),
                        fma(Sg[2], T1[0], fma(Sg[4], T1[1], Sg[5] * T1[2]))};
  const double dil = (double)pc.dilation;
  const double ca = fma(T0[0], S0[0], fma(T0[1], S0[1], fma(T0[2], S0[2], dil)));
  const double cb = fma(T1[0], S0[0], fma(T1[1], S0[1], T1[2] * S0[2]));
  const double cc = fma(T1[0], S1[0], fma(T1[1], S1[1], fma(T1[2], S1[2], dil)));
  const double idet = 1.0 / fma(ca, cc, -(cb * cb));
  const double u = fma(f, xz, pc.cx);
  const double w = fma(f, yz, pc.cy);
  // conservative half-extents of the cutoff ellipse (FP32 square roots; the margins dwarf their error)
  const float ex = sqrtf((float)(g.qlim * ca)) * (1.0f + 1e-4f) + 1e-3f;
  const float ey = sqrtf((float)(g.qlim * cc)) * (1.0f + 1e-4f) + 1e-3f;
  // the ellipse must reach a pixel centre: centres span [0.5, W - 0.5] x [0.5, H - 0.5]
  vis = (u + ex >= 0.5) && (u - ex <= pc.W - 0.5) && (w + ey >= 0.5) && (w - ey <= pc.H - 0.5);
  if (!vis) return false;
  r[0] = (float)u; r[1] = (float)w;
  r[2] = (float)(ks * cc * idet); r[3] = (float)(-2.0 * ks * cb * idet); r[4] = (float)(ks * ca * idet);
  r[5] = (float)(ks * g.qlim); r[6] = ex; r[7] = ey;
  r[8] = g.o32;
  const uint64_t zb = (uint64_t)__double_as_longlong(Z);
  const int e = (int)(zb >> 52) - pc.key_e0;  // >= 0 since Z > z_near
  key = e > kDepthExpMax ? (((uint64_t)(kDepthExpMax + 1) << kDepthMantBits) - 1)
                         : (((uint64_t)e << kDepthMantBits) |
                            ((zb >> (52 - kDepthMantBits)) & ((1ull << kDepthMantBits) - 1)));
  return true;
}

// Record words 9-11: the view-dependent colour, SH evaluated in FP32 in the direction from the camera centre.
template <int DEG>
__device__ __forceinline__ void view_colour(const double* cam, const GaussTerms& g, const float* shc, float* r) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const float dx = (float)(g.mx - cam[12]), dy = (float)(g.my - cam[13]), dz = (float)(g.mz - cam[14]);
  const float dn = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  float Yb[16];
  sh_basis(DEG, dx * dn, dy * dn, dz * dn, Yb);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.5f;
#pragma unroll
    for (int l = 0; l < NB; ++l) acc = fmaf(Yb[l], shc[l * 3 + c], acc);
    r[9 + c] = fmaxf(acc, 0.0f);
  }
}

// Per-Gaussian block (kGaussBlockF4 float4): Sigma (6 doubles), mean (3 doubles), q_lim (double), opacity
// (float, then 3 unused words), SH (NSH <= 48 floats, zero-padded to whole float4).
template <int NSH>
__device__ __forceinline__ void store_block(float4* blk, const GaussTerms& g, const float* shc) {
  double2* d2 = reinterpret_cast<double2*>(blk);
  d2[0] = make_double2(g.Sg[0], g.Sg[1]);
  d2[1] = make_double2(g.Sg[2], g.Sg[3]);
  d2[2] = make_double2(g.Sg[4], g.Sg[5]);
  d2[3] = make_double2(g.mx, g.my);
  d2[4] = make_double2(g.mz, g.qlim);
  blk[5] = make_float4(g.o32, 0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int k = 0; k < (NSH + 3) / 4; ++k)
    blk[6 + k] = make_float4(shc[4 * k], 4 * k + 1 < NSH ? shc[4 * k + 1] : 0.0f,
                             4 * k + 2 < NSH ? shc[4 * k + 2] : 0.0f, 4 * k + 3 < NSH ? shc[4 * k + 3] : 0.0f);
}

template <int NSH>
__device__ __forceinline__ void load_block(const float4* blk, GaussTerms& g, float* shc) {
  const double2* d2 = reinterpret_cast<const double2*>(blk);
  const double2 a = d2[0], b = d2[1], c = d2[2], d = d2[3], e = d2[4];
  g.Sg[0] = a.x; g.Sg[1] = a.y; g.Sg[2] = b.x; g.Sg[3] = b.y; g.Sg[4] = c.x; g.Sg[5] = c.y;
  g.mx = d.x; g.my = d.y; g.mz = e.x; g.qlim = e.y;
  g.o32 = blk[5].x;
#pragma unroll
  for (int k = 0; k < (NSH + 3) / 4; ++k) {
    const float4 q = blk[6 + k];
    shc[4 * k] = q.x;
    if (4 * k + 1 < NSH) shc[4 * k + 1] = q.y;
    if (4 * k + 2 < NSH) shc[4 * k + 2] = q.z;
    if (4 * k + 3 < NSH) shc[4 * k + 3] = q.w;
  }
}

// Projection of every (view, Gaussian), one thread per Gaussian looping over the views.  RECORDS: every live
// lane writes its 48-byte record (zeros when culled: full 128-byte lines reach HBM, where the visible records
// alone, with holes in most lines, were written 20% slower despite 30% fewer bytes).  Otherwise only the keys
// are written, with each Gaussian's block of view-independent terms, from which the records of the depth-sorted
// ranks are built later (project_ranks_kernel, the same arithmetic).
template <int DEG, bool RECORDS>
__global__ __launch_bounds__(256, 4) void project_kernel(const float* __restrict__ soa, const double* __restrict__ cams,
                                                      ProjConst pc, float4* __restrict__ rec,
                                                      uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                      double* __restrict__ depth_out, uint32_t* __restrict__ fhist) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < pc.G;
  const int64_t ii = live ? i : 0;
  GaussTerms g;
  float shc[NB * 3];
  gaussian_terms<DEG>(soa, pc.n_pad, ii, pc, g, shc);
  if (!RECORDS && live) store_block<NB * 3>(rec + i * kGaussBlockF4, g, shc);
  const bool sampled = fhist && (i % kFrontSamplePeriod) < kFrontSampleRun;
  // two views per loop step (their FP64 chains are independent; 72 VGPRs, no spill): the same time at 300k
  // Gaussians, 0.5% faster frames at 3M
#pragma unroll 2
  for (int v = 0; v < pc.N; ++v) {
    const double* cam = cams + v * kCamDoubles;
    float r[12] = {};
    uint64_t key;
    double Z;
    const bool vis = live && view_geometry(cam, pc, g, r, key, Z);
    if (RECORDS && vis) view_colour<DEG>(cam, g, shc, r);
    const int64_t o = (int64_t)v * pc.G + i;
    if (live) {
      keys[o] = vis ? key : kDepthCulled;
      if (sampled && vis)
        atomicAdd(&fhist[((int64_t)v << kFrontBits) + (uint32_t)(key >> (kDepthKeyBits - kFrontBits))], 1u);
      if (vals) vals[o] = (uint32_t)i;
      if (RECORDS) {
        float4* dst = rec + o * kRecF4;
        dst[0] = make_float4(r[0], r[1], r[2], r[3]);
        dst[1] = make_float4(r[4], r[5], r[6], r[7]);
        dst[2] = make_float4(r[8], r[9], r[10], r[11]);
      }
      if (depth_out) depth_out[o] = vis ? Z : __longlong_as_double(0x7ff8000000000000ll);
    }
  }
}

// Records in depth order, built from the Gaussians' blocks: out[v][r] = record of (view v, Gaussian
// sorted[v][r]) for the ranks r in [rank_lo[v], rank_hi[v]) of view v (rank_lo nullptr: 0), so that binning
// reads consecutive records and the blend's list entries are ranks.  Every such Gaussian is visible in view v.
template <int DEG>
__global__ __launch_bounds__(256) void project_ranks_kernel(const float4* __restrict__ blocks,
                                                            const double* __restrict__ cams, ProjConst pc,
                                                            const uint32_t* __restrict__ sorted,
                                                            const uint32_t* __restrict__ rank_lo,
                                                            const uint32_t* __restrict__ rank_hi,
                                                            float4* __restrict__ out) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const int v = blockIdx.y;
  const int64_t G = pc.G;
  const int64_t o = (int64_t)v * G;
  const int64_t hi = rank_hi[v];
  const double* cam = cams + v * kCamDoubles;
  for (int64_t r = (rank_lo ? rank_lo[v] : 0) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < hi;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = sorted[o + r];
    GaussTerms g;
    float shc[NB * 3];
    load_block<NB * 3>(blocks + (int64_t)i * kGaussBlockF4, g, shc);
    float rr[12] = {};
    uint64_t key;
    double Z;
    view_geometry(cam, pc, g, rr, key, Z);
    view_colour<DEG>(cam, g, shc, rr);
    float4* dst = out + (o + r) * kRecF4;
    dst[0] = make_float4(rr[0], rr[1], rr[2], rr[3]);
    dst[1] = make_float4(rr[4], rr[5], rr[6], rr[7]);
    dst[2] = make_float4(rr[8], rr[9], rr[10], rr[11]);
  }
}

__global__ __launch_bounds__(256) void scene_transpose_kernel(const float* __restrict__ means,
                                                              const float* __restrict__ log_scales,
                                                              const float* __restrict__ quats,
                                                              const float* __restrict__ logits,
                                                              const float* __restrict__ sh, int64_t n, int64_t n_pad,
                                                              float* __restrict__ soa) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) soa[(kRowMean + k) * n_pad + i] = means[i * 3 + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) soa[(kRowLogScale + k) * n_pad + i] = log_scales[i * 3 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) soa[(kRowQuat + k) * n_pad + i] = quats[i * 4 + k];
  soa[kRowLogit * n_pad + i] = logits[i];
  for (int k = 0; k < 48; ++k) soa[(kRowSH + k) * n_pad + i] = sh[i * 48 + k];
}

}  // namespace

hipError_t launch_project(const float* soa, const double* cams, const ProjConst& pc, float4* rec, uint64_t* keys,
                          uint32_t* vals, double* depth_out, hipStream_t s) {
  const dim3 grid((unsigned)((pc.G + 255) / 256));
  switch (pc.sh_degree) {
    case 0: hipLaunchKernelGGL((project_kernel<0, true>), grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out, nullptr); break;
    case 1: hipLaunchKernelGGL((project_kernel<1, true>), grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out, nullptr); break;
    case 2: hipLaunchKernelGGL((project_kernel<2, true>), grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out, nullptr); break;
    default: hipLaunchKernelGGL((project_kernel<3, true>), grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out, nullptr); break;
  }
  return hipGetLastError();
}

hipError_t launch_project_keys(const float* soa, const double* cams, const ProjConst& pc, float4* blocks,
                               uint64_t* keys, uint32_t* fhist, hipStream_t s) {
  const dim3 grid((unsigned)((pc.G + 255) / 256));
  switch (pc.sh_degree) {
    case 0: hipLaunchKernelGGL((project_kernel<0, false>), grid, dim3(256), 0, s, soa, cams, pc, blocks, keys, nullptr, nullptr, fhist); break;
    case 1: hipLaunchKernelGGL((project_kernel<1, false>), grid, dim3(256), 0, s, soa, cams, pc, blocks, keys, nullptr, nullptr, fhist); break;
    case 2: hipLaunchKernelGGL((project_kernel<2, false>), grid, dim3(256), 0, s, soa, cams, pc, blocks, keys, nullptr, nullptr, fhist); break;
    default: hipLaunchKernelGGL((project_kernel<3, false>), grid, dim3(256), 0, s, soa, cams, pc, blocks, keys, nullptr, nullptr, fhist); break;
  }
  return hipGetLastError();
}

hipError_t launch_project_ranks(const float4* blocks, const double* cams, const ProjConst& pc,
                                const uint32_t* sorted, const uint32_t* rank_lo, const uint32_t* rank_hi,
                                int64_t max_ranks, float4* out, hipStream_t s) {
  const int64_t m = std::max<int64_t>(1, std::min<int64_t>(max_ranks, pc.G));
  const dim3 grid((unsigned)std::min<int64_t>((m + 255) / 256, 256), (unsigned)pc.N);
  switch (pc.sh_degree) {
    case 0: hipLaunchKernelGGL(project_ranks_kernel<0>, grid, dim3(256), 0, s, blocks, cams, pc, sorted, rank_lo, rank_hi, out); break;
    case 1: hipLaunchKernelGGL(project_ranks_kernel<1>, grid, dim3(256), 0, s, blocks, cams, pc, sorted, rank_lo, rank_hi, out); break;
    case 2: hipLaunchKernelGGL(project_ranks_kernel<2>, grid, dim3(256), 0, s, blocks, cams, pc, sorted, rank_lo, rank_hi, out); break;
    default: hipLaunchKernelGGL(project_ranks_kernel<3>, grid, dim3(256), 0, s, blocks, cams, pc, sorted, rank_lo, rank_hi, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_scene_transpose(const float* means, const float* log_scales, const float* quats,
                                  const float* logits, const float* sh, int64_t n, int64_t n_pad, float* soa,
                                  hipStream_t s) {
  hipLaunchKernelGGL(scene_transpose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, means, log_scales,
                     quats, logits, sh, n, n_pad, soa);
  return hipGetLastError();
}

}  // namespace dl

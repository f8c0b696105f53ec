// Per-view EWA projection and SH colour of every Gaussian (Eq. (7)-(9) and Sec. 3.3), gfx950.
//
// One thread per Gaussian reads its 59 parameters once (coalesced structure-of-arrays rows), builds
// Sigma = R S S^T R^T once, then loops over the N views of the rig: camera transform, Jacobian J of the
// perspective map, Sigma' = J W Sigma W^T J^T + h I, its inverse (the conic), the projected mean and the
// cutoff ellipse, the depth key and the view-dependent colour.  Geometry runs in FP64 (the chip's vector
// FP64 rate makes this free next to the memory traffic) and the record is rounded to FP32 once, so the
// FP32 blend starts from correctly rounded inputs; depth keys keep 31 mantissa bits of the FP64 z and its
// exponent counted from that of z_near (36 bits: four radix passes of 9 bits).
// The conic is stored pre-multiplied by log2(e)/2 (A, C) and log2(e) (B), so that the blend evaluates
// alpha = o * 2^-(A dx^2 + B dx dy + C dy^2) with one hardware exp2.
#include "dl_internal.h"

namespace dl {
namespace {

template <int DEG>
__global__ __launch_bounds__(256, 4) void project_kernel(const float* __restrict__ soa, const double* __restrict__ cams,
                                                      ProjConst pc, float4* __restrict__ rec,
                                                      uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                      double* __restrict__ depth_out) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < pc.G;
  const int64_t ii = live ? i : 0;
  const int64_t np = pc.n_pad;
  const double mx = soa[kRowMean * np + ii], my = soa[(kRowMean + 1) * np + ii], mz = soa[(kRowMean + 2) * np + ii];
  // Sigma = R diag(s^2) R^T (Eq. (8)), quaternion (w, x, y, z) normalised
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
    const double s = exp((double)soa[(kRowLogScale + k) * np + ii]);
    s2[k] = s * s;
  }
  double Sg[6];  // symmetric: xx xy xz yy yz zz
  {
    int o = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        Sg[o++] = Rq[a * 3 + 0] * s2[0] * Rq[b * 3 + 0] + Rq[a * 3 + 1] * s2[1] * Rq[b * 3 + 1] +
                  Rq[a * 3 + 2] * s2[2] * Rq[b * 3 + 2];
      }
  }
  const double opac = 1.0 / (1.0 + exp(-(double)soa[kRowLogit * np + ii]));
  const float o32 = (float)opac;
  // effective cutoff of the ellipse for tile tests: beyond q = 2 ln(o / alpha_min) alpha < alpha_min
  double qlim = pc.q_cut;
  if (opac > pc.alpha_min) qlim = fmin(qlim, 2.0 * log(opac / (double)pc.alpha_min));
  qlim = qlim * (1.0 + 1e-4) + 1e-3;
  float shc[NB * 3];
#pragma unroll
  for (int k = 0; k < NB * 3; ++k) shc[k] = soa[(kRowSH + k) * np + ii];

  const double ks = 0.72134752044448170368;  // log2(e) / 2
  for (int v = 0; v < pc.N; ++v) {
    const double* cam = cams + v * kCamDoubles;
    // FP64 chain as explicit FMAs (one rounding per multiply-add)
    const double X = fma(cam[0], mx, fma(cam[1], my, fma(cam[2], mz, cam[9])));
    const double Y = fma(cam[3], mx, fma(cam[4], my, fma(cam[5], mz, cam[10])));
    const double Z = fma(cam[6], mx, fma(cam[7], my, fma(cam[8], mz, cam[11])));
    bool vis = live && (Z > (double)pc.z_near) && (o32 >= pc.alpha_min);
    uint64_t key = kDepthCulled;
    float r[12] = {};
    if (vis) {
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
      const float ex = sqrtf((float)(qlim * ca)) * (1.0f + 1e-4f) + 1e-3f;
      const float ey = sqrtf((float)(qlim * cc)) * (1.0f + 1e-4f) + 1e-3f;
      // the ellipse must reach a pixel centre: centres span [0.5, W - 0.5] x [0.5, H - 0.5]
      vis = (u + ex >= 0.5) && (u - ex <= pc.W - 0.5) && (w + ey >= 0.5) && (w - ey <= pc.H - 0.5);
      if (vis) {
        // view direction for the colour, normalised in FP32 (the SH basis is evaluated in FP32)
        const float dx = (float)(mx - cam[12]), dy = (float)(my - cam[13]), dz = (float)(mz - cam[14]);
        const float dn = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
        float Yb[16];
        sh_basis(DEG, dx * dn, dy * dn, dz * dn, Yb);
        float rgb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          float acc = 0.5f;
#pragma unroll
          for (int l = 0; l < NB; ++l) acc = fmaf(Yb[l], shc[l * 3 + c], acc);
          rgb[c] = fmaxf(acc, 0.0f);
        }
        r[0] = (float)u; r[1] = (float)w;
        r[2] = (float)(ks * cc * idet); r[3] = (float)(-2.0 * ks * cb * idet); r[4] = (float)(ks * ca * idet);
        r[5] = (float)(ks * qlim); r[6] = ex; r[7] = ey;
        r[8] = o32; r[9] = rgb[0]; r[10] = rgb[1]; r[11] = rgb[2];
        const uint64_t zb = (uint64_t)__double_as_longlong(Z);
        const int e = (int)(zb >> 52) - pc.key_e0;  // >= 0 since Z > z_near
        key = e > kDepthExpMax ? (((uint64_t)(kDepthExpMax + 1) << kDepthMantBits) - 1)
                               : (((uint64_t)e << kDepthMantBits) |
                                  ((zb >> (52 - kDepthMantBits)) & ((1ull << kDepthMantBits) - 1)));
      }
    }
    const int64_t o = (int64_t)v * pc.G + i;
    if (live) {
      keys[o] = key;
      if (vals) vals[o] = (uint32_t)i;
      {
        // every live lane writes its record (zeros when culled): full 128-byte lines reach HBM, where the
        // visible records alone, with holes in most lines, were written 20% slower despite 30% fewer bytes
        float4* dst = rec + o * kRecF4;
        dst[0] = make_float4(r[0], r[1], r[2], r[3]);
        dst[1] = make_float4(r[4], r[5], r[6], r[7]);
        dst[2] = make_float4(r[8], r[9], r[10], r[11]);
      }
      if (depth_out) depth_out[o] = vis ? Z : __longlong_as_double(0x7ff8000000000000ll);
    }
  }
}

// Records in depth order: rec_sorted[v][r] = rec[v][sorted[v][r]] for the ranks r in [rank_lo[v], rank_hi[v]) of
// view v (rank_lo nullptr: 0), so that binning reads consecutive records and the blend's list entries are ranks.
__global__ __launch_bounds__(256) void gather_records_kernel(const float4* __restrict__ rec,
                                                             const uint32_t* __restrict__ sorted,
                                                             const uint32_t* __restrict__ rank_lo,
                                                             const uint32_t* __restrict__ rank_hi, int64_t G,
                                                             float4* __restrict__ out) {
  const int v = blockIdx.y;
  const int64_t o = (int64_t)v * G;
  const int64_t hi = rank_hi[v];
  for (int64_t r = (rank_lo ? rank_lo[v] : 0) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < hi;
       r += (int64_t)gridDim.x * blockDim.x) {
    const float4* src = rec + (o + sorted[o + r]) * kRecF4;
    float4* dst = out + (o + r) * kRecF4;
    dst[0] = src[0];
    dst[1] = src[1];
    dst[2] = src[2];
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
    case 0: hipLaunchKernelGGL(project_kernel<0>, grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out); break;
    case 1: hipLaunchKernelGGL(project_kernel<1>, grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out); break;
    case 2: hipLaunchKernelGGL(project_kernel<2>, grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out); break;
    default: hipLaunchKernelGGL(project_kernel<3>, grid, dim3(256), 0, s, soa, cams, pc, rec, keys, vals, depth_out); break;
  }
  return hipGetLastError();
}

hipError_t launch_gather_records(const float4* rec, const uint32_t* sorted, const uint32_t* rank_lo,
                                 const uint32_t* rank_hi, int64_t G, int N, float4* out, hipStream_t s) {
  const unsigned per_view = (unsigned)std::min<int64_t>((G + 255) / 256, 256);
  hipLaunchKernelGGL(gather_records_kernel, dim3(per_view, (unsigned)N), dim3(256), 0, s, rec, sorted, rank_lo,
                     rank_hi, G, out);
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

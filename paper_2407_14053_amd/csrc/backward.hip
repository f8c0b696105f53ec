// Backward pass of the DirectL forward (gfx950): gradients of a loss on the encoded image with respect to the
// Gaussian parameters.
//
// The forward is replayed over the same depth chunks and (view, tile) lists, with the same per-ray arithmetic,
// so every threshold and termination decision is the forward's.  Per blended pair j of a ray, with g = dL/dC
// on the ray's owned channels (zero elsewhere) and C the ray's forward output there:
//   dC/dc_j     = alpha_j T_j
//   dC/dalpha_j = T_j c_j - (C - C_<=j) / (1 - alpha_j)        (C_<=j: colour accumulated up to j)
// because C - C_<=j = sum_{k>j} alpha_k T_k c_k + T_end bg is exactly what 1 - alpha_j scales.  This walks
// front to back with no stored per-pixel blend state and no division by a transmittance.  Through
// alpha = min(cap, o 2^-Q) (the forward's clamp, blend_cap; zero gradient when clamped) and Q = A dx^2 + B dx dy + C dy^2 the pair gives
// gradients of the record (u, v, A, B, C, o, r, g, b); they are summed over the wavefront, then over the
// workgroup, and added to a per-(view, Gaussian) accumulator with one atomic per component per tile.
//
// A second kernel (one thread per Gaussian, looping over the views like the projection) chains those through
// the projection in FP64: conic = inverse of Sigma' = T Sigma T^T + h I with T = J W, Sigma = R S^2 R^T,
// the projected mean, the sigmoid, and the SH colour in the direction camera -> mean, and writes the
// gradients in the user layouts, summed over views.
#include "dl_internal.h"

namespace dl {
namespace {

constexpr int kG = 9;  // gradient components per (view, Gaussian): u, v, A, B, C, o, r, g, b

__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t q = nb / 8, rem = nb % 8;
  const uint32_t x = b % 8, k = b / 8;
  return x * q + min(x, rem) + k;
}

// Sums of 9 values over the 64 lanes of a wavefront, as a reduce-scatter: each exchange step halves the values a
// lane carries (8 + 4 + 2 + 1 shuffles, then 2 to finish) instead of reducing every value separately.  On return
// lane l holds the sum of value index(l) = (l5 l4 l3 l2) read as a binary number (bit k of l is lk); lanes with
// l & 3 == 0 carry distinct indices 0..15, of which 0..8 are the values.
__device__ inline float wave_reduce9(const float* g, int lane, int* index) {
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
  float x[8], y[4], z[2];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float lo = g[j], hi = j == 0 ? g[8] : 0.0f;  // indices j and 8 + j
    x[j] = (b5 ? hi : lo) + __shfl_xor(b5 ? lo : hi, 32, 64);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] = (b4 ? x[4 + j] : x[j]) + __shfl_xor(b4 ? x[j] : x[4 + j], 16, 64);
#pragma unroll
  for (int j = 0; j < 2; ++j) z[j] = (b3 ? y[2 + j] : y[j]) + __shfl_xor(b3 ? y[j] : y[2 + j], 8, 64);
  float w = (b2 ? z[1] : z[0]) + __shfl_xor(b2 ? z[0] : z[1], 4, 64);
  w += __shfl_xor(w, 2, 64);
  w += __shfl_xor(w, 1, 64);
  *index = (b5 ? 8 : 0) | (b4 ? 4 : 0) | (b3 ? 2 : 0) | (b2 ? 1 : 0);
  return w;
}

template <int RPT, int NT>
__global__ __launch_bounds__(NT) void blend_bwd_kernel(const float4* __restrict__ rec,
                                                             const uint32_t* __restrict__ tile_start,
                                                             const uint32_t* __restrict__ gidx,
                                                             const uint32_t* __restrict__ sorted,
                                                             const uint32_t* __restrict__ ray_off,
                                                             const uint32_t* __restrict__ ray_ent, BlendConst bc,
                                                             BlendChunk bk, uint8_t* __restrict__ alive,
                                                             float4* __restrict__ state, const float* __restrict__ fwd,
                                                             const float* __restrict__ gout, float* __restrict__ acc) {
  __shared__ float4 sm[NT * kRecF4];
  __shared__ uint32_t sg[NT];          // Gaussian index of each staged entry
  __shared__ float part[NT][kG];       // workgroup sums per staged entry (wavefront sums added in LDS)
  const uint32_t wi = xcd_remap(blockIdx.x, gridDim.x);
  const int v = (int)(wi / (uint32_t)bc.T);
  const int t = (int)(wi - (uint32_t)v * (uint32_t)bc.T);
  const int64_t vt = (int64_t)v * bc.T + t;
  if (!alive[vt]) return;
  const int tx = t % bc.ntx, ty = t / bc.ntx;
  const int ox = tx * bc.tw, oy = ty * bc.th;
  const int r0 = (int)ray_off[vt];
  const int nr = (int)ray_off[vt + 1] - r0;
  if (nr <= 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

  float px[RPT], py[RPT], Tr[RPT], C0[RPT], C1[RPT], C2[RPT];
  float g0[RPT], g1[RPT], g2[RPT], F0[RPT], F1[RPT], F2[RPT];
  int64_t gid[RPT];
  bool live[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * NT;
    const bool valid = idx < nr;
    int lx = 0, ly = 0;
    uint32_t mask = 0, slot = 0;
    if (valid) {
      const uint32_t e = ray_ent[r0 + idx];
      lx = (int)(e & 0xfffu);
      ly = (int)((e >> 12) & 0xfffu);
      mask = (e >> 24) & 7u;
      slot = (e >> 27) & 3u;
    }
    px[j] = (float)(ox + lx) + 0.5f;
    py[j] = (float)(oy + ly) + 0.5f;
    gid[j] = (int64_t)r0 + idx;
    // the subpixel each channel of the ray fills: its own pixel's, or on a repurposed panel the listed one
    const int64_t pix = (int64_t)(oy + ly) * bc.W + ox + lx;
    int64_t at[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) at[k] = bc.tgt ? (int64_t)max(bc.tgt[(3 * pix + slot) * 3 + k], 0) : 3 * pix + k;
    g0[j] = (valid && (mask & 1u)) ? gout[at[0]] : 0.0f;
    g1[j] = (valid && (mask & 2u)) ? gout[at[1]] : 0.0f;
    g2[j] = (valid && (mask & 4u)) ? gout[at[2]] : 0.0f;
    F0[j] = (valid && (mask & 1u)) ? fwd[at[0]] : 0.0f;
    F1[j] = (valid && (mask & 2u)) ? fwd[at[1]] : 0.0f;
    F2[j] = (valid && (mask & 4u)) ? fwd[at[2]] : 0.0f;
    Tr[j] = 1.0f;
    C0[j] = C1[j] = C2[j] = 0.0f;
    live[j] = valid;
    if (valid && !bk.first) {
      const float4 st = state[gid[j]];
      live[j] = !signbit(st.x);
      Tr[j] = fabsf(st.x);
      C0[j] = st.y;
      C1[j] = st.z;
      C2[j] = st.w;
    }
  }
  const float t_min = bc.t_min;
  const uint32_t ls = tile_start[vt];
  const uint32_t le = tile_start[vt + 1];
  const int64_t vG = (int64_t)v * bc.G;
  const float4* vrec = rec + vG * kRecF4;
  const int64_t NG = (int64_t)bc.N * bc.G;
  const float ln2 = 0.69314718055994531f;

  for (uint32_t base = ls; base < le; base += NT) {
    const int n = (int)min((uint32_t)NT, le - base);
    if ((int)threadIdx.x < n) {
      const uint32_t rk = gidx[base + threadIdx.x];
      const float4* src = vrec + (int64_t)rk * kRecF4;
      const float4 r1 = src[1], r2 = src[2];
      const float lo = __builtin_amdgcn_logf(r2.x);
      sm[threadIdx.x * kRecF4 + 0] = src[0];
      // the forward's staging (log2(o), the bound on E = log2(o) - Q and the clamp of alpha), with o itself
      sm[threadIdx.x * kRecF4 + 1] = make_float4(r1.x, blend_elim(lo, bc), r2.x, blend_cap(r2.x, bc));
      sm[threadIdx.x * kRecF4 + 2] = make_float4(lo, r2.y, r2.z, r2.w);
      sg[threadIdx.x] = sorted[vG + rk];
    }
    for (int i = threadIdx.x; i < NT * kG; i += NT) (&part[0][0])[i] = 0.0f;
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int j = 0; j < RPT; ++j) any |= live[j];
    if (__ballot(any) != 0ull) {
      for (int k = 0; k < n; ++k) {
        const float4 A = sm[k * kRecF4 + 0];
        const float4 CQ = sm[k * kRecF4 + 1];  // conic C (scaled), E limit, opacity, clamp of alpha
        const float cC = CQ.x;
        const float4 B = sm[k * kRecF4 + 2];    // log2(opacity), r, g, b
        float gr[kG];
#pragma unroll
        for (int c = 0; c < kG; ++c) gr[c] = 0.0f;
        bool any_live = false, any_take = false;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          // the forward's arithmetic, operation for operation
          const float dx = px[j] - A.x, dy = py[j] - A.y;
          const float E = fmaf(-fmaf(A.w, dy, A.z * dx), dx, fmaf(-(cC * dy), dy, B.x));
          const float ga = __builtin_amdgcn_exp2f(E);  // o 2^-Q
          const float alpha = fminf(CQ.w, ga);
          const bool ok = live[j] && (E >= CQ.y);
          const float tn = fmaf(-alpha, Tr[j], Tr[j]);
          const bool stop = ok && (tn < t_min);
          const bool take = ok && !stop;
          live[j] = live[j] && !stop;
          const float w = take ? Tr[j] - tn : 0.0f;
          const float n0 = fmaf(w, B.y, C0[j]), n1 = fmaf(w, B.z, C1[j]), n2 = fmaf(w, B.w, C2[j]);
          if (take) {
            // dC/dc = alpha T ; dC/dalpha = T c - (C_end - C_<=j) / (1 - alpha)
            const float gc = g0[j] * B.y + g1[j] * B.z + g2[j] * B.w;
            const float gR = g0[j] * (F0[j] - n0) + g1[j] * (F1[j] - n1) + g2[j] * (F2[j] - n2);
            const float da = Tr[j] * gc - gR * __builtin_amdgcn_rcpf(1.0f - alpha);
            gr[6] += g0[j] * w;
            gr[7] += g1[j] * w;
            gr[8] += g2[j] * w;
            if (ga <= CQ.w) {
              const float dQ = -da * ln2 * ga;  // alpha = o 2^-Q
              gr[5] += da * ga * __builtin_amdgcn_rcpf(CQ.z);  // d alpha / d o = 2^-Q
              gr[2] += dQ * dx * dx;
              gr[3] += dQ * dx * dy;
              gr[4] += dQ * dy * dy;
              gr[0] -= dQ * (2.0f * A.z * dx + A.w * dy);
              gr[1] -= dQ * (A.w * dx + 2.0f * cC * dy);
            }
          }
          C0[j] = n0;
          C1[j] = n1;
          C2[j] = n2;
          Tr[j] = take ? tn : Tr[j];
          any_live |= live[j];
          any_take |= take;
        }
        if (__ballot(any_take) != 0ull) {
          int c;
          const float s = wave_reduce9(gr, lane, &c);
          if ((lane & 3) == 0 && c < kG && s != 0.0f) atomicAdd(&part[k][c], s);
        }
        if (__ballot(any_live) == 0ull) break;
      }
    }
    __syncthreads();
    // one atomic per (entry, component) for the whole workgroup
    if ((int)threadIdx.x < n) {
      const uint32_t g = sg[threadIdx.x];
#pragma unroll
      for (int c = 0; c < kG; ++c) {
        const float s = part[threadIdx.x][c];
        if (s != 0.0f) atomicAdd(&acc[(int64_t)c * NG + vG + g], s);
      }
    }
    bool mine = false;
#pragma unroll
    for (int j = 0; j < RPT; ++j) mine |= live[j];
    if (!__syncthreads_or(mine)) break;
  }
  bool mine = false;
#pragma unroll
  for (int j = 0; j < RPT; ++j) mine |= live[j];
  const bool tile_live = __syncthreads_or(mine);
  if (!tile_live && threadIdx.x == 0) alive[vt] = 0;
  if (tile_live && threadIdx.x == 0 && bk.later) *bk.later = 1ull;  // every writer stores the same value
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int idx = threadIdx.x + j * NT;
    if (idx < nr && !bk.last && tile_live) state[gid[j]] = make_float4(live[j] ? Tr[j] : -Tr[j], C0[j], C1[j], C2[j]);
  }
}

// Real SH basis (as in the projection) and its gradient with respect to the unit direction (x, y, z).
template <typename F>
__device__ inline void sh_basis_grad(int deg, F x, F y, F z, F* Y, F* dYx, F* dYy, F* dYz) {
  const F k0 = (F)0.28209479177387814, k1 = (F)0.4886025119029199, k2 = (F)1.0925484305920792,
          k3 = (F)0.31539156525252005, k4 = (F)0.5462742152960396, k5 = (F)0.5900435899266435,
          k6 = (F)2.890611442640554, k7 = (F)0.4570457994644658, k8 = (F)0.3731763325901154, k9 = (F)1.445305721320277;
  for (int l = 0; l < 16; ++l) Y[l] = dYx[l] = dYy[l] = dYz[l] = (F)0;
  Y[0] = k0;
  if (deg < 1) return;
  Y[1] = k1 * y; dYy[1] = k1;
  Y[2] = k1 * z; dYz[2] = k1;
  Y[3] = k1 * x; dYx[3] = k1;
  if (deg < 2) return;
  Y[4] = k2 * x * y; dYx[4] = k2 * y; dYy[4] = k2 * x;
  Y[5] = k2 * y * z; dYy[5] = k2 * z; dYz[5] = k2 * y;
  Y[6] = k3 * (3 * z * z - 1); dYz[6] = 6 * k3 * z;
  Y[7] = k2 * x * z; dYx[7] = k2 * z; dYz[7] = k2 * x;
  Y[8] = k4 * (x * x - y * y); dYx[8] = 2 * k4 * x; dYy[8] = -2 * k4 * y;
  if (deg < 3) return;
  Y[9] = k5 * y * (3 * x * x - y * y); dYx[9] = 6 * k5 * x * y; dYy[9] = k5 * (3 * x * x - 3 * y * y);
  Y[10] = k6 * x * y * z; dYx[10] = k6 * y * z; dYy[10] = k6 * x * z; dYz[10] = k6 * x * y;
  Y[11] = k7 * y * (5 * z * z - 1); dYy[11] = k7 * (5 * z * z - 1); dYz[11] = 10 * k7 * y * z;
  Y[12] = k8 * z * (5 * z * z - 3); dYz[12] = k8 * (15 * z * z - 3);
  Y[13] = k7 * x * (5 * z * z - 1); dYx[13] = k7 * (5 * z * z - 1); dYz[13] = 10 * k7 * x * z;
  Y[14] = k9 * z * (x * x - y * y); dYx[14] = 2 * k9 * x * z; dYy[14] = -2 * k9 * y * z; dYz[14] = k9 * (x * x - y * y);
  Y[15] = k5 * x * (x * x - 3 * y * y); dYx[15] = k5 * (3 * x * x - 3 * y * y); dYy[15] = -6 * k5 * x * y;
}

// The forward's FP32 colour of one channel before the clamp (same operations as the projection).
__device__ inline float raw_colour_f32(int deg, float x, float y, float z, const float* shc, int c) {
  float Y[16];
  Y[0] = 0.28209479177387814f;
  const int nb = (deg + 1) * (deg + 1);
  if (deg >= 1) {
    Y[1] = 0.4886025119029199f * y;
    Y[2] = 0.4886025119029199f * z;
    Y[3] = 0.4886025119029199f * x;
  }
  if (deg >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * (x * y);
    Y[5] = 1.0925484305920792f * (y * z);
    Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
    Y[7] = 1.0925484305920792f * (x * z);
    Y[8] = 0.5462742152960396f * (xx - yy);
    if (deg >= 3) {
      Y[9] = 0.5900435899266435f * y * (3.0f * xx - yy);
      Y[10] = 2.890611442640554f * (x * y) * z;
      Y[11] = 0.4570457994644658f * y * (5.0f * zz - 1.0f);
      Y[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
      Y[13] = 0.4570457994644658f * x * (5.0f * zz - 1.0f);
      Y[14] = 1.445305721320277f * z * (xx - yy);
      Y[15] = 0.5900435899266435f * x * (xx - 3.0f * yy);
    }
  }
  float a = 0.5f;
  for (int l = 0; l < nb; ++l) a = fmaf(Y[l], shc[l * 3 + c], a);
  return a;
}

// DEG: SH degree as a compile-time constant, so that the coefficient and gradient arrays stay in registers
template <int DEG>
__global__ __launch_bounds__(128) void project_bwd_kernel(const float* __restrict__ soa, const double* __restrict__ cams,
                                                          ProjConst pc, const float* __restrict__ acc,
                                                          float* __restrict__ g_means, float* __restrict__ g_log_scales,
                                                          float* __restrict__ g_quats, float* __restrict__ g_logits,
                                                          float* __restrict__ g_sh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pc.G) return;
  const int64_t np = pc.n_pad, G = pc.G;
  const int64_t NG = (int64_t)pc.N * G;
  constexpr int deg = DEG;
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const double mu[3] = {soa[kRowMean * np + i], soa[(kRowMean + 1) * np + i], soa[(kRowMean + 2) * np + i]};
  double q4[4] = {soa[kRowQuat * np + i], soa[(kRowQuat + 1) * np + i], soa[(kRowQuat + 2) * np + i],
                  soa[(kRowQuat + 3) * np + i]};
  const double qnorm = sqrt(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
  const double qw = q4[0] / qnorm, qx = q4[1] / qnorm, qy = q4[2] / qnorm, qz = q4[3] / qnorm;
  const double R[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                       2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                       2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
  double s2[3];
  for (int k = 0; k < 3; ++k) {
    const double s = exp((double)soa[(kRowLogScale + k) * np + i]);
    s2[k] = s * s;
  }
  double Sg[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Sg[a * 3 + b] = R[a * 3 + 0] * s2[0] * R[b * 3 + 0] + R[a * 3 + 1] * s2[1] * R[b * 3 + 1] +
                      R[a * 3 + 2] * s2[2] * R[b * 3 + 2];
  const double opac = 1.0 / (1.0 + exp(-(double)soa[kRowLogit * np + i]));
  float shc[48];
#pragma unroll
  for (int k = 0; k < 48; ++k) shc[k] = k < nb * 3 ? soa[(kRowSH + k) * np + i] : 0.0f;

  double gmu[3] = {0, 0, 0}, gSig[9] = {0}, glogit = 0;
  float gsh[48];  // FP32: the SH colour itself is FP32
#pragma unroll
  for (int k = 0; k < 48; ++k) gsh[k] = 0.0f;
  const double ks = 0.72134752044448170368;
  const double f = pc.focal;
  for (int v = 0; v < pc.N; ++v) {
    float ag[kG];
    bool any = false;
    for (int c = 0; c < kG; ++c) {
      ag[c] = acc[(int64_t)c * NG + (int64_t)v * G + i];
      any |= ag[c] != 0.0f;
    }
    if (!any) continue;
    const double* cam = cams + v * kCamDoubles;
    const double* W = cam;
    const double X = W[0] * mu[0] + W[1] * mu[1] + W[2] * mu[2] + cam[9];
    const double Y = W[3] * mu[0] + W[4] * mu[1] + W[5] * mu[2] + cam[10];
    const double Z = W[6] * mu[0] + W[7] * mu[1] + W[8] * mu[2] + cam[11];
    const double iz = 1.0 / Z;
    double T[6];
    for (int k = 0; k < 3; ++k) {
      T[k] = f * iz * (W[k] - X * iz * W[6 + k]);
      T[3 + k] = f * iz * (W[3 + k] - Y * iz * W[6 + k]);
    }
    // Sigma' = T Sigma T^T + h I
    double TS[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        TS[r * 3 + c] = T[r * 3] * Sg[c] + T[r * 3 + 1] * Sg[3 + c] + T[r * 3 + 2] * Sg[6 + c];
    const double ma = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2] + (double)pc.dilation;
    const double mb = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
    const double mc = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5] + (double)pc.dilation;
    const double det = ma * mc - mb * mb;
    // K = Sigma'^-1 = [[ka, kb], [kb, kc]]; record A = ks ka, B = 2 ks kb, C = ks kc
    const double ka = mc / det, kb = -mb / det, kc = ma / det;
    const double gka = ks * ag[2], gkb = 2.0 * ks * ag[3], gkc = ks * ag[4];
    // dL/dM = -K G K with the symmetric G = [[gka, gkb/2], [gkb/2, gkc]]
    const double Gk[4] = {gka, 0.5 * gkb, 0.5 * gkb, gkc};
    const double K[4] = {ka, kb, kb, kc};
    double KG[4], GM[4];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) KG[a * 2 + b] = K[a * 2] * Gk[b] + K[a * 2 + 1] * Gk[2 + b];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) GM[a * 2 + b] = -(KG[a * 2] * K[b] + KG[a * 2 + 1] * K[2 + b]);
    // Sigma' = T Sigma T^T: dL/dSigma = T^T GM T, dL/dT = 2 GM T Sigma (GM, Sigma symmetric)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) s += T[r * 3 + a] * GM[r * 2 + c] * T[c * 3 + b];
        gSig[a * 3 + b] += s;
      }
    double gT[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) gT[r * 3 + c] = 2.0 * (GM[r * 2] * TS[c] + GM[r * 2 + 1] * TS[3 + c]);
    // T0 = (f/Z)(W0 - (X/Z) W2), T1 = (f/Z)(W1 - (Y/Z) W2)
    double gX = 0, gY = 0, gZ = 0;
    const double fz2 = f * iz * iz;
    for (int k = 0; k < 3; ++k) {
      gX += gT[k] * (-fz2 * W[6 + k]);
      gY += gT[3 + k] * (-fz2 * W[6 + k]);
      gZ += gT[k] * (-fz2 * W[k] + 2.0 * f * X * iz * iz * iz * W[6 + k]);
      gZ += gT[3 + k] * (-fz2 * W[3 + k] + 2.0 * f * Y * iz * iz * iz * W[6 + k]);
    }
    // projected mean u = f X / Z + cx, v = f Y / Z + cy
    gX += ag[0] * f * iz;
    gY += ag[1] * f * iz;
    gZ += -(ag[0] * f * X + ag[1] * f * Y) * iz * iz;
    for (int k = 0; k < 3; ++k) gmu[k] += W[k] * gX + W[3 + k] * gY + W[6 + k] * gZ;
    // opacity
    glogit += (double)ag[5] * opac * (1.0 - opac);
    // colour: rgb = max(0, SH(dir) + 0.5), dir = (mu - eye) / |mu - eye|, in FP32 with the forward's operations
    // (the clamp decision must be the forward's)
    const float dx = (float)(mu[0] - cam[12]), dy = (float)(mu[1] - cam[13]), dz = (float)(mu[2] - cam[14]);
    const float dn = sqrtf(dx * dx + dy * dy + dz * dz);
    const float idn = 1.0f / dn;
    const float dir[3] = {dx * idn, dy * idn, dz * idn};
    float Yb[16], dYx[16], dYy[16], dYz[16];
    sh_basis_grad<float>(deg, dir[0], dir[1], dir[2], Yb, dYx, dYy, dYz);
    float gdir[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float gcol = ag[6 + c];
      if (gcol == 0.0f) continue;
      if (!(raw_colour_f32(deg, dir[0], dir[1], dir[2], shc, c) > 0.0f)) continue;
#pragma unroll
      for (int l = 0; l < nb; ++l) {
        gsh[l * 3 + c] += gcol * Yb[l];
        gdir[0] += gcol * shc[l * 3 + c] * dYx[l];
        gdir[1] += gcol * shc[l * 3 + c] * dYy[l];
        gdir[2] += gcol * shc[l * 3 + c] * dYz[l];
      }
    }
    const float gd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
    for (int k = 0; k < 3; ++k) gmu[k] += (double)((gdir[k] - gd * dir[k]) / dn);
  }
  // Sigma = R diag(s^2) R^T: dL/dR = 2 G R S^2 (G symmetrised), dL/ds^2_k = (R^T G R)_kk
  double Gs[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Gs[a * 3 + b] = 0.5 * (gSig[a * 3 + b] + gSig[b * 3 + a]);
  double gR[9];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k)
      gR[a * 3 + k] = 2.0 * (Gs[a * 3 + 0] * R[0 * 3 + k] + Gs[a * 3 + 1] * R[1 * 3 + k] + Gs[a * 3 + 2] * R[2 * 3 + k]) * s2[k];
  for (int k = 0; k < 3; ++k) {
    double s = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s += R[a * 3 + k] * Gs[a * 3 + b] * R[b * 3 + k];
    g_log_scales[i * 3 + k] = (float)(s * 2.0 * s2[k]);
  }
  // R(q) for the normalised quaternion (w, x, y, z)
  const double* Gq = gR;
  double dq[4];
  dq[0] = 2.0 * (-qz * Gq[1] + qy * Gq[2] + qz * Gq[3] - qx * Gq[5] - qy * Gq[6] + qx * Gq[7]);
  dq[1] = 2.0 * (qy * Gq[1] + qz * Gq[2] + qy * Gq[3] - 2.0 * qx * Gq[4] - qw * Gq[5] + qz * Gq[6] + qw * Gq[7] -
                 2.0 * qx * Gq[8]);
  dq[2] = 2.0 * (-2.0 * qy * Gq[0] + qx * Gq[1] + qw * Gq[2] + qx * Gq[3] + qz * Gq[5] - qw * Gq[6] + qz * Gq[7] -
                 2.0 * qy * Gq[8]);
  dq[3] = 2.0 * (-2.0 * qz * Gq[0] - qw * Gq[1] + qx * Gq[2] + qw * Gq[3] - 2.0 * qz * Gq[4] + qy * Gq[5] +
                 qx * Gq[6] + qy * Gq[7]);
  // through the normalisation q_hat = q / |q|
  const double qh[4] = {qw, qx, qy, qz};
  const double dqh = dq[0] * qh[0] + dq[1] * qh[1] + dq[2] * qh[2] + dq[3] * qh[3];
  for (int k = 0; k < 4; ++k) g_quats[i * 4 + k] = (float)((dq[k] - dqh * qh[k]) / qnorm);
  for (int k = 0; k < 3; ++k) g_means[i * 3 + k] = (float)gmu[k];
  g_logits[i] = (float)glogit;
#pragma unroll
  for (int k = 0; k < 48; ++k) g_sh[i * 48 + k] = gsh[k];
}

}  // namespace

hipError_t launch_blend_backward(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                 const uint32_t* sorted, const uint32_t* ray_off, const uint32_t* ray_ent,
                                 int max_rays, const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state,
                                 const float* fwd, const float* gout, float* acc, hipStream_t s) {
  const unsigned nb = (unsigned)((int64_t)bc.N * bc.T);
  if (nb == 0) return hipSuccess;
  // the forward blend's workgroup shape: 256 lanes with up to 4 rays each, else 512 lanes with up to 8
  const bool wide = max_rays > 4 * 256;
  const int lanes = wide ? 512 : 256;
  const int rpt = std::max(1, (max_rays + lanes - 1) / lanes);
#define DL_BWD_CASE(R, L)                                                                                       \
  case R:                                                                                                      \
    hipLaunchKernelGGL((blend_bwd_kernel<R, L>), dim3(nb), dim3(L), 0, s, rec, tile_start, gidx, sorted,      \
                       ray_off, ray_ent, bc, bk, alive, state, fwd, gout, acc);                                \
    break;
  if (!wide) {
    switch (rpt) {
      DL_BWD_CASE(1, 256)
      DL_BWD_CASE(2, 256)
      DL_BWD_CASE(3, 256)
      DL_BWD_CASE(4, 256)
      default:
        return hipErrorInvalidValue;
    }
  } else {
    switch (rpt) {
      DL_BWD_CASE(2, 512)
      DL_BWD_CASE(3, 512)
      DL_BWD_CASE(4, 512)
      DL_BWD_CASE(5, 512)
      DL_BWD_CASE(6, 512)
      DL_BWD_CASE(7, 512)
      DL_BWD_CASE(8, 512)
      default:
        return hipErrorInvalidValue;
    }
  }
#undef DL_BWD_CASE
  return hipGetLastError();
}

hipError_t launch_project_backward(const float* soa, const double* cams, const ProjConst& pc, const float* acc,
                                   float* g_means, float* g_log_scales, float* g_quats, float* g_logits, float* g_sh,
                                   hipStream_t s) {
  const dim3 grid((unsigned)((pc.G + 127) / 128));
  switch (pc.sh_degree) {
    case 0:
      hipLaunchKernelGGL(project_bwd_kernel<0>, grid, dim3(128), 0, s, soa, cams, pc, acc, g_means, g_log_scales,
                         g_quats, g_logits, g_sh);
      break;
    case 1:
      hipLaunchKernelGGL(project_bwd_kernel<1>, grid, dim3(128), 0, s, soa, cams, pc, acc, g_means, g_log_scales,
                         g_quats, g_logits, g_sh);
      break;
    case 2:
      hipLaunchKernelGGL(project_bwd_kernel<2>, grid, dim3(128), 0, s, soa, cams, pc, acc, g_means, g_log_scales,
                         g_quats, g_logits, g_sh);
      break;
    default:
      hipLaunchKernelGGL(project_bwd_kernel<3>, grid, dim3(128), 0, s, soa, cams, pc, acc, g_means, g_log_scales,
                         g_quats, g_logits, g_sh);
      break;
  }
  return hipGetLastError();
}

}  // namespace dl

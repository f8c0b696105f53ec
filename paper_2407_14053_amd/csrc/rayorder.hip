// Ray-order 3DGS (Sec. "Ray-Order 3DGS", Alg. 3, Eq. (22)-(23)) on gfx950: one ray per lane.
//
// Per ray (origin o = the view's camera centre, unit direction d through the pixel centre) the result is the
// front-to-back blend of the c_h hits nearest by peak distance t_j (Eq. (22)), each with
// alpha_j = o_j G(o + t_j d) (Eq. (23)) and the SH colour in direction d.  The paper collects those hits in a
// per-ray max-heap of capacity c_h filled during one traversal.  Here they are gathered in rounds instead: a
// round traverses the BVH for the K smallest keys (t_j, j) above the last key blended, kept sorted in
// registers, and blends them; the ray ends when c_h hits are blended, the transmittance stops the blend, or a
// round finds fewer than K.  The set and order blended are the heap's (keys are totally ordered), but no
// per-ray memory grows with c_h, and rays that the transmittance stops early never gather the rest.
//
// Traversal: a per-lane stack in LDS ([entry][lane], so lanes at the same depth hit distinct banks) of node
// and leaf references; a node's children that the ray's current interval [t_lo, t_hi] meets are pushed far to
// near after a sorting network on their entry distance.  t_lo is the current round's lowest key's t (and
// z_near), t_hi the K-th key's t once K keys are held: a hit's peak lies in its leaf box, so boxes outside
// the interval cannot hold a key the round still needs.
#include "dl_internal.h"

namespace dl {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

__device__ inline void cswap(float& ta, uint32_t& ra, float& tb, uint32_t& rb) {
  const bool sw = tb < ta;
  const float t = sw ? tb : ta;
  tb = sw ? ta : tb;
  ta = t;
  const uint32_t r = sw ? rb : ra;
  rb = sw ? ra : rb;
  ra = r;
}

// slab test of a box against the ray's interval; returns the entry distance (or +inf when missed)
__device__ inline float slab(float lx, float ly, float lz, float hx, float hy, float hz, float ox, float oy, float oz,
                             float ix, float iy, float iz, float tlo, float thi) {
  const float ax = (lx - ox) * ix, bx = (hx - ox) * ix;
  const float ay = (ly - oy) * iy, by = (hy - oy) * iy;
  const float az = (lz - oz) * iz, bz = (hz - oz) * iz;
  const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), tlo));
  // far distance rounded up by 3 ulp: the FP32 slab must not cut a box the exact one meets
  const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz)) * 1.0000004f;
  return tn <= fminf(tf, thi) ? tn : INFINITY;
}

// peak distance (Eq. (22)) and the quadratic form there, from the record [mu, o], [a00 a01 a02 a11],
// [a12 a22 q_lim, index]
__device__ inline void peak(const float4& r0, const float4& r1, const float4& r2, float ox, float oy, float oz,
                            float dx, float dy, float dz, float& t, float& q) {
  const float px = ox - r0.x, py = oy - r0.y, pz = oz - r0.z;  // o - mu
  const float adx = r1.x * dx + r1.y * dy + r1.z * dz;
  const float ady = r1.y * dx + r1.w * dy + r2.x * dz;
  const float adz = r1.z * dx + r2.x * dy + r2.y * dz;
  const float den = dx * adx + dy * ady + dz * adz;
  const float num = -(px * adx + py * ady + pz * adz);
  t = num / den;
  const float rx = px + t * dx, ry = py + t * dy, rz = pz + t * dz;  // o + t d - mu
  const float arx = r1.x * rx + r1.y * ry + r1.z * rz;
  const float ary = r1.y * rx + r1.w * ry + r2.x * rz;
  const float arz = r1.z * rx + r2.x * ry + r2.y * rz;
  q = rx * arx + ry * ary + rz * arz;
}

template <bool STATS, int kRoundKeys>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void rayorder_kernel(const float* __restrict__ nodes, const float4* __restrict__ rec,
                                                      const float4* __restrict__ shl, const double* __restrict__ cams,
                                                      const uint32_t* __restrict__ ray_off,
                                                      const uint32_t* __restrict__ ray_ent, RoConst rc,
                                                      float* __restrict__ out) {
  extern __shared__ uint32_t stk[];  // [stack_cap][64]
  const int lane = threadIdx.x;
  // lists of neighbouring tiles on one XCD (workgroups go round-robin over the 8 XCDs): they share Gaussians
  const int64_t nb = (int64_t)rc.N * rc.T, bid = blockIdx.x;
  const int64_t q8 = nb / 8, rem = nb % 8, xcd = bid % 8, kx = bid / 8;
  const int64_t list = xcd < rem ? xcd * (q8 + 1) + kx : rem * (q8 + 1) + (xcd - rem) * q8 + kx;
  const int v = (int)(list / rc.T), tile = (int)(list - (int64_t)v * rc.T);
  const int ty = tile / rc.ntx, tx = tile - ty * rc.ntx;
  const uint32_t r0 = ray_off[list], r1 = ray_off[list + 1];
  const double* cam = cams + (int64_t)v * kCamDoubles;
  unsigned long long n_tests = 0, n_blend = 0, n_rays = 0;

  for (uint32_t base = r0; base < r1; base += 64) {
    const uint32_t ri = base + lane;
    if (ri < r1) {
      const uint32_t e = ray_ent[ri];
      const int xr = ty * rc.th + (int)((e >> 12) & 0xfffu), yc = tx * rc.tw + (int)(e & 0xfffu);
      const uint32_t mask = (e >> 24) & 7u;
      // ray in world space (FP64 once per ray, then FP32)
      const double u = ((double)yc + 0.5 - rc.cx) / rc.focal, w = ((double)xr + 0.5 - rc.cy) / rc.focal;
      const double wx = cam[0] * u + cam[3] * w + cam[6], wy = cam[1] * u + cam[4] * w + cam[7],
                   wz = cam[2] * u + cam[5] * w + cam[8];
      const double inv = 1.0 / sqrt(wx * wx + wy * wy + wz * wz);
      const float dx = (float)(wx * inv), dy = (float)(wy * inv), dz = (float)(wz * inv);
      const float ox = (float)cam[12], oy = (float)cam[13], oz = (float)cam[14];
      const float ix = 1.0f / (fabsf(dx) > 1e-20f ? dx : copysignf(1e-20f, dx));
      const float iy = 1.0f / (fabsf(dy) > 1e-20f ? dy : copysignf(1e-20f, dy));
      const float iz = 1.0f / (fabsf(dz) > 1e-20f ? dz : copysignf(1e-20f, dz));

      float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
      int used = 0;
      bool done = false;
      uint64_t lo_key = (uint64_t)__float_as_uint(rc.z_near) << 32;
      while (!done) {
        uint64_t kb[kRoundKeys];
#pragma unroll
        for (int i = 0; i < kRoundKeys; ++i) kb[i] = ~0ull;
        const float tlo = __uint_as_float((uint32_t)(lo_key >> 32));
        float thi = INFINITY;
        int sp = 1;
        stk[lane] = 0u;  // root
        while (sp > 0) {
          --sp;
          const uint32_t ref = stk[sp * 64 + lane];
          if (ref & kBvhLeafBit) {
            const uint32_t first = ref & 0x0fffffffu, cnt = ((ref >> 28) & 7u) + 1u;
            for (uint32_t i = 0; i < cnt; ++i) {
              const uint32_t j = first + i;
              const float4 a = rec[3 * (size_t)j], b = rec[3 * (size_t)j + 1], c = rec[3 * (size_t)j + 2];
              float t, q;
              peak(a, b, c, ox, oy, oz, dx, dy, dz, t, q);
              if (STATS) ++n_tests;
              if (q <= c.z && t >= rc.z_near) {
                uint64_t key = ((uint64_t)__float_as_uint(t) << 32) | j;
                if (key >= lo_key && key < kb[kRoundKeys - 1]) {
#pragma unroll
                  for (int k = 0; k < kRoundKeys; ++k) {
                    const uint64_t o = kb[k];
                    const bool lt = key < o;
                    kb[k] = lt ? key : o;
                    key = lt ? o : key;
                  }
                  if (kb[kRoundKeys - 1] != ~0ull) thi = __uint_as_float((uint32_t)(kb[kRoundKeys - 1] >> 32));
                }
              }
            }
            continue;
          }
          const float4* nd = reinterpret_cast<const float4*>(nodes + (size_t)ref * kBvhNodeFloats);
          const float4 own0 = nd[14], own1 = nd[15];
          if (slab(own0.x, own0.y, own0.z, own0.w, own1.x, own1.y, ox, oy, oz, ix, iy, iz, tlo, thi) == INFINITY)
            continue;
          // the child boxes in two halves of four (fewer registers live at once)
          float tn[8];
          uint32_t cr[8];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float4 lx = nd[0 + h], ly = nd[2 + h], lz = nd[4 + h];
            const float4 hx = nd[6 + h], hy = nd[8 + h], hz = nd[10 + h], rf = nd[12 + h];
            const float lxa[4] = {lx.x, lx.y, lx.z, lx.w}, lya[4] = {ly.x, ly.y, ly.z, ly.w};
            const float lza[4] = {lz.x, lz.y, lz.z, lz.w}, hxa[4] = {hx.x, hx.y, hx.z, hx.w};
            const float hya[4] = {hy.x, hy.y, hy.z, hy.w}, hza[4] = {hz.x, hz.y, hz.z, hz.w};
            const uint32_t ra[4] = {__float_as_uint(rf.x), __float_as_uint(rf.y), __float_as_uint(rf.z),
                                    __float_as_uint(rf.w)};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const float tt = slab(lxa[c], lya[c], lza[c], hxa[c], hya[c], hza[c], ox, oy, oz, ix, iy, iz, tlo, thi);
              tn[4 * h + c] = ra[c] == kBvhEmpty ? INFINITY : tt;
              cr[4 * h + c] = ra[c];
            }
            if (h == 0) __builtin_amdgcn_sched_barrier(0);  // keep the second half's loads after the first's use
          }
          // sort the 8 children by entry distance (19 compare-exchanges)
          cswap(tn[0], cr[0], tn[1], cr[1]); cswap(tn[2], cr[2], tn[3], cr[3]);
          cswap(tn[4], cr[4], tn[5], cr[5]); cswap(tn[6], cr[6], tn[7], cr[7]);
          cswap(tn[0], cr[0], tn[2], cr[2]); cswap(tn[1], cr[1], tn[3], cr[3]);
          cswap(tn[4], cr[4], tn[6], cr[6]); cswap(tn[5], cr[5], tn[7], cr[7]);
          cswap(tn[1], cr[1], tn[2], cr[2]); cswap(tn[5], cr[5], tn[6], cr[6]);
          cswap(tn[0], cr[0], tn[4], cr[4]); cswap(tn[3], cr[3], tn[7], cr[7]);
          cswap(tn[1], cr[1], tn[5], cr[5]); cswap(tn[2], cr[2], tn[6], cr[6]);
          cswap(tn[1], cr[1], tn[4], cr[4]); cswap(tn[3], cr[3], tn[6], cr[6]);
          cswap(tn[2], cr[2], tn[4], cr[4]); cswap(tn[3], cr[3], tn[5], cr[5]);
          cswap(tn[3], cr[3], tn[4], cr[4]);
          // push far to near (the nearest is popped first); the stack bound of the tree keeps sp < stack_cap
#pragma unroll
          for (int c = 7; c >= 0; --c)
            if (tn[c] != INFINITY && sp < rc.stack_cap) {
              stk[sp * 64 + lane] = cr[c];
              ++sp;
            }
        }
        // blend this round's keys in order (taken from the front of the buffer, which shifts down: no dynamic
        // register indexing)
        const bool full = kb[kRoundKeys - 1] != ~0ull;
#pragma unroll 1
        for (int i = 0; i < kRoundKeys && !done; ++i) {
          const uint64_t key = kb[0];
#pragma unroll
          for (int k = 0; k < kRoundKeys - 1; ++k) kb[k] = kb[k + 1];
          kb[kRoundKeys - 1] = ~0ull;
          if (key == ~0ull) {
            done = true;
            break;
          }
          const uint32_t j = (uint32_t)key;
          const float t = __uint_as_float((uint32_t)(key >> 32));
          const float4 a = rec[3 * (size_t)j], b = rec[3 * (size_t)j + 1], c = rec[3 * (size_t)j + 2];
          const float px = ox - a.x + t * dx, py = oy - a.y + t * dy, pz = oz - a.z + t * dz;
          const float arx = b.x * px + b.y * py + b.z * pz;
          const float ary = b.y * px + b.w * py + c.x * pz;
          const float arz = b.z * px + c.x * py + c.y * pz;
          const float q = px * arx + py * ary + pz * arz;
          const float alpha = fminf(rc.alpha_max, a.w * __builtin_amdgcn_exp2f(-0.5f * kLog2e * q));
          const float nt = T * (1.0f - alpha);
          if (nt < rc.t_min) {
            done = true;
            break;
          }
          float Y[16];
#pragma unroll
          for (int k = 0; k < 16; ++k) Y[k] = 0.0f;
          sh_basis(rc.sh_degree, dx, dy, dz, Y);
          const float wgt = T * alpha;
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            if (!(mask & (1u << ch))) continue;
            const float4* s4 = shl + ((size_t)j * 3 + ch) * 4;
            const float4 s0 = s4[0], s1 = s4[1], s2 = s4[2], s3 = s4[3];
            float col = Y[0] * s0.x + Y[1] * s0.y + Y[2] * s0.z + Y[3] * s0.w + Y[4] * s1.x + Y[5] * s1.y +
                        Y[6] * s1.z + Y[7] * s1.w + Y[8] * s2.x + Y[9] * s2.y + Y[10] * s2.z + Y[11] * s2.w +
                        Y[12] * s3.x + Y[13] * s3.y + Y[14] * s3.z + Y[15] * s3.w + 0.5f;
            col = fmaxf(col, 0.0f);
            if (ch == 0) C0 = fmaf(wgt, col, C0);
            if (ch == 1) C1 = fmaf(wgt, col, C1);
            if (ch == 2) C2 = fmaf(wgt, col, C2);
          }
          T = nt;
          ++used;
          if (STATS) ++n_blend;
          lo_key = key + 1;
          if (used >= rc.heap_cap) done = true;
        }
        if (!full) done = true;  // the round found every remaining hit
      }
      if (STATS) ++n_rays;
      const float c3[3] = {fmaf(T, rc.bg[0], C0), fmaf(T, rc.bg[1], C1), fmaf(T, rc.bg[2], C2)};
      if (rc.tgt) {
        const uint32_t slot = (e >> 27) & 3u;
        const int32_t* tg = rc.tgt + ((int64_t)3 * ((int64_t)xr * rc.W + yc) + slot) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (mask & (1u << k)) out[tg[k]] = c3[k];
      } else {
        float* dst = out + ((int64_t)xr * rc.W + yc) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (mask & (1u << k)) dst[k] = c3[k];
      }
    }
  }
  if (STATS) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      n_tests += __shfl_down(n_tests, off);
      n_blend += __shfl_down(n_blend, off);
      n_rays += __shfl_down(n_rays, off);
    }
    if (lane == 0) {
      unsigned long long* slot = rc.stats + 3 * (blockIdx.x % kStatSlots);
      atomicAdd(&slot[0], n_tests);
      atomicAdd(&slot[1], n_blend);
      atomicAdd(&slot[2], n_rays);
    }
  }
}

}  // namespace

hipError_t launch_rayorder(const float* nodes, const float4* rec, const float4* sh, const double* cams,
                           const uint32_t* ray_off, const uint32_t* ray_ent, const RoConst& rc, float* out,
                           hipStream_t s) {
  const int64_t nb = (int64_t)rc.N * rc.T;
  if (nb == 0) return hipSuccess;
  if (rc.stack_cap < 1 || rc.stack_cap > kBvhStackMax || nb >= (1ll << 31)) return hipErrorInvalidValue;
  const size_t lds = (size_t)rc.stack_cap * 64 * 4;
#define DL_RO_LAUNCH(K)                                                                                          \
  if (rc.stats)                                                                                                  \
    hipLaunchKernelGGL((rayorder_kernel<true, K>), dim3((unsigned)nb), dim3(64), lds, s, nodes, rec, sh, cams,  \
                       ray_off, ray_ent, rc, out);                                                               \
  else                                                                                                           \
    hipLaunchKernelGGL((rayorder_kernel<false, K>), dim3((unsigned)nb), dim3(64), lds, s, nodes, rec, sh, cams, \
                       ray_off, ray_ent, rc, out);
  if (rc.heap_cap <= 16) {
    DL_RO_LAUNCH(16)
  } else {
    DL_RO_LAUNCH(32)
  }
#undef DL_RO_LAUNCH
  return hipGetLastError();
}

}  // namespace dl

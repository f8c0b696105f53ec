// Issue-rate probe of the vector ALU (gfx950): the ceilings the blend's roofline fraction is taken against.
//
// Fourteen kernels run a fixed number of dependent-chain steps per lane, with 8 independent chains per lane and a
// grid of 8 wavefronts per SIMD on every compute unit, so that latency is hidden and only the issue rate
// remains:
//   0: v_fma_f32 chains               (one full-rate FP32 operation per step)
//   1: v_exp_f32 chains               (the transcendental the blend issues once per pair)
//   2: 4 v_fma_f32 then 1 v_exp_f32   (does the transcendental overlap the FMAs or take issue cycles of its own)
//   3: the blend's per-pair instruction sequence for a one-channel ray (two subtractions, the quadratic form,
//      exp2, the transmittance update with its two compares and two selects, one colour FMA: 15 VALU)
//   4: the same for a three-channel ray with the clamp at alpha_max (18 VALU)
//   5-12: single instruction classes (which instructions the SIMD can issue two of at once): v_add_f32,
//        v_fmac_f32 (accumulator as destination), v_mul_f32 with a negated operand, v_fma_f32 with three VGPR
//        operands, v_cndmask_b32 with an SGPR-pair mask, v_cmp_gt_f32 into an SGPR pair, v_fmac_f32 with three
//        distinct registers, v_fma_f32 with an SGPR operand
//   13: one v_exp_f32 beside four independent v_fma_f32 (does the transcendental hold the others back)
// Modes 9-12 pin their instruction with inline assembly (register operands only, no memory access).
// Lane 0 of workgroup 0 also reads the shader clock counter (s_memtime) and the 100 MHz constant clock
// (s_memrealtime) at its start and end, which gives the engine clock the kernels actually ran at.
// Packed FP32 instructions are disabled at compile time, so these are the non-packed rates.
#include "dl_internal.h"

namespace dl {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;
constexpr int kUnroll = 8;

template <int MODE>
__global__ __launch_bounds__(kProbeThreads) void issue_rate_kernel(float* __restrict__ sink, uint64_t* __restrict__ clk,
                                                                  int iters, float b, float c) {
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = (float)(threadIdx.x & 63) * 1e-3f + (float)j * 0.125f;
  uint64_t t0 = 0, w0 = 0;
  const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
  if (timer) {
    t0 = clock64();
    w0 = wall_clock64();
  }
  // the 16 floats the blend mode reads as "the record" and "the ray"
  const float rx = b * 3.0f, ry = c * 5.0f, cA = b * 0.01f, cB = c * 0.002f, cC = b * 0.015f, lo = -c;
  const float lim = -9.0f, amax = 0.99f, tmin = 1e-4f, cr = b * 0.5f, cg = c * 0.25f, cb = b * 0.125f;
  uint64_t acc = 0;
  const uint64_t smask = (uint64_t)(uint32_t)iters * 0x9e3779b97f4a7c15ull;  // uniform, not a constant
  float C0[kChains], C1[kChains], C2[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    // modes 5-8 read these as VGPR operands (lane-dependent, so not folded into literals): values near 1e-7,
    // 0.999 and 1e-3 keep every chain finite
    const float tiny = (float)(threadIdx.x & 7) * 1e-10f;
    C0[j] = MODE >= 5 ? (MODE == 7 ? -0.999f - tiny : 1e-7f + tiny) : 0.0f;
    C1[j] = MODE >= 5 ? (MODE == 6 ? 1e-7f + tiny : 1e-3f + tiny) : 0.0f;
    C2[j] = MODE == 13 ? 1e-3f + tiny : 0.0f;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int j = 0; j < kChains; ++j) {
        if (MODE == 0) {
          a[j] = fmaf(a[j], b, c);
        } else if (MODE == 1) {
          a[j] = __builtin_amdgcn_exp2f(-a[j]);
        } else if (MODE == 5) {
          a[j] = a[j] + C0[j];  // v_add_f32 (two VGPR operands)
        } else if (MODE == 6) {
          a[j] = fmaf(C0[j], C1[j], a[j]);  // v_fmac_f32: the accumulator is the destination
        } else if (MODE == 7) {
          a[j] = -C0[j] * a[j];  // v_mul_f32 with a negated operand
        } else if (MODE == 8) {
          a[j] = fmaf(-a[j], C0[j], C1[j]);  // v_fma_f32, three VGPR operands, one negated
        } else if (MODE == 9) {
          // v_cndmask_b32 with a mask held in an SGPR pair
          asm("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a[j]) : "v"(C0[j]), "s"(smask));
        } else if (MODE == 10) {
          // v_cmp_gt_f32 writing an SGPR pair, its operands in VGPRs (the results are folded into one mask)
          uint64_t m;
          asm volatile("v_cmp_gt_f32_e64 %0, %1, %2" : "=s"(m) : "v"(a[j]), "v"(C0[j]));
          acc ^= m;
          a[j] = a[j] + C1[j];
        } else if (MODE == 11) {
          // v_fmac_f32 with three distinct registers
          asm("v_fmac_f32_e32 %0, %1, %2" : "+v"(a[j]) : "v"(C0[j]), "v"(C1[j]));
        } else if (MODE == 12) {
          // v_fma_f32 with one SGPR operand
          asm("v_fma_f32 %0, %1, %2, %0" : "+v"(a[j]) : "s"(b), "v"(C0[j]));
        } else if (MODE == 13) {
          // one v_exp_f32 and four independent three-VGPR v_fma_f32
          a[j] = __builtin_amdgcn_exp2f(-a[j]);
          C1[j] = fmaf(-C1[j], C0[j], C2[j]);
          C2[j] = fmaf(-C2[j], C0[j], C1[j]);
          C1[j] = fmaf(-C1[j], C0[j], C2[j]);
          C2[j] = fmaf(-C2[j], C0[j], C1[j]);
        } else if (MODE == 2) {
          float x = fmaf(a[j], b, c);
          x = fmaf(x, b, c);
          x = fmaf(x, b, c);
          x = fmaf(x, b, c);
          a[j] = __builtin_amdgcn_exp2f(-x);
        } else {
          // the chain value serves as the ray position and as T, so that no step can be hoisted out of the
          // loop and the instruction count per step is the blend's
          const float dx = a[j] - rx, dy = a[j] - ry;
          const float E = fmaf(-fmaf(cB, dy, cA * dx), dx, fmaf(-(cC * dy), dy, lo));
          const float ga = __builtin_amdgcn_exp2f(E);
          const float alpha = MODE == 4 ? fminf(amax, ga) : ga;
          const float T = a[j];
          const float tn = fmaf(-alpha, T, T);
          const bool ok = E >= lim;
          const bool stop = ok && (tn < tmin);
          const bool take = ok != stop;
          const float Tt = take ? tn : T;
          const float w = T - Tt;
          C0[j] = fmaf(w, cr, C0[j]);
          if (MODE == 4) {
            C1[j] = fmaf(w, cg, C1[j]);
            C2[j] = fmaf(w, cb, C2[j]);
          }
          a[j] = stop ? -fabsf(T) : Tt;
        }
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += a[j] + C0[j] + C1[j] + C2[j];
  // never true for these inputs: keeps the chains live without a store per lane
  if (s == 1234567.0f || acc == 0x123456789ull) sink[blockIdx.x * kProbeThreads + threadIdx.x] = s;
  if (timer) {
    clk[0] = clock64() - t0;
    clk[1] = wall_clock64() - w0;
  }
}

template <int M>
void launch_one(int blocks, hipStream_t s, float* sink, uint64_t* clk, int iters) {
  hipLaunchKernelGGL(issue_rate_kernel<M>, dim3(blocks), dim3(kProbeThreads), 0, s, sink, clk, iters, 0.999f, 0.001f);
}

void launch_mode(int mode, int blocks, hipStream_t s, float* sink, uint64_t* clk, int iters) {
  switch (mode) {
    case 0: launch_one<0>(blocks, s, sink, clk, iters); break;
    case 1: launch_one<1>(blocks, s, sink, clk, iters); break;
    case 2: launch_one<2>(blocks, s, sink, clk, iters); break;
    case 3: launch_one<3>(blocks, s, sink, clk, iters); break;
    case 4: launch_one<4>(blocks, s, sink, clk, iters); break;
    case 5: launch_one<5>(blocks, s, sink, clk, iters); break;
    case 6: launch_one<6>(blocks, s, sink, clk, iters); break;
    case 7: launch_one<7>(blocks, s, sink, clk, iters); break;
    case 8: launch_one<8>(blocks, s, sink, clk, iters); break;
    case 9: launch_one<9>(blocks, s, sink, clk, iters); break;
    case 10: launch_one<10>(blocks, s, sink, clk, iters); break;
    case 11: launch_one<11>(blocks, s, sink, clk, iters); break;
    case 12: launch_one<12>(blocks, s, sink, clk, iters); break;
    default: launch_one<13>(blocks, s, sink, clk, iters); break;
  }
}

constexpr int kModes = 14;

}  // namespace

int probe_issue_rates(double* out, int n_out, std::string* why) {
  auto hip_fail = [&](hipError_t e, const char* what) {
    *why = std::string(what) + ": " + hipGetErrorString(e);
    return DL_EHIP;
  };
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  const int blocks = cus * 4 * 8 / (kProbeThreads / 64);  // 8 wavefronts per SIMD, 4 SIMDs per CU
  const int iters = 512;
  float* sink = nullptr;
  uint64_t* clk = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = DL_OK;
  double res[kModes] = {};
  double clock_hz = 0.0;
  if ((e = hipMalloc(&sink, (size_t)blocks * kProbeThreads * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&clk, 2 * sizeof(uint64_t))) != hipSuccess || (e = hipStreamCreate(&s)) != hipSuccess ||
      (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    rc = hip_fail(e, "probe set-up");
  }
  for (int mode = 0; mode < kModes && rc == DL_OK; ++mode) {
    float best = 1e30f;
    for (int rep = 0; rep < 4 && rc == DL_OK; ++rep) {
      (void)hipEventRecord(e0, s);
      launch_mode(mode, blocks, s, sink, clk, iters);
      (void)hipEventRecord(e1, s);
      if ((e = hipGetLastError()) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
        rc = hip_fail(e, "probe kernel");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best = std::min(best, ms);  // the first launch warms the clocks
      if (mode == 0 && rep == 3) {
        uint64_t h[2] = {0, 0};
        if ((e = hipMemcpy(h, clk, sizeof(h), hipMemcpyDeviceToHost)) != hipSuccess) {
          rc = hip_fail(e, "probe clock readback");
          break;
        }
        if (h[1] > 0) clock_hz = (double)h[0] / ((double)h[1] / 1e8);
      }
    }
    const double steps = (double)blocks * kProbeThreads * iters * kUnroll * kChains;  // chain steps, all lanes
    res[mode] = steps / (best * 1e-3);
  }
  if (sink) (void)hipFree(sink);
  if (clk) (void)hipFree(clk);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (rc != DL_OK) return rc;
  // out: [0] FMA lane-ops/s, [1] exp lane-ops/s, [2] (4 FMA + 1 exp) steps/s, [3] one-channel blend pairs/s,
  //      [4] three-channel blend pairs/s (lanes), [5] engine clock Hz (measured), [6] compute units,
  //      [7] v_add_f32, [8] v_fmac_f32, [9] v_mul_f32 (negated operand), [10] v_fma_f32 (three VGPRs) lane-ops/s,
  //      [11] v_cndmask_b32 (SGPR-pair mask), [12] v_cmp_gt_f32 to an SGPR pair (+ one v_add_f32) steps/s,
  //      [13] v_fmac_f32 (three distinct registers), [14] v_fma_f32 (one SGPR operand) lane-ops/s,
  //      [15] (1 v_exp_f32 + 4 independent v_fma_f32) steps/s
  const double vals[16] = {res[0], res[1], res[2], res[3], res[4], clock_hz, (double)cus, res[5],
                           res[6], res[7], res[8], res[9], res[10], res[11], res[12], res[13]};
  for (int i = 0; i < n_out && i < 16; ++i) out[i] = vals[i];
  return DL_OK;
}

}  // namespace dl

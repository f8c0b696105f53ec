// Test harness (host only): builds the ray-order BVH of a synthetic scene with the library's host builder and
// checks what a traversal relies on.  Prints one line "ok <prims> <nodes> <leaves> <depth> <stack>" or the first
// violation, and exits non-zero on a violation.
//   - every child reference is a node index in range, a leaf range inside the Gaussians, or empty;
//   - every Gaussian of the BVH sits in exactly one leaf;
//   - a child box lies inside its node's own box, an internal child's own box inside the parent's child box;
//   - each Gaussian's ellipsoid q <= q_lim (sampled on its surface) lies inside its leaf box;
//   - a depth-first walk that pushes all children never holds more entries than the reported stack bound.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../paper_2407_14053_amd/csrc/dl_internal.h"

using namespace dl;

static int fail(const char* m) {
  std::printf("violation: %s\n", m);
  return 1;
}

int main(int argc, char** argv) {
  const long n = argc > 1 ? std::atol(argv[1]) : 2000;
  const int kind = argc > 2 ? std::atoi(argv[2]) : 0;  // 0 uniform, 1 clustered, 2 coincident means
  const long np = (n + 63) / 64 * 64;
  std::vector<float> soa((size_t)kSceneRows * np, 0.0f);
  std::mt19937 rng(7 + kind);
  std::uniform_real_distribution<float> U(-2.0f, 2.0f), S(-4.0f, -2.0f);
  std::normal_distribution<float> N(0.0f, 1.0f);
  std::vector<float> centres(3 * 16);
  for (float& c : centres) c = U(rng);
  for (long i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) {
      float m = U(rng);
      if (kind == 1) m = centres[3 * (i % 16) + k] + 0.02f * N(rng);
      if (kind == 2) m = 0.5f;
      soa[(size_t)(kRowMean + k) * np + i] = m;
      soa[(size_t)(kRowLogScale + k) * np + i] = S(rng);
    }
    for (int k = 0; k < 4; ++k) soa[(size_t)(kRowQuat + k) * np + i] = N(rng);
    soa[(size_t)kRowLogit * np + i] = N(rng) * 2.0f;
  }
  const float q_cut = 9.0f, a_min = 1.0f / 255.0f;
  BvhHost b;
  std::string why;
  if (bvh_build_host(soa.data(), n, np, q_cut, a_min, &b, &why)) return fail(why.c_str());
  // expected membership: opacity >= alpha_min
  long expect = 0;
  for (long i = 0; i < n; ++i) {
    const double o = 1.0 / (1.0 + std::exp(-(double)soa[(size_t)kRowLogit * np + i]));
    expect += (std::fmin((double)q_cut, 2.0 * std::log(o / a_min)) > 0) ? 1 : 0;
  }
  if (b.n_prims != expect) return fail("Gaussians in the BVH != Gaussians with opacity >= alpha_min");
  std::vector<int> seen(b.n_prims, 0);
  std::vector<uint32_t> st{0};
  size_t most = 1;
  auto inside = [](float lo, float hi, float a, float z) { return a >= lo && z <= hi; };
  std::mt19937 r2(3);
  while (!st.empty()) {
    const uint32_t ref = st.back();
    st.pop_back();
    if (ref & kBvhLeafBit) continue;
    if (ref >= (uint32_t)b.n_nodes) return fail("node reference out of range");
    const float* nd = &b.nodes[(size_t)ref * kBvhNodeFloats];
    for (int c = 0; c < 8; ++c) {
      uint32_t cr;
      std::memcpy(&cr, &nd[48 + c], 4);
      if (cr == kBvhEmpty) continue;
      const float lo[3] = {nd[c], nd[8 + c], nd[16 + c]}, hi[3] = {nd[24 + c], nd[32 + c], nd[40 + c]};
      for (int k = 0; k < 3; ++k)
        if (!inside(nd[56 + k], nd[59 + k], lo[k], hi[k])) return fail("child box outside its node's box");
      if (cr & kBvhLeafBit) {
        const uint32_t first = cr & 0x0fffffffu, cnt = ((cr >> 28) & 7u) + 1u;
        if (cnt > (uint32_t)kBvhLeafMax || first + cnt > (uint32_t)b.n_prims) return fail("leaf range out of range");
        for (uint32_t j = first; j < first + cnt; ++j) {
          seen[j]++;
          // sample the ellipsoid q = q_lim: x = mu + L z with L L^T = Sigma, |z| = sqrt(q_lim)
          const float* g = &b.rec[(size_t)j * 12];
          const double A[3][3] = {{g[4], g[5], g[6]}, {g[5], g[7], g[8]}, {g[6], g[8], g[9]}};
          // Sigma = A^-1 by cofactors
          const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                             A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                             A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
          double Sg[3][3];
          for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) {
              const int a1 = (bb + 1) % 3, a2 = (bb + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
              Sg[a][bb] = (A[a1][b1] * A[a2][b2] - A[a1][b2] * A[a2][b1]) / det;
            }
          // Cholesky of Sigma
          double L[3][3] = {{0}};
          for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb <= a; ++bb) {
              double s = Sg[a][bb];
              for (int k = 0; k < bb; ++k) s -= L[a][k] * L[bb][k];
              L[a][bb] = a == bb ? std::sqrt(std::fmax(s, 0.0)) : s / L[bb][bb];
            }
          std::normal_distribution<double> Z(0.0, 1.0);
          for (int t = 0; t < 64; ++t) {
            double z[3] = {Z(r2), Z(r2), Z(r2)};
            const double nz = std::sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
            for (double& e : z) e *= std::sqrt((double)g[10]) / nz;
            for (int a = 0; a < 3; ++a) {
              const double x = g[a] + L[a][0] * z[0] + L[a][1] * z[1] + L[a][2] * z[2];
              if (x < lo[a] || x > hi[a]) return fail("Gaussian's q_lim ellipsoid leaves its leaf box");
            }
          }
        }
      } else {
        if (cr >= (uint32_t)b.n_nodes) return fail("node reference out of range");
        const float* cn = &b.nodes[(size_t)cr * kBvhNodeFloats];
        for (int k = 0; k < 3; ++k)
          if (!inside(lo[k], hi[k], cn[56 + k], cn[59 + k])) return fail("child node's box outside its slot's box");
      }
      st.push_back(cr);
    }
    most = std::max(most, st.size());
  }
  for (long j = 0; j < b.n_prims; ++j)
    if (seen[j] != 1) return fail("a Gaussian is not in exactly one leaf");
  if ((int)most > b.stack_bound) return fail("walk exceeded the stack bound");
  std::printf("ok %ld %ld %ld %d %d\n", (long)b.n_prims, (long)b.n_nodes, (long)b.n_leaves, b.depth, b.stack_bound);
  return 0;
}

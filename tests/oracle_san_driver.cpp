// Runs the oracle's C++ entry points (per-ray compositing with its admissible outcomes, the adjoint, the
// projection, and the compiled Alg. 2 walk) on a small deterministic scene, so that a build with the address
// and undefined-behaviour sanitizers checks their memory accesses and arithmetic.  Test infrastructure only.
#include "../oracle/dlo.cpp"
#include "../oracle/srwalk.cpp"

#include <cstdio>
#include <vector>

namespace {
struct Lcg {
  uint64_t s;
  double next() {  // uniform in [0, 1)
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0);
  }
};
}  // namespace

int main() {
  const int64_t G = 300;
  const int N = 3, W = 24, H = 16;
  Lcg rng{12345};
  std::vector<float> means(G * 3), ls(G * 3), quats(G * 4), logits(G), sh(G * 48);
  for (auto& m : means) m = (float)(2.0 * rng.next() - 1.0);
  for (auto& l : ls) l = (float)(-3.0 + 1.5 * rng.next());
  for (auto& q : quats) q = (float)(2.0 * rng.next() - 1.0);
  for (auto& o : logits) o = (float)(4.0 * rng.next() - 2.0);
  for (auto& c : sh) c = (float)(0.2 * rng.next() - 0.1);
  // coincident pairs and near-equal depths exercise the near-tie groups
  for (int64_t i = 0; i < 20; ++i)
    for (int k = 0; k < 3; ++k) means[(i + 20) * 3 + k] = means[i * 3 + k] + (k == 2 ? 1e-8f * (float)i : 0.0f);
  // cameras on the z axis at distance 3, looking at the origin (OpenCV axes: y down, z forward)
  std::vector<double> R(N * 9, 0.0), t(N * 3, 0.0), eye(N * 3, 0.0);
  for (int v = 0; v < N; ++v) {
    R[v * 9 + 0] = 1.0;
    R[v * 9 + 4] = -1.0;
    R[v * 9 + 8] = -1.0;
    eye[v * 3 + 0] = 0.1 * (v - 1);
    eye[v * 3 + 2] = 3.0;
    for (int r = 0; r < 3; ++r) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += R[v * 9 + r * 3 + c] * eye[v * 3 + c];
      t[v * 3 + r] = -s;
    }
  }
  dlo_opts o{};
  o.focal = 20.0;
  o.cx = W / 2.0;
  o.cy = H / 2.0;
  o.z_near = 0.2;
  o.q_cut = 9.0;
  o.alpha_min = 1.0 / 255.0;
  o.alpha_max = 0.99;
  o.t_min = 1e-4;
  o.dilation = 0.3;
  o.band_q = 2e-4;
  o.band_a = 2e-4;
  o.band_z = 1e-6;  // wide, so that groups form
  o.band_znear = 1e-9;
  o.eps_alpha = 3e-5;
  o.eps_mul = 1e-6;
  o.budget = 4;
  o.sh_degree = 3;
  const int64_t n = (int64_t)N * W * H;
  std::vector<int32_t> rv(n), rx(n), ry(n);
  for (int64_t i = 0; i < n; ++i) {
    rv[i] = (int32_t)(i / (W * H));
    rx[i] = (int32_t)((i / W) % H);
    ry[i] = (int32_t)(i % W);
  }
  std::vector<double> prim(n * 3), var(n * 3 * 32);
  std::vector<int32_t> nvar(n), info(n * 4);
  if (dlo_render_rays(G, means.data(), ls.data(), quats.data(), logits.data(), sh.data(), N, R.data(), t.data(),
                      eye.data(), &o, n, rv.data(), rx.data(), ry.data(), prim.data(), nvar.data(), var.data(),
                      info.data()))
    return 1;
  std::vector<double> grad(n * 3);
  for (auto& g : grad) g = 2.0 * rng.next() - 1.0;
  std::vector<double> gm(G * 3), gl(G * 3), gq(G * 4), go(G), gs(G * 48);
  if (dlo_backward_rays(G, means.data(), ls.data(), quats.data(), logits.data(), sh.data(), N, R.data(), t.data(),
                        eye.data(), &o, n, rv.data(), rx.data(), ry.data(), grad.data(), gm.data(), gl.data(),
                        gq.data(), go.data(), gs.data()))
    return 2;
  std::vector<double> rec(G * 16);
  if (dlo_project(G, means.data(), ls.data(), quats.data(), logits.data(), sh.data(), R.data(), t.data(),
                  eye.data(), &o, rec.data()))
    return 3;
  // Alg. 2 on a small panel with a negative slant and an offset
  const int pw_w = 40, pw_h = 30;
  std::vector<uint8_t> V((size_t)pw_h * 3 * pw_w);
  std::vector<int32_t> src((size_t)pw_h * pw_w * 3);
  if (dlo_repurpose(pw_w, pw_h, 9, -1, 4, 9, 2, 7, 3, 2, V.data(), src.data())) return 4;
  if (dlo_count_rays(pw_w, pw_h, V.data(), src.data()) < pw_w * pw_h) return 5;
  int64_t groups = 0;
  for (int64_t i = 0; i < n; ++i) groups += info[i * 4 + 3];
  std::printf("ok %lld rays, %lld near-tie groups\n", (long long)n, (long long)groups);
  return 0;
}

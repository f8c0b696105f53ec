// Oracle (test infrastructure only): a plain, slow CPU FP64 renderer of the light-field image.
//
// Only tests, the smoke check and the CPU-baseline leg of the benchmark link this file.  It shares no code
// with the HIP path.  Every ray is rendered by brute force over all Gaussians of its view.
//
// What it computes (paper Sec. 3.3, Eq. (7)-(10), and the per-ray view of Sec. 5):
//   * Sigma = R S S^T R^T from the normalised quaternion and exp(log-scale)              Eq. (8)
//   * Sigma' = J W Sigma W^T J^T (EWA, J the Jacobian of the perspective map), plus a
//     screen-space low-pass dilation h*I                                                   Eq. (9)
//   * alpha = min(alpha_max, o * exp(-q/2)) with q = d^T Sigma'^{-1} d at the pixel centre  Eq. (10)
//   * front-to-back compositing C = sum alpha_i T_i c_i, T_i = prod_{j<i} (1 - alpha_j)       Eq. (5)-(6)
//     over the Gaussians that pass the per-pixel rule (z > z_near, q <= q_cut,
//     alpha >= alpha_min), ordered by camera depth, ties by Gaussian index; the walk stops
//     before a Gaussian whose blend would take T below t_min.
//   * colour: real spherical harmonics of degree <= 3 in the direction from the camera to the
//     Gaussian mean, plus 0.5, clamped below at 0.
//
// Several results are correct where FP32 arithmetic on the GPU and FP64 here can take a threshold
// decision differently (q at q_cut, alpha at alpha_min, T at t_min, z at z_near, near-equal depths).
// Such "fragile" decisions are evaluated both ways (at most `budget` of them per ray), and every reachable
// outcome is returned; a GPU value is admissible if it is close to any of them.
//
// The adjoint (for gradient checks) reverses the compositing by hand and obtains the Jacobian of the
// per-view projection (mean2d, conic, opacity, colour) with respect to the Gaussian's parameters by
// forward-mode dual numbers, so that no chain rule of the projection is derived by hand here.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------------------------------------------
// forward-mode dual numbers with a fixed number of tangents
// ------------------------------------------------------------------------------------------------
constexpr int NT = 11;  // mu(3), log-scale(3), quaternion(4), opacity logit(1)

struct Dual {
  double v;
  double d[NT];
  Dual() : v(0) { std::memset(d, 0, sizeof d); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof d); }  // NOLINT: implicit constant
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int i = 0; i < NT; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int i = 0; i < NT; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); Dual r(e); for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * e; return r; }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); Dual r(s); for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] / (2 * s); return r; }
inline double val(const Dual& a) { return a.v; }
inline double val(double a) { return a; }
using std::exp;
using std::sqrt;

// ------------------------------------------------------------------------------------------------
// options and camera
// ------------------------------------------------------------------------------------------------
}  // namespace

extern "C" {
typedef struct {
  double focal, cx, cy;                     // intrinsics: focal (px), principal point (px)
  double z_near, q_cut, alpha_min, alpha_max, t_min, dilation;
  double bg[3];
  double band_q;       // q is fragile if |q - q_cut| <= band_q * q_cut
  double band_a;       // alpha is fragile if |alpha - alpha_min| <= band_a * alpha_min
  double band_z;       // adjacent depths are a near-tie if |dz| <= band_z * max(z, 1)
  double band_znear;   // z is fragile if |z - z_near| <= band_znear * z_near
  double eps_alpha;    // relative error bound of the GPU's alpha (termination band)
  double eps_mul;      // per-step relative error of the GPU's transmittance update
  int32_t budget;      // max fragile decisions explored per ray (<= 4)
  int32_t sh_degree;   // 0..3
} dlo_opts;
}

namespace {

struct Cam {
  double R[9], t[3], eye[3];
};

// ------------------------------------------------------------------------------------------------
// real spherical harmonics (no Condon-Shortley phase), index l*l + l + m, m = -l..l
//   Y_l^0     = N_l0 P_l(z)
//   Y_l^{+m}  = sqrt(2) N_lm Q_l^m(z) Re((x + i y)^m)
//   Y_l^{-m}  = sqrt(2) N_lm Q_l^m(z) Im((x + i y)^m)
// with P_l^m(z) = (1 - z^2)^{m/2} Q_l^m(z) the associated Legendre function and
// N_lm = sqrt((2l + 1) / (4 pi) * (l - m)! / (l + m)!).  On the unit sphere (x + i y)^m = sin^m(theta) e^{i m phi}.
// ------------------------------------------------------------------------------------------------
double factorial(int n) { double r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }

template <class S>
void sh_basis(int degree, const S& x, const S& y, const S& z, S* Y) {
  // Q_l^m by the Legendre recurrence in l for fixed m
  S Q[4][4];
  for (int m = 0; m <= degree; ++m) {
    double dfact = 1;  // (2m-1)!!
    for (int k = 2 * m - 1; k > 1; k -= 2) dfact *= k;
    Q[m][m] = S(dfact);
    if (m + 1 <= degree) Q[m + 1][m] = z * double(2 * m + 1) * Q[m][m];
    for (int l = m + 2; l <= degree; ++l)
      Q[l][m] = (z * double(2 * l - 1) * Q[l - 1][m] - double(l + m - 1) * Q[l - 2][m]) / double(l - m);
  }
  // (x + i y)^m
  S re[4], im[4];
  re[0] = S(1.0); im[0] = S(0.0);
  for (int m = 1; m <= degree; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
  for (int l = 0; l <= degree; ++l) {
    for (int m = 0; m <= l; ++m) {
      double N = std::sqrt((2 * l + 1) / (4 * M_PI) * factorial(l - m) / factorial(l + m));
      if (m == 0) {
        Y[l * l + l] = Q[l][0] * N;
      } else {
        double c = std::sqrt(2.0) * N;
        Y[l * l + l + m] = Q[l][m] * re[m] * c;
        Y[l * l + l - m] = Q[l][m] * im[m] * c;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------------
// per-view projection of one Gaussian
// ------------------------------------------------------------------------------------------------
template <class S>
struct Proj {
  S u, v;            // mean in image coordinates (column, row), pixel centres at +0.5
  S ca, cb, cc;      // conic = inverse of Sigma' = [[ca, cb], [cb, cc]]
  S cov_a, cov_b, cov_c;  // Sigma'
  S opac;            // sigmoid(logit)
  S raw[3];          // SH colour + 0.5, before the clamp at 0
  S z;               // camera depth
  S dir[3];          // unit direction camera -> mean
};

template <class S>
void project(const S mu[3], const S ls[3], const S qt[4], const S& logit, const Cam& cam, const dlo_opts& o,
             const float* sh, int64_t sh_stride_coef, Proj<S>& P, double* Yout) {
  const double* W = cam.R;
  S X = mu[0] * W[0] + mu[1] * W[1] + mu[2] * W[2] + cam.t[0];
  S Y = mu[0] * W[3] + mu[1] * W[4] + mu[2] * W[5] + cam.t[1];
  S Z = mu[0] * W[6] + mu[1] * W[7] + mu[2] * W[8] + cam.t[2];
  P.z = Z;
  // Eq. (8): Sigma = R S S^T R^T, R from the normalised quaternion (w, x, y, z)
  S qn = sqrt(qt[0] * qt[0] + qt[1] * qt[1] + qt[2] * qt[2] + qt[3] * qt[3]);
  S w = qt[0] / qn, qx = qt[1] / qn, qy = qt[2] / qn, qz = qt[3] / qn;
  S Rq[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - w * qz), 2.0 * (qx * qz + w * qy),
             2.0 * (qx * qy + w * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - w * qx),
             2.0 * (qx * qz - w * qy), 2.0 * (qy * qz + w * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
  S s2[3];
  for (int k = 0; k < 3; ++k) { S s = exp(ls[k]); s2[k] = s * s; }
  S Sig[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      S acc(0.0);
      for (int k = 0; k < 3; ++k) acc = acc + Rq[a * 3 + k] * s2[k] * Rq[b * 3 + k];
      Sig[a * 3 + b] = acc;
    }
  // view-space covariance W Sigma W^T
  S Sc[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      S acc(0.0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc = acc + W[a * 3 + i] * Sig[i * 3 + j] * W[b * 3 + j];
      Sc[a * 3 + b] = acc;
    }
  // Eq. (9): Sigma' = J Sc J^T (+ h I), J = d(f X/Z, f Y/Z)/d(X, Y, Z)
  const double f = o.focal;
  S J[6] = {f / Z, S(0.0), -f * X / (Z * Z), S(0.0), f / Z, -f * Y / (Z * Z)};
  S C2[4];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      S acc(0.0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc = acc + J[a * 3 + i] * Sc[i * 3 + j] * J[b * 3 + j];
      C2[a * 2 + b] = acc;
    }
  P.cov_a = C2[0] + o.dilation;
  P.cov_b = C2[1];
  P.cov_c = C2[3] + o.dilation;
  S det = P.cov_a * P.cov_c - P.cov_b * P.cov_b;
  P.ca = P.cov_c / det;
  P.cb = -P.cov_b / det;
  P.cc = P.cov_a / det;
  P.u = f * X / Z + o.cx;
  P.v = f * Y / Z + o.cy;
  P.opac = 1.0 / (1.0 + exp(-logit));
  // colour from SH in the direction eye -> mean
  S dx = mu[0] - cam.eye[0], dy = mu[1] - cam.eye[1], dz = mu[2] - cam.eye[2];
  S dn = sqrt(dx * dx + dy * dy + dz * dz);
  P.dir[0] = dx / dn; P.dir[1] = dy / dn; P.dir[2] = dz / dn;
  S Yb[16];
  const int deg = o.sh_degree;
  sh_basis(deg, P.dir[0], P.dir[1], P.dir[2], Yb);
  const int nb = (deg + 1) * (deg + 1);
  for (int c = 0; c < 3; ++c) {
    S acc(0.5);
    for (int l = 0; l < nb; ++l) acc = acc + Yb[l] * double(sh[l * sh_stride_coef + c]);
    P.raw[c] = acc;
  }
  if (Yout)
    for (int l = 0; l < nb; ++l) Yout[l] = val(Yb[l]);
}

struct Scene {
  int64_t G;
  const float *means, *log_scales, *quats, *logits, *sh;
};

void project_double(const Scene& sc, int64_t i, const Cam& cam, const dlo_opts& o, Proj<double>& P) {
  double mu[3] = {sc.means[i * 3], sc.means[i * 3 + 1], sc.means[i * 3 + 2]};
  double ls[3] = {sc.log_scales[i * 3], sc.log_scales[i * 3 + 1], sc.log_scales[i * 3 + 2]};
  double qt[4] = {sc.quats[i * 4], sc.quats[i * 4 + 1], sc.quats[i * 4 + 2], sc.quats[i * 4 + 3]};
  double lg = sc.logits[i];
  project<double>(mu, ls, qt, lg, cam, o, sc.sh + i * 48, 3, P, nullptr);
}

// ------------------------------------------------------------------------------------------------
// per-ray compositing
// ------------------------------------------------------------------------------------------------
struct Cand {
  double z;
  int64_t idx;
  double alpha;      // min(alpha_max, o exp(-q/2))
  bool clamped;      // alpha took the alpha_max branch
  double rgb[3];
  int state;         // 1 = included, 2 = fragile (included or not), truth in `truth`
  bool truth;
};

constexpr int kMaxVar = 32;      // admissible outcomes kept per ray
constexpr int kMaxOrders = 24;   // depth orders of near-tie groups explored per ray

struct RayOut {
  double prim[3];
  double var[kMaxVar][3];
  int nvar;
  int over;       // more fragile decisions or near-tie orders than explored on some path
  int nfrag;      // fragile decisions met on the primary path
  int nblend;     // Gaussians blended on the primary path
  int nties;      // near-tie groups among the candidates the walks reach
  double t_final;
};

struct Walker {
  const dlo_opts* o;
  RayOut* out;
  size_t reach;   // furthest candidate position any path examined (a stop there, or the list's end)
  void emit(const double C[3], double T) {
    if (out->nvar >= kMaxVar) { out->over = 1; return; }
    for (int c = 0; c < 3; ++c) out->var[out->nvar][c] = C[c] + T * o->bg[c];
    out->nvar++;
  }
  // Walk the candidate list from position j.  Fragile decisions branch while budget lasts.
  void walk(const std::vector<Cand>& cs, size_t j, double T, const double Cin[3], double errT, int budget) {
    double C[3] = {Cin[0], Cin[1], Cin[2]};
    for (; j < cs.size(); ++j) {
      const Cand& c = cs[j];
      if (c.state == 2) {
        if (budget > 0) {
          walk(cs, j + 1, T, C, errT, budget - 1);  // variant that leaves this Gaussian out
          budget -= 1;                               // this path blends it
        } else {
          out->over = 1;
          if (!c.truth) continue;
        }
      }
      const double a = c.alpha;
      const double Tn = T * (1.0 - a);
      double errTn = errT + o->eps_mul + (c.clamped ? 0.0 : (a / (1.0 - a)) * o->eps_alpha);
      bool stop = Tn < o->t_min;
      bool tfrag = std::fabs(Tn - o->t_min) <= errTn * o->t_min;
      if (tfrag) {
        if (budget > 0) {
          budget -= 1;
          if (stop) {
            // variant: continue past this Gaussian
            double C2[3];
            for (int k = 0; k < 3; ++k) C2[k] = C[k] + a * T * c.rgb[k];
            walk(cs, j + 1, Tn, C2, errTn, budget);
          } else {
            reach = std::max(reach, j);
            emit(C, T);  // variant: stop here
          }
        } else {
          out->over = 1;
        }
      }
      if (stop) { reach = std::max(reach, j); emit(C, T); return; }
      for (int k = 0; k < 3; ++k) C[k] += a * T * c.rgb[k];
      T = Tn;
      errT = errTn;
    }
    reach = std::max(reach, cs.size());
    emit(C, T);
  }
};

// Primary (FP64 truth) walk; also records the blended sequence for the adjoint.
void walk_primary(const std::vector<Cand>& cs, const dlo_opts& o, double C[3], double& T, int& nblend, int& nfrag,
                  std::vector<int>* seq) {
  C[0] = C[1] = C[2] = 0.0;
  T = 1.0;
  nblend = 0;
  nfrag = 0;
  double errT = 0.0;
  for (size_t j = 0; j < cs.size(); ++j) {
    const Cand& c = cs[j];
    if (c.state == 2) { nfrag++; if (!c.truth) continue; }
    const double a = c.alpha;
    const double Tn = T * (1.0 - a);
    errT += o.eps_mul + (c.clamped ? 0.0 : (a / (1.0 - a)) * o.eps_alpha);
    if (std::fabs(Tn - o.t_min) <= errT * o.t_min) nfrag++;
    if (Tn < o.t_min) return;
    for (int k = 0; k < 3; ++k) C[k] += a * T * c.rgb[k];
    T = Tn;
    nblend++;
    if (seq) seq->push_back((int)j);
  }
}

// Collect the candidates of ray (px, py) over all Gaussians of a projected view.
void collect(const std::vector<Proj<double>>& P, double px, double py, const dlo_opts& o, std::vector<Cand>& cs) {
  cs.clear();
  const int64_t G = (int64_t)P.size();
  for (int64_t i = 0; i < G; ++i) {
    const Proj<double>& p = P[i];
    const double z = p.z;
    if (!(z > 0.0)) continue;
    bool z_in = z > o.z_near;
    bool z_frag = std::fabs(z - o.z_near) <= o.band_znear * o.z_near;
    if (!z_in && !z_frag) continue;
    const double dx = px - p.u, dy = py - p.v;
    const double q = p.ca * dx * dx + 2.0 * p.cb * dx * dy + p.cc * dy * dy;  // Eq. (10) exponent
    bool q_in = q <= o.q_cut;
    bool q_frag = std::fabs(q - o.q_cut) <= o.band_q * o.q_cut;
    if (!q_in && !q_frag) continue;
    const double g = p.opac * std::exp(-0.5 * q);
    const bool clamped = g > o.alpha_max;
    const double alpha = clamped ? o.alpha_max : g;
    bool a_in = alpha >= o.alpha_min;
    bool a_frag = std::fabs(alpha - o.alpha_min) <= o.band_a * o.alpha_min;
    if (!a_in && !a_frag) continue;
    const bool truth = z_in && q_in && a_in;
    const bool frag = truth ? (z_frag || q_frag || a_frag)
                            : ((z_in || z_frag) && (q_in || q_frag) && (a_in || a_frag));
    if (!truth && !frag) continue;
    Cand c;
    c.z = z;
    c.idx = i;
    c.alpha = alpha;
    c.clamped = clamped;
    for (int k = 0; k < 3; ++k) c.rgb[k] = std::max(0.0, p.raw[k]);
    c.state = frag ? 2 : 1;
    c.truth = truth;
    cs.push_back(c);
  }
  std::sort(cs.begin(), cs.end(), [](const Cand& a, const Cand& b) {
    return a.z < b.z || (a.z == b.z && a.idx < b.idx);
  });
}

// Near-tie groups: maximal runs cs[a..b] (b > a) of consecutive candidates whose adjacent depths differ by
// at most the band (but are not equal: equal FP64 depths come from equal means, which both sides order by
// index).  Within a group the depth order is not defined at the GPU's precision, so every permutation of it is
// an admissible order.  Only groups that start at or before `reach` can change the composite: a walk never
// examines a candidate after the position where it stopped.
struct TieGroup { size_t a, n; };

void tie_groups(const std::vector<Cand>& cs, size_t reach, double band, std::vector<TieGroup>& gs) {
  gs.clear();
  size_t j = 0;
  while (j + 1 < cs.size() && j <= reach) {
    size_t b = j;
    while (b + 1 < cs.size()) {
      const double dz = std::fabs(cs[b + 1].z - cs[b].z);
      if (dz == 0.0 || dz > band * std::max(cs[b].z, 1.0)) break;
      ++b;
    }
    if (b > j) gs.push_back({j, b - j + 1});
    j = b + 1;
  }
}

void render_ray(const std::vector<Proj<double>>& P, double px, double py, const dlo_opts& o, std::vector<Cand>& cs,
                RayOut& out) {
  collect(P, px, py, o, cs);
  double T;
  walk_primary(cs, o, out.prim, T, out.nblend, out.nfrag, nullptr);
  for (int k = 0; k < 3; ++k) out.prim[k] += T * o.bg[k];
  out.t_final = T;
  out.nvar = 0;
  out.over = 0;
  out.nties = 0;
  const int budget = std::min(o.budget, 4);
  Walker w{&o, &out, 0};
  const double C0[3] = {0, 0, 0};
  w.walk(cs, 0, 1.0, C0, 0.0, budget);  // the exact order, fragile thresholds both ways
  // orders of the near-tie groups the walks reach; a permuted order can carry a walk past the first reach,
  // so the groups are taken again up to the new reach until they no longer change
  std::vector<TieGroup> gs, seen;
  std::vector<Cand> alt;
  size_t done_reach = 0;
  for (int round = 0; round < 4; ++round) {
    tie_groups(cs, w.reach, o.band_z, gs);
    if (round > 0 && w.reach == done_reach) break;
    done_reach = w.reach;
    if (gs.size() == seen.size()) break;   // groups are found in order: same count = same groups
    seen = gs;
    out.nties = (int)gs.size();
    // mixed-radix enumeration of one permutation per group (index 0 = the exact order)
    long total = 1;
    for (const TieGroup& g : gs) {
      long f = 1;
      for (size_t i = 2; i <= g.n; ++i) f *= (long)i;
      total *= f;
      if (total > kMaxOrders) break;
    }
    if (total > kMaxOrders) { out.over = 1; return; }
    out.nvar = 0;
    w.walk(cs, 0, 1.0, C0, 0.0, budget);
    for (long code = 1; code < total; ++code) {
      alt = cs;
      long c = code;
      int used = 0;
      for (const TieGroup& g : gs) {
        long f = 1;
        for (size_t i = 2; i <= g.n; ++i) f *= (long)i;
        long pc = c % f;
        c /= f;
        if (pc == 0) continue;
        used++;
        std::vector<size_t> perm(g.n);
        for (size_t i = 0; i < g.n; ++i) perm[i] = i;
        for (long r = 0; r < pc; ++r) std::next_permutation(perm.begin(), perm.end());
        for (size_t i = 0; i < g.n; ++i) alt[g.a + i] = cs[g.a + perm[i]];
      }
      w.walk(alt, 0, 1.0, C0, 0.0, std::max(0, budget - used));
    }
  }
  if (w.reach != done_reach) {
    tie_groups(cs, w.reach, o.band_z, gs);
    if (gs.size() != seen.size()) out.over = 1;  // still growing after the last round: not explored
  }
}

void make_cams(int N, const double* R, const double* t, const double* eye, std::vector<Cam>& cams) {
  cams.resize(N);
  for (int v = 0; v < N; ++v) {
    std::memcpy(cams[v].R, R + v * 9, 9 * sizeof(double));
    std::memcpy(cams[v].t, t + v * 3, 3 * sizeof(double));
    std::memcpy(cams[v].eye, eye + v * 3, 3 * sizeof(double));
  }
}

void project_view(const Scene& sc, const Cam& cam, const dlo_opts& o, std::vector<Proj<double>>& P) {
  P.resize(sc.G);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < sc.G; ++i) project_double(sc, i, cam, o, P[i]);
}

std::vector<std::vector<int64_t>> rays_by_view(int N, int64_t n_rays, const int32_t* ray_v) {
  std::vector<std::vector<int64_t>> by(N);
  for (int64_t r = 0; r < n_rays; ++r) by[ray_v[r]].push_back(r);
  return by;
}

}  // namespace

extern "C" {

int dlo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Projected records of all Gaussians for one camera, 16 doubles each:
// u, v, conic a, b, c, opacity, r, g, b (clamped colour), z, cov a, b, c, raw r, g, b.
int dlo_project(int64_t G, const float* means, const float* log_scales, const float* quats, const float* logits,
                const float* sh, const double* R, const double* t, const double* eye, const dlo_opts* o,
                double* out) {
  Scene sc{G, means, log_scales, quats, logits, sh};
  Cam cam;
  std::memcpy(cam.R, R, sizeof cam.R);
  std::memcpy(cam.t, t, sizeof cam.t);
  std::memcpy(cam.eye, eye, sizeof cam.eye);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < G; ++i) {
    Proj<double> P;
    project_double(sc, i, cam, *o, P);
    double* r = out + i * 16;
    r[0] = P.u; r[1] = P.v; r[2] = P.ca; r[3] = P.cb; r[4] = P.cc; r[5] = P.opac;
    for (int k = 0; k < 3; ++k) { r[6 + k] = std::max(0.0, P.raw[k]); r[13 + k] = P.raw[k]; }
    r[9] = P.z; r[10] = P.cov_a; r[11] = P.cov_b; r[12] = P.cov_c;
  }
  return 0;
}

// Real SH basis values (no Condon-Shortley phase) at unit directions dirs[n][3] -> Y[n][16].
void dlo_sh_basis(int64_t n, int32_t degree, const double* dirs, double* Y) {
  for (int64_t i = 0; i < n; ++i) {
    double y[16] = {0};
    sh_basis<double>(degree, dirs[i * 3], dirs[i * 3 + 1], dirs[i * 3 + 2], y);
    std::memcpy(Y + i * 16, y, sizeof y);
  }
}

// Render rays (v, x = row, y = column).  out_prim[n][3]: FP64 truth; out_var[n][32][3] with out_nvar[n]
// admissible outcomes; out_info[n][4] = (over-budget flag, fragile decisions on the primary path,
// Gaussians blended, near-tie groups explored).
int dlo_render_rays(int64_t G, const float* means, const float* log_scales, const float* quats, const float* logits,
                    const float* sh, int32_t N, const double* R, const double* t, const double* eye,
                    const dlo_opts* o, int64_t n_rays, const int32_t* ray_v, const int32_t* ray_x,
                    const int32_t* ray_y, double* out_prim, int32_t* out_nvar, double* out_var, int32_t* out_info) {
  Scene sc{G, means, log_scales, quats, logits, sh};
  std::vector<Cam> cams;
  make_cams(N, R, t, eye, cams);
  auto by = rays_by_view(N, n_rays, ray_v);
  std::vector<Proj<double>> P;
  for (int v = 0; v < N; ++v) {
    if (by[v].empty()) continue;
    project_view(sc, cams[v], *o, P);
    const auto& rays = by[v];
#pragma omp parallel
    {
      std::vector<Cand> cs;
      cs.reserve(1024);
#pragma omp for schedule(dynamic, 16)
      for (int64_t k = 0; k < (int64_t)rays.size(); ++k) {
        const int64_t r = rays[k];
        RayOut ro;
        render_ray(P, ray_y[r] + 0.5, ray_x[r] + 0.5, *o, cs, ro);
        for (int c = 0; c < 3; ++c) out_prim[r * 3 + c] = ro.prim[c];
        if (out_var) {
          out_nvar[r] = ro.nvar;
          std::memcpy(out_var + r * 3 * kMaxVar, ro.var, sizeof(double) * 3 * std::min(ro.nvar, kMaxVar));
        }
        if (out_info) {
          out_info[r * 4 + 0] = ro.over;
          out_info[r * 4 + 1] = ro.nfrag;
          out_info[r * 4 + 2] = ro.nblend;
          out_info[r * 4 + 3] = ro.nties;
        }
      }
    }
  }
  return 0;
}

// FP64 adjoint of sum_r grad_rgb[r] . C(r) over the given rays, along the primary (FP64 truth) path;
// threshold decisions carry no gradient.  Gradients are accumulated (+=) into the outputs, in the user
// layouts means[G][3], log_scales[G][3], quats[G][4], logits[G], sh[G][16][3].
int dlo_backward_rays(int64_t G, const float* means, const float* log_scales, const float* quats, const float* logits,
                      const float* sh, int32_t N, const double* R, const double* t, const double* eye,
                      const dlo_opts* o, int64_t n_rays, const int32_t* ray_v, const int32_t* ray_x,
                      const int32_t* ray_y, const double* grad_rgb, double* g_means, double* g_log_scales,
                      double* g_quats, double* g_logits, double* g_sh) {
  Scene sc{G, means, log_scales, quats, logits, sh};
  std::vector<Cam> cams;
  make_cams(N, R, t, eye, cams);
  auto by = rays_by_view(N, n_rays, ray_v);
  std::vector<Proj<double>> P;
  int nth = dlo_num_threads();
  // per-thread accumulators of d loss / d (u, v, ca, cb, cc, opac, raw r, g, b) per Gaussian
  std::vector<double> acc((size_t)nth * G * 9);
  std::vector<double> tot((size_t)G * 9);
  for (int v = 0; v < N; ++v) {
    if (by[v].empty()) continue;
    project_view(sc, cams[v], *o, P);
    std::fill(acc.begin(), acc.end(), 0.0);
    const auto& rays = by[v];
#pragma omp parallel
    {
#ifdef _OPENMP
      const int tid = omp_get_thread_num();
#else
      const int tid = 0;
#endif
      double* A = acc.data() + (size_t)tid * G * 9;
      std::vector<Cand> cs;
      std::vector<int> seq;
#pragma omp for schedule(dynamic, 16)
      for (int64_t k = 0; k < (int64_t)rays.size(); ++k) {
        const int64_t r = rays[k];
        const double px = ray_y[r] + 0.5, py = ray_x[r] + 0.5;
        const double* g = grad_rgb + r * 3;
        if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
        collect(P, px, py, *o, cs);
        seq.clear();
        double C[3], Tf;
        int nb, nf;
        walk_primary(cs, *o, C, Tf, nb, nf, &seq);
        // reverse sweep: Rv = sum_{k>j} alpha_k T_k c_k + T_final bg
        double Rv[3] = {Tf * o->bg[0], Tf * o->bg[1], Tf * o->bg[2]};
        double T = Tf;
        for (int s = (int)seq.size() - 1; s >= 0; --s) {
          const Cand& c = cs[seq[s]];
          const double a = c.alpha;
          T = T / (1.0 - a);  // transmittance before this Gaussian
          double gc = 0.0, gR = 0.0;
          for (int ch = 0; ch < 3; ++ch) { gc += g[ch] * c.rgb[ch]; gR += g[ch] * Rv[ch]; }
          const double dalpha = T * gc - gR / (1.0 - a);
          double* Ai = A + c.idx * 9;
          for (int ch = 0; ch < 3; ++ch) {
            const Proj<double>& p = P[c.idx];
            if (p.raw[ch] > 0.0) Ai[6 + ch] += g[ch] * a * T;
            Rv[ch] += a * T * c.rgb[ch];
          }
          if (!c.clamped) {
            const Proj<double>& p = P[c.idx];
            const double dx = px - p.u, dy = py - p.v;
            const double G0 = std::exp(-0.5 * (p.ca * dx * dx + 2.0 * p.cb * dx * dy + p.cc * dy * dy));
            const double dq = dalpha * (-0.5 * a);
            Ai[5] += dalpha * G0;
            Ai[0] += dq * (-2.0) * (p.ca * dx + p.cb * dy);
            Ai[1] += dq * (-2.0) * (p.cb * dx + p.cc * dy);
            Ai[2] += dq * dx * dx;
            Ai[3] += dq * 2.0 * dx * dy;
            Ai[4] += dq * dy * dy;
          }
        }
      }
    }
    std::fill(tot.begin(), tot.end(), 0.0);
    for (int th = 0; th < nth; ++th) {
      const double* A = acc.data() + (size_t)th * G * 9;
      for (int64_t i = 0; i < G * 9; ++i) tot[i] += A[i];
    }
    // chain through the projection of view v by forward-mode duals
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < G; ++i) {
      const double* T9 = tot.data() + i * 9;
      bool any = false;
      for (int k = 0; k < 9; ++k) any |= T9[k] != 0.0;
      if (!any) continue;
      Dual mu[3], ls[3], qt[4], lg;
      for (int k = 0; k < 3; ++k) { mu[k] = Dual(sc.means[i * 3 + k]); mu[k].d[k] = 1.0; }
      for (int k = 0; k < 3; ++k) { ls[k] = Dual(sc.log_scales[i * 3 + k]); ls[k].d[3 + k] = 1.0; }
      for (int k = 0; k < 4; ++k) { qt[k] = Dual(sc.quats[i * 4 + k]); qt[k].d[6 + k] = 1.0; }
      lg = Dual(sc.logits[i]);
      lg.d[10] = 1.0;
      Proj<Dual> Pd;
      double Yb[16];
      project<Dual>(mu, ls, qt, lg, cams[v], *o, sc.sh + i * 48, 3, Pd, Yb);
      const Dual* outs[9] = {&Pd.u, &Pd.v, &Pd.ca, &Pd.cb, &Pd.cc, &Pd.opac, &Pd.raw[0], &Pd.raw[1], &Pd.raw[2]};
      double gp[NT] = {0};
      for (int k = 0; k < 9; ++k)
        for (int d = 0; d < NT; ++d) gp[d] += T9[k] * outs[k]->d[d];
      for (int k = 0; k < 3; ++k) g_means[i * 3 + k] += gp[k];
      for (int k = 0; k < 3; ++k) g_log_scales[i * 3 + k] += gp[3 + k];
      for (int k = 0; k < 4; ++k) g_quats[i * 4 + k] += gp[6 + k];
      g_logits[i] += gp[10];
      const int nb = (o->sh_degree + 1) * (o->sh_degree + 1);
      for (int l = 0; l < nb; ++l)
        for (int c = 0; c < 3; ++c) g_sh[i * 48 + l * 3 + c] += T9[6 + c] * Yb[l];
    }
  }
  return 0;
}

}  // extern "C"

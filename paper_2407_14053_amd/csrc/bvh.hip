// Bounding volume hierarchy over the scene's Gaussians for ray-order rendering (Sec. "Ray-Order 3DGS",
// Eq. (21)), built on the host once per scene.
//
// Leaves hold Gaussians; each Gaussian's box bounds the ellipsoid q = (x - mu)^T Sigma^-1 (x - mu) <= q_lim with
// q_lim = min(q_cut, 2 ln(o / alpha_min)): where along any ray a Gaussian can pass the hit rule (q <= q_cut and
// o exp(-q/2) >= alpha_min at its peak), the peak lies in that ellipsoid, so the traversal finds every hit.
// Gaussians whose opacity is below alpha_min can never be hit and are left out.
//
// Build: a binary tree by binned SAH (16 bins on each axis, the cost of Eq. (21) with c_node = c_prim = 1,
// leaves of at most kBvhLeafMax Gaussians, object-median splits below binary depth 48 so that depth stays
// bounded), then collapsed to 8-wide nodes by opening, at each wide node, the largest-area internal child
// until it has 8 children.  Children of a wide node are its internal nodes and leaf ranges of the Gaussian
// order the tree induces (records are stored in that order).
#include "dl_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace dl {
namespace {

struct Box {
  double lo[3], hi[3];
  void reset() {
    for (int k = 0; k < 3; ++k) {
      lo[k] = INFINITY;
      hi[k] = -INFINITY;
    }
  }
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b.lo[k]);
      hi[k] = std::max(hi[k], b.hi[k]);
    }
  }
  double area() const {
    const double e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
    if (!(e0 >= 0) || !(e1 >= 0) || !(e2 >= 0)) return 0.0;
    return 2.0 * (e0 * e1 + e1 * e2 + e2 * e0);
  }
};

struct BNode {  // binary node
  Box box;
  int left = -1, right = -1;  // internal: child indices
  int start = 0, count = 0;   // leaf: Gaussian range in the build order
  bool leaf() const { return left < 0; }
};

constexpr int kBins = 16;
constexpr int kMedianDepth = 48;
constexpr double kCostNode = 1.0, kCostPrim = 1.0;

struct Builder {
  const std::vector<Box>& pb;
  std::vector<double> cen;  // centroid [3 n]
  std::vector<int32_t>& ord;
  std::vector<BNode> nodes;

  Builder(const std::vector<Box>& b, std::vector<int32_t>& o) : pb(b), ord(o) {
    cen.resize(3 * pb.size());
    for (size_t i = 0; i < pb.size(); ++i)
      for (int k = 0; k < 3; ++k) cen[3 * i + k] = 0.5 * (pb[i].lo[k] + pb[i].hi[k]);
  }

  int build() {
    struct Task {
      int node, start, end, depth;
    };
    nodes.reserve(2 * pb.size() / kBvhLeafMax + 16);
    nodes.push_back(BNode());
    std::vector<Task> st{{0, 0, (int)ord.size(), 0}};
    while (!st.empty()) {
      Task tk = st.back();
      st.pop_back();
      const int n = tk.end - tk.start;
      Box box, cb;
      box.reset();
      cb.reset();
      for (int i = tk.start; i < tk.end; ++i) {
        box.grow(pb[ord[i]]);
        Box c;
        for (int k = 0; k < 3; ++k) c.lo[k] = c.hi[k] = cen[3 * ord[i] + k];
        cb.grow(c);
      }
      nodes[tk.node].box = box;
      int mid = -1;
      const double pa = box.area();
      if (tk.depth < kMedianDepth && n > 1) {
        // binned SAH over the centroid bounds
        double best = INFINITY;
        int bax = -1, bsplit = -1;
        for (int ax = 0; ax < 3; ++ax) {
          const double ext = cb.hi[ax] - cb.lo[ax];
          if (!(ext > 0)) continue;
          Box bb[kBins];
          int bc[kBins] = {0};
          for (int b = 0; b < kBins; ++b) bb[b].reset();
          const double sc = kBins / ext;
          for (int i = tk.start; i < tk.end; ++i) {
            int b = (int)((cen[3 * ord[i] + ax] - cb.lo[ax]) * sc);
            b = std::min(std::max(b, 0), kBins - 1);
            bc[b]++;
            bb[b].grow(pb[ord[i]]);
          }
          double ra[kBins];
          int rc[kBins];
          Box acc;
          acc.reset();
          int cnt = 0;
          for (int b = kBins - 1; b > 0; --b) {
            acc.grow(bb[b]);
            cnt += bc[b];
            ra[b] = acc.area();
            rc[b] = cnt;
          }
          acc.reset();
          cnt = 0;
          for (int b = 0; b < kBins - 1; ++b) {
            acc.grow(bb[b]);
            cnt += bc[b];
            if (cnt == 0 || rc[b + 1] == 0) continue;
            const double cost = kCostNode + kCostPrim * (acc.area() * cnt + ra[b + 1] * rc[b + 1]) / std::max(pa, 1e-300);
            if (cost < best) {
              best = cost;
              bax = ax;
              bsplit = b;
            }
          }
        }
        const double leaf_cost = kCostPrim * n;
        if (bax >= 0 && (n > kBvhLeafMax || best < leaf_cost)) {
          const double sc = kBins / (cb.hi[bax] - cb.lo[bax]);
          auto it = std::partition(ord.begin() + tk.start, ord.begin() + tk.end, [&](int32_t g) {
            int b = (int)((cen[3 * g + bax] - cb.lo[bax]) * sc);
            return std::min(std::max(b, 0), kBins - 1) <= bsplit;
          });
          mid = (int)(it - ord.begin());
          if (mid == tk.start || mid == tk.end) mid = -1;
        }
      }
      if (mid < 0 && n > kBvhLeafMax) {
        // object median on the widest centroid axis (also for coincident centroids: index order)
        int ax = 0;
        for (int k = 1; k < 3; ++k)
          if (cb.hi[k] - cb.lo[k] > cb.hi[ax] - cb.lo[ax]) ax = k;
        mid = tk.start + n / 2;
        std::nth_element(ord.begin() + tk.start, ord.begin() + mid, ord.begin() + tk.end, [&](int32_t a, int32_t b) {
          const double ca = cen[3 * a + ax], cb2 = cen[3 * b + ax];
          return ca < cb2 || (ca == cb2 && a < b);
        });
      }
      if (mid < 0) {
        nodes[tk.node].start = tk.start;
        nodes[tk.node].count = n;
        continue;
      }
      const int l = (int)nodes.size();
      nodes.push_back(BNode());
      nodes.push_back(BNode());
      nodes[tk.node].left = l;
      nodes[tk.node].right = l + 1;
      st.push_back({l + 1, mid, tk.end, tk.depth + 1});
      st.push_back({l, tk.start, mid, tk.depth + 1});
    }
    return 0;
  }
};

float round_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -INFINITY);
  return f;
}
float round_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

}  // namespace

int bvh_build_host(const float* soa, int64_t n, int64_t n_pad, float q_cut, float alpha_min, BvhHost* out,
                   std::string* why) {
  // Gaussians in FP64 from the FP32 parameters: Sigma^-1 = R S^-2 R^T, box half-extents k sqrt(Sigma_ii)
  std::vector<Box> boxes;
  std::vector<int32_t> ids;
  std::vector<double> inv6, mu3, op1, ql1;
  boxes.reserve(n);
  const double lam = 2.0 * std::log(1.0 / (double)alpha_min);
  for (int64_t i = 0; i < n; ++i) {
    double mu[3], s[3], q[4];
    for (int k = 0; k < 3; ++k) mu[k] = soa[(kRowMean + k) * n_pad + i];
    for (int k = 0; k < 3; ++k) s[k] = std::exp((double)soa[(kRowLogScale + k) * n_pad + i]);
    for (int k = 0; k < 4; ++k) q[k] = soa[(kRowQuat + k) * n_pad + i];
    const double lg = soa[kRowLogit * n_pad + i];
    const double o = 1.0 / (1.0 + std::exp(-lg));
    const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    bool ok = std::isfinite(qn) && qn > 0 && std::isfinite(o);
    for (int k = 0; k < 3; ++k) ok = ok && std::isfinite(mu[k]) && std::isfinite(s[k]) && s[k] > 0;
    if (!ok) continue;
    const double ql = std::min((double)q_cut, 2.0 * std::log(o) + lam);
    if (!(ql > 0)) continue;  // opacity below alpha_min: never hit
    const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    double A[3][3], Sg[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double ai = 0, sg = 0;
        for (int k = 0; k < 3; ++k) {
          ai += R[a][k] * R[b][k] / (s[k] * s[k]);
          sg += R[a][k] * R[b][k] * (s[k] * s[k]);
        }
        A[a][b] = ai;
        Sg[a][b] = sg;
      }
    // ellipsoid q <= ql (1 + 2e-3): hits the FP32 traversal accepts near q_lim stay inside; plus a margin for
    // the FP32 slab test
    const double kk = std::sqrt(ql * (1.0 + 2e-3));
    Box b;
    double mag = 1.0;
    for (int k = 0; k < 3; ++k) mag = std::max(mag, std::fabs(mu[k]));
    for (int k = 0; k < 3; ++k) {
      const double e = kk * std::sqrt(Sg[k][k]) * (1.0 + 1e-5) + 1e-6 * mag;
      b.lo[k] = mu[k] - e;
      b.hi[k] = mu[k] + e;
    }
    boxes.push_back(b);
    ids.push_back((int32_t)i);
    const double a6[6] = {A[0][0], A[0][1], A[0][2], A[1][1], A[1][2], A[2][2]};
    inv6.insert(inv6.end(), a6, a6 + 6);
    mu3.insert(mu3.end(), mu, mu + 3);
    op1.push_back(o);
    ql1.push_back(ql);
  }
  const int64_t m = (int64_t)boxes.size();
  if (m >= (1ll << 28)) {
    *why = "too many Gaussians for the BVH (2^28)";
    return DL_EINVAL;
  }
  out->n_prims = m;
  std::vector<int32_t> ord(m);
  for (int64_t i = 0; i < m; ++i) ord[i] = (int32_t)i;
  std::vector<BNode> bn;
  if (m > 0) {
    Builder B(boxes, ord);
    B.build();
    bn.swap(B.nodes);
  }
  // collapse to 8-wide nodes (breadth first); children per wide node: binary node ids
  struct WTask {
    int bnode, wnode;
  };
  std::vector<WTask> q;
  out->nodes.clear();
  int nw = 0;
  auto new_wide = [&]() {
    out->nodes.resize(out->nodes.size() + kBvhNodeFloats);
    return nw++;
  };
  new_wide();
  if (m > 0) q.push_back({0, 0});
  for (size_t qi = 0; qi < q.size(); ++qi) {
    const WTask t = q[qi];
    std::vector<int> ch;
    if (bn[t.bnode].leaf()) {
      ch.push_back(t.bnode);
    } else {
      ch.push_back(bn[t.bnode].left);
      ch.push_back(bn[t.bnode].right);
      while ((int)ch.size() < 8) {
        int bi = -1;
        double ba = -1;
        for (int c = 0; c < (int)ch.size(); ++c)
          if (!bn[ch[c]].leaf() && bn[ch[c]].box.area() > ba) {
            ba = bn[ch[c]].box.area();
            bi = c;
          }
        if (bi < 0) break;
        const int b = ch[bi];
        ch[bi] = bn[b].left;
        ch.push_back(bn[b].right);
      }
    }
    float* node = &out->nodes[(size_t)t.wnode * kBvhNodeFloats];
    for (int c = 0; c < 8; ++c) {
      uint32_t ref = kBvhEmpty;
      float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
      if (c < (int)ch.size()) {
        const BNode& b = bn[ch[c]];
        for (int k = 0; k < 3; ++k) {
          lo[k] = round_down(b.box.lo[k]);
          hi[k] = round_up(b.box.hi[k]);
        }
        if (b.leaf()) {
          ref = kBvhLeafBit | ((uint32_t)(b.count - 1) << 28) | (uint32_t)b.start;
        } else {
          const int w = new_wide();
          node = &out->nodes[(size_t)t.wnode * kBvhNodeFloats];  // storage may have moved
          ref = (uint32_t)w;
          q.push_back({ch[c], w});
        }
      }
      for (int k = 0; k < 3; ++k) {
        node[k * 8 + c] = lo[k];
        node[(3 + k) * 8 + c] = hi[k];
      }
      std::memcpy(&node[48 + c], &ref, 4);
    }
    // own box (for pruning a node when it is popped)
    Box own;
    own.reset();
    for (int c : ch) own.grow(bn[c].box);
    for (int k = 0; k < 3; ++k) {
      node[56 + k] = round_down(own.lo[k]);
      node[59 + k] = round_up(own.hi[k]);
    }
    node[62] = node[63] = 0.0f;
  }
  if (m == 0) {
    float* node = &out->nodes[0];
    for (int c = 0; c < 8; ++c) {
      for (int k = 0; k < 3; ++k) {
        node[k * 8 + c] = 3e38f;
        node[(3 + k) * 8 + c] = -3e38f;
      }
      uint32_t ref = kBvhEmpty;
      std::memcpy(&node[48 + c], &ref, 4);
    }
    for (int k = 0; k < 3; ++k) {
      node[56 + k] = 3e38f;
      node[59 + k] = -3e38f;
    }
  }
  out->n_nodes = nw;
  // stack bound (a node's children, internal and leaf, are pushed together and popped one at a time) and
  // depth, bottom-up
  std::vector<int> bound(nw, 0), depth(nw, 1);
  int64_t leaves = 0;
  double sah = 0.0;
  const double root_area = m > 0 ? std::max(bn[0].box.area(), 1e-300) : 1.0;
  for (int w = nw - 1; w >= 0; --w) {
    int mcnt = 0, mb = 0, md = 0;
    for (int c = 0; c < 8; ++c) {
      uint32_t ref;
      std::memcpy(&ref, &out->nodes[(size_t)w * kBvhNodeFloats + 48 + c], 4);
      if (ref == kBvhEmpty) continue;
      ++mcnt;
      if (ref & kBvhLeafBit) {
        ++leaves;
        continue;
      }
      mb = std::max(mb, bound[ref]);
      md = std::max(md, depth[ref]);
    }
    bound[w] = mcnt ? std::max(mcnt, mcnt - 1 + mb) : 0;
    depth[w] = 1 + md;
  }
  // Eq. (21) over the binary tree the wide tree was cut from (areas relative to the root)
  for (const BNode& b : bn)
    sah += b.leaf() ? b.box.area() / root_area * b.count * kCostPrim : b.box.area() / root_area * kCostNode;
  out->n_leaves = leaves;
  out->depth = depth[0];
  out->stack_bound = std::max(1, bound[0]);
  out->sah_cost = sah;
  // records in leaf order: [mu, o], [a00 a01 a02 a11], [a12 a22 q_lim, index]
  out->rec.assign((size_t)m * 12, 0.0f);
  out->perm.assign(m, 0);
  for (int64_t r = 0; r < m; ++r) {
    const int32_t j = ord[r];
    float* d = &out->rec[(size_t)r * 12];
    for (int k = 0; k < 3; ++k) d[k] = (float)mu3[3 * j + k];
    d[3] = (float)op1[j];
    for (int k = 0; k < 4; ++k) d[4 + k] = (float)inv6[6 * j + k];
    d[8] = (float)inv6[6 * j + 4];
    d[9] = (float)inv6[6 * j + 5];
    d[10] = (float)ql1[j];
    const uint32_t gi = (uint32_t)ids[j];
    std::memcpy(&d[11], &gi, 4);
    out->perm[r] = ids[j];
  }
  return DL_OK;
}

}  // namespace dl

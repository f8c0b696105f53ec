// Oracle (test infrastructure only): subpixel repurposing (paper Sec. "Subpixel Repurposing", Eq. (11)-(14)),
// compiled for full-size panels.  Only tests link this file; it shares no code with the HIP path, and it is the
// same reading as oracle/repurpose.py (which runs on small panels in pure Python; the tests check the two agree).
//
// What it computes: for every subpixel (x, y, k), whose view is v = V(x, 3y + k) (Eq. (1)-(3)), the pixel
// (x', y') of view v whose channel k it shows (the index matrix of Eq. (11)/(13); the view and the channel are
// kept).  A pixel rendered for one of its channels lends its two other channels to later subpixels of the same
// view nearby (Eq. (12)), so fewer distinct rays (v, x', y') are rendered.
//
// Reading of the heuristic (the text leaves it open; each point is one line of the design notes):
//   * areas: a pixel belongs to the slanted strip of P_w grating units that its left edge lies in:
//     area = floor(d_offset(x, y, 0) / (P_w L_x)) with d_offset of Eq. (1); areas are taken in increasing
//     order, the subpixels of an area in row-major order (row, column, channel);
//   * each subpixel not yet assigned starts a chain of its view v with nothing held for v;
//   * a chain assigns its current subpixel: if a pixel is held for its channel, that pixel is shown and no
//     longer held (Eq. (13)); otherwise the subpixel shows its own pixel, which is then held for the view's two
//     other channels in place of anything held there (Eq. (11)-(12));
//   * it then looks for its next subpixel in the window of Eq. (14) (rows min(x + 2, h - 1) .. min(x +
//     floor(5 N / (2 L_x)), h - 1), columns max(y - floor(N / (3 L_x)), 0) .. y): a subpixel of view v not yet
//     assigned, preferring one whose channel has a held pixel, first in row-major order either way; the search
//     does not look at areas, and the chain goes on only if the subpixel found lies in the chain's area;
//   * when it stops, whatever it still holds is dropped.
#include <algorithm>
#include <cstdint>
#include <vector>

namespace {

using i128 = __int128;

int64_t floordiv(i128 a, i128 b) {  // b > 0
  i128 q = a / b;
  if (a % b != 0 && a < 0) --q;
  return (int64_t)q;
}

struct Panel {
  int W, H, N;
  int64_t a, b, p, q, r, c;  // tan(alpha) = a/b, L_x = p/q, K_offset = r/c
};

// d_offset(x, s) times b c (an integer): (s b c + 3 x a c - r b)
i128 doff_bc(const Panel& P, int x, int64_t s) {
  return (i128)s * P.b * P.c + (i128)3 * x * P.a * P.c - (i128)P.r * P.b;
}

}  // namespace

extern "C" {

// View map V[H][3W] (Eq. (1)-(3), exact) and src[H][W][3] = source pixel index x' W + y' of every subpixel.
// Returns 0, or -1 when the integers do not fit.
int dlo_repurpose(int W, int H, int N, int64_t a, int64_t b, int64_t p, int64_t q, int64_t r, int64_t c, int pw,
                  uint8_t* V, int32_t* src) {
  if (W < 1 || H < 1 || N < 1 || N > 255 || b <= 0 || p <= 0 || q <= 0 || c <= 0 || pw < 1) return -1;
  if ((int64_t)W * H > (int64_t)1 << 30) return -1;
  const Panel P{W, H, N, a, b, p, q, r, c};
  const int W3 = 3 * W;
  const i128 Qv = (i128)b * c * p;            // view: floor(N frac(d_offset / L_x))
  const i128 Qa = (i128)b * c * p * pw;       // area: floor(d_offset / (P_w L_x))
  for (int x = 0; x < H; ++x)
    for (int s = 0; s < W3; ++s) {
      i128 rho = (doff_bc(P, x, s) * q) % Qv;
      if (rho < 0) rho += Qv;
      V[(int64_t)x * W3 + s] = (uint8_t)((N * rho) / Qv);
    }
  // pixel areas, then the pixels of every area in row-major order (counting sort, stable)
  const int64_t npix = (int64_t)W * H;
  std::vector<int64_t> area(npix);
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  for (int x = 0; x < H; ++x)
    for (int y = 0; y < W; ++y) {
      const int64_t A = floordiv(doff_bc(P, x, 3 * (int64_t)y) * q, Qa);
      area[(int64_t)x * W + y] = A;
      lo = std::min(lo, A);
      hi = std::max(hi, A);
    }
  const int64_t nA = hi - lo + 1;
  if (nA > ((int64_t)1 << 31)) return -1;
  std::vector<int64_t> start(nA + 1, 0);
  for (int64_t i = 0; i < npix; ++i) ++start[area[i] - lo + 1];
  for (int64_t k = 0; k < nA; ++k) start[k + 1] += start[k];
  std::vector<int32_t> order(npix);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < npix; ++i) order[fill[area[i] - lo]++] = (int32_t)i;
  }
  // Eq. (14) window extents
  const int drow = (int)floordiv((i128)5 * N * q, (i128)2 * p);  // 2 N / L_x + N / (2 L_x)
  const int dcol = (int)floordiv((i128)N * q, (i128)3 * p);      // N / (3 L_x)
  std::fill(src, src + (int64_t)H * W3, -1);
  for (int64_t i = 0; i < npix; ++i) {
    const int32_t pix0 = order[i];
    const int x0 = pix0 / W, y0 = pix0 % W;
    for (int k0 = 0; k0 < 3; ++k0) {
      if (src[(int64_t)pix0 * 3 + k0] >= 0) continue;
      const int v = V[(int64_t)x0 * W3 + 3 * y0 + k0];
      const int64_t A = area[pix0];
      int32_t held[3] = {-1, -1, -1};  // pixel held for each channel of view v
      int x = x0, y = y0, k = k0;
      for (;;) {
        const int32_t here = x * W + y;
        if (held[k] >= 0) {
          src[(int64_t)here * 3 + k] = held[k];
          held[k] = -1;
        } else {
          src[(int64_t)here * 3 + k] = here;
          held[(k + 1) % 3] = here;
          held[(k + 2) % 3] = here;
        }
        const int r_lo = std::min(x + 2, H - 1), r_hi = std::min(x + drow, H - 1);
        const int c_lo = std::max(y - dcol, 0), c_hi = y;
        int fx = -1, fy = -1, fk = -1, px = -1, py = -1, pk = -1;
        for (int xx = r_lo; xx <= r_hi && px < 0; ++xx)
          for (int yy = c_lo; yy <= c_hi && px < 0; ++yy)
            for (int kk = 0; kk < 3; ++kk) {
              const int64_t j = (int64_t)xx * W3 + 3 * yy + kk;
              if (V[j] != v || src[j] >= 0) continue;
              if (fx < 0) {
                fx = xx;
                fy = yy;
                fk = kk;
              }
              if (held[kk] >= 0) {
                px = xx;
                py = yy;
                pk = kk;
                break;
              }
            }
        if (px >= 0) {
          fx = px;
          fy = py;
          fk = pk;
        }
        if (fx < 0 || area[(int64_t)fx * W + fy] != A) break;
        x = fx;
        y = fy;
        k = fk;
      }
    }
  }
  return 0;
}

// Distinct rays (v, x', y') of a source map: a ray is named by its pixel and the first of that pixel's subpixels
// that has its view.  Returns the count, or -1 if a source does not show the subpixel's view.
int64_t dlo_count_rays(int W, int H, const uint8_t* V, const int32_t* src) {
  const int64_t npix = (int64_t)W * H;
  std::vector<uint8_t> used(npix, 0);
  int64_t n = 0;
  for (int64_t s = 0; s < 3 * npix; ++s) {
    const int64_t pix = src[s];
    if (pix < 0 || pix >= npix) return -1;
    const uint8_t v = V[s];
    int j = -1;
    for (int i = 2; i >= 0; --i)
      if (V[3 * pix + i] == v) j = i;
    if (j < 0) return -1;
    if (!(used[pix] & (1u << j))) {
      used[pix] |= (uint8_t)(1u << j);
      ++n;
    }
  }
  return n;
}

}  // extern "C"

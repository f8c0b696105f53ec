// Internal declarations shared by the gfx950 kernels and the host runtime of the light-field renderer.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include <cstdint>

#include "../../include/directl.h"

namespace dl {

// Scene structure-of-arrays: row r of length n_pad holds one float parameter of every Gaussian.
constexpr int kRowMean = 0;      // 3 rows: x, y, z
constexpr int kRowLogScale = 3;  // 3 rows
constexpr int kRowQuat = 6;      // 4 rows: w, x, y, z
constexpr int kRowLogit = 10;    // 1 row
constexpr int kRowSH = 11;       // 48 rows: coefficient l, channel c at kRowSH + 3 l + c
constexpr int kSceneRows = 59;

// Projected record of one (view, Gaussian): 12 floats = 3 x float4 (binning reads only the first two).
//   [0] u  [1] v  [2] A  [3] B  [4] C  [5] Q_limit (tile-test cutoff, same scale as A, B, C)
//   [6] ext_x  [7] ext_y (half extents of the cutoff ellipse, px)  [8] opacity  [9..11] rgb
// with A = a log2(e)/2, B = b log2(e), C = c log2(e)/2 for the conic [[a, b], [b, c]] = Sigma'^{-1}, so that
// Q = A dx^2 + B dx dy + C dy^2 = q log2(e)/2 and o exp(-q/2) = o 2^-Q.
constexpr int kRecF4 = 3;
constexpr int kGaussBlockF4 = 18;  // per-Gaussian block of the projection's view-independent terms (288 B)

// Per-view camera block uploaded for every frame: 16 doubles = rotation rows (9), t (3), eye (3), 0.
constexpr int kCamDoubles = 16;

// The camera rig of a frame (Sec. 3.1, the light-field centre extrinsic): the centre camera-to-world pose, the
// convergence distance, the baseline and the view count.  rig_camera writes view v's camera (kCamDoubles: the
// world-to-camera rotation rows right, down, forward, the translation, the eye, 0): the eye at
// eye_0 + baseline (v / (N - 1) - 1/2) right_0, aimed at eye_0 + converge_dist forward_0 with down_0 as the
// reference down axis.  Host and device run this one function (IEEE division and square root, no contraction),
// so the cameras an eager frame builds on the device equal those the host validates and stages for plans.
// Returns 1 if the forward axis vanishes or is parallel to down_0 (the host rejects such poses).
struct CamRig {
  double c2w[16];
  double converge_dist, baseline;
  int n;
};
__host__ __device__ inline int rig_camera(const CamRig& r, int v, double* c) {
  const double* m = r.c2w;
  const double right0[3] = {m[0], m[4], m[8]}, down0[3] = {m[1], m[5], m[9]}, fwd0[3] = {m[2], m[6], m[10]};
  const double eye0[3] = {m[3], m[7], m[11]};
  double target[3];
  for (int k = 0; k < 3; ++k) target[k] = eye0[k] + r.converge_dist * fwd0[k];
  const double s = r.n > 1 ? r.baseline * ((double)v / (double)(r.n - 1) - 0.5) : 0.0;
  double eye[3], f[3], rt[3], dn[3];
  for (int k = 0; k < 3; ++k) eye[k] = eye0[k] + s * right0[k];
  for (int k = 0; k < 3; ++k) f[k] = target[k] - eye[k];
  const double nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(nf > 0)) return 1;
  for (int k = 0; k < 3; ++k) f[k] /= nf;
  // right = down0 x forward, down = forward x right
  rt[0] = down0[1] * f[2] - down0[2] * f[1];
  rt[1] = down0[2] * f[0] - down0[0] * f[2];
  rt[2] = down0[0] * f[1] - down0[1] * f[0];
  const double nr = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
  if (!(nr > 0)) return 1;
  for (int k = 0; k < 3; ++k) rt[k] /= nr;
  dn[0] = f[1] * rt[2] - f[2] * rt[1];
  dn[1] = f[2] * rt[0] - f[0] * rt[2];
  dn[2] = f[0] * rt[1] - f[1] * rt[0];
  for (int k = 0; k < 3; ++k) {
    c[k] = rt[k];
    c[3 + k] = dn[k];
    c[6 + k] = f[k];
  }
  for (int a = 0; a < 3; ++a) c[9 + a] = -(c[a * 3] * eye[0] + c[a * 3 + 1] * eye[1] + c[a * 3 + 2] * eye[2]);
  for (int k = 0; k < 3; ++k) c[12 + k] = eye[k];
  c[15] = 0.0;
  return 0;
}

struct ProjConst {
  int64_t G;        // Gaussians
  int64_t n_pad;    // scene row stride
  int N, W, H;
  int sh_degree;
  double focal, cx, cy;
  float z_near, q_cut, alpha_min, alpha_max, dilation;
  int key_e0;  // biased FP64 exponent of z_near: depth keys count exponents from it
};

// Depth keys: (exponent of z - key_e0, saturated at kDepthExpMax) << 31 | top 31 mantissa bits of the FP64 z.
// Monotone in z (strictly, to 2^-31 relative, below 2^kDepthExpMax z_near); culled items carry kDepthCulled.
// 36 bits: four radix passes of 9 bits.
constexpr int kDepthMantBits = 31;
constexpr int kDepthKeyBits = 5 + kDepthMantBits;
constexpr int kDepthExpMax = 30;
constexpr uint64_t kDepthCulled = (1ull << kDepthKeyBits) - 1;

struct BlendConst {
  int W, H;
  int tw, th, ntx, nty;  // tile size and tile grid of the panel
  int T;                 // ntx * nty
  int N;                 // views
  int64_t G;             // record stride per view
  float q_cut;  // in the scaled units of the record (q_cut log2(e)/2)
  float alpha_min, alpha_max, t_min;
  float log2_alpha_min;
  float bg[3];
  unsigned long long* stats;  // optional work counters, kStatSlots x {evaluations, blends, rays}
  // repurposed panel (nullptr: every ray fills channels of its own pixel): tgt[(3 p + j) * 3 + k] = the subpixel
  // filled by channel k of the ray of pixel p whose entry carries slot j (bits 27-28), or -1
  const int32_t* tgt;
  // DirectL: every ray of the panel fills exactly one channel (its three subpixels belong to three views)
  int single_channel;
};
constexpr int kStatSlots = 1024;

// The blend's bound on E = log2(o) - Q (Q = q log2(e)/2, the scaled quadratic form) for a record with
// lo = log2(o): a pair blends iff E >= max(lo - Q_cut, log2 alpha_min), i.e. q <= q_cut and
// o exp(-q/2) >= alpha_min.
__device__ inline float blend_elim(float lo, const BlendConst& bc) {
  return fmaxf(lo - bc.q_cut, bc.log2_alpha_min);
}

// The clamp of a record's alpha, alpha = min(cap, o 2^-Q): alpha_max for a Gaussian whose opacity comes within
// 2^-10 of alpha_max, else +inf (then o 2^-Q <= o stays below alpha_max and min(alpha_max, .) never applies, so
// alpha = min(alpha_max, o exp(-q/2)) either way; a rounding excess of the computed 2^-Q above 1 would have to
// exceed 2^-10 to make the two differ).
__device__ inline float blend_cap(float o, const BlendConst& bc) {
  return o > bc.alpha_max * (1.0f - 1.0f / 1024.0f) ? bc.alpha_max : __builtin_inff();
}

// Depth chunk: ranks [n_v num_lo / den, n_v num_hi / den) of every view; `stride` bounds its length.
struct ChunkArgs {
  int64_t num_lo, num_hi, den;
  // front[v]: size of view v's front (the first chunk); later chunks start no earlier.  The chunk of view v is
  // ranks [0, front) for the first chunk, else [max(front, n lo), max(that, n hi)) of its n visible ranks (the
  // second chunk has lo = 0, so that the chunks tile the ranks whatever the front's size).
  const uint32_t* front;
  int first;
  int64_t stride;   // item slots per view (a multiple of 64 is not required)
  int64_t wstride;  // wavefront slots per view: ceil(stride / 64)
  uint32_t cap;     // key capacity
  int64_t tgx;      // workgroups per view of the table-form binning (set by its launchers)
  int64_t front_max;  // table form: an upper bound of any view's first-chunk ranks (sizes the grid; 0: stride)
};

// Real spherical harmonics without the Condon-Shortley phase, index l*l + l + m, m = -l..l, written as
// polynomials of the unit direction (x, y, z):
//   l=0: 1/(2 sqrt(pi))
//   l=1: sqrt(3/(4pi)) * (y, z, x)
//   l=2: (1/2)sqrt(15/pi) xy, (1/2)sqrt(15/pi) yz, (1/4)sqrt(5/pi)(3z^2 - 1), (1/2)sqrt(15/pi) xz,
//        (1/4)sqrt(15/pi)(x^2 - y^2)
//   l=3: (1/4)sqrt(35/(2pi)) y(3x^2 - y^2), (1/2)sqrt(105/pi) xyz, (1/4)sqrt(21/(2pi)) y(5z^2 - 1),
//        (1/4)sqrt(7/pi) z(5z^2 - 3), (1/4)sqrt(21/(2pi)) x(5z^2 - 1), (1/4)sqrt(105/pi) z(x^2 - y^2),
//        (1/4)sqrt(35/(2pi)) x(x^2 - 3y^2)
__device__ inline void sh_basis(int deg, float x, float y, float z, float* Y) {
  Y[0] = 0.28209479177387814f;
  if (deg < 1) return;
  Y[1] = 0.4886025119029199f * y;
  Y[2] = 0.4886025119029199f * z;
  Y[3] = 0.4886025119029199f * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = 1.0925484305920792f * (x * y);
  Y[5] = 1.0925484305920792f * (y * z);
  Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
  Y[7] = 1.0925484305920792f * (x * z);
  Y[8] = 0.5462742152960396f * (xx - yy);
  if (deg < 3) return;
  Y[9] = 0.5900435899266435f * y * (3.0f * xx - yy);
  Y[10] = 2.890611442640554f * (x * y) * z;
  Y[11] = 0.4570457994644658f * y * (5.0f * zz - 1.0f);
  Y[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
  Y[13] = 0.4570457994644658f * x * (5.0f * zz - 1.0f);
  Y[14] = 1.445305721320277f * z * (xx - yy);
  Y[15] = 0.5900435899266435f * x * (xx - 3.0f * yy);
}

// Per-chunk blend flags
struct BlendChunk {
  int first, last;
  unsigned long long* later;  // given: set to 1 by every workgroup whose tile keeps a live ray
};

// ---- view map and ray lists (viewmap.hip) ----
hipError_t launch_view_map(uint8_t* V, int W, int H, int N, int64_t As, int64_t Ax, int64_t C, int64_t Q, int wide,
                           hipStream_t s);
hipError_t launch_rays_emit(const uint8_t* V, int W, int H, int tw, int th, int ntx, int T, uint32_t* keys,
                            uint32_t* vals, hipStream_t s);
hipError_t launch_interleave(const uint8_t* V, const float* views, float* out, int W, int H, hipStream_t s);
// *count += ray entries ent[0, n) whose channel mask holds more than one channel (count zeroed by the caller)
hipError_t launch_count_multichannel(const uint32_t* ent, int64_t n, uint32_t* count, hipStream_t s);
// Alg. 1 with a bilinear Resize of views[N][vh][vw][3] to the panel (src: source pixels of a repurposed panel)
hipError_t launch_interleave_resize(const uint8_t* V, const int32_t* src, const float* views, float* out, int W,
                                   int H, int vw, int vh, hipStream_t s);

// ---- subpixel repurposing (repurpose.hip) ----
// Host: src[(x W + y) 3 + k] = source pixel x' W + y' of subpixel (x, y, k) for the panel d with P_w = pw, from
// the view map V[H][3W] (host copy).  Returns a DL_ code (message in *why).
int repurpose_sources(const dl_display_desc& d, int pw, const uint8_t* V, int32_t* src, std::string* why);
// tgt[9 W H] from src (see BlendConst::tgt); *err = 1 if a source pixel does not show its subpixel's view.
hipError_t launch_tgt_build(const uint8_t* V, const int32_t* src, int W, int H, int32_t* tgt, int32_t* err,
                            hipStream_t s);
// Ray entries of a repurposed panel (as launch_rays_emit, with the target slot in bits 27-28).
hipError_t launch_rays_emit_sr(const uint8_t* V, const int32_t* tgt, int W, int H, int tw, int th, int ntx, int T,
                               uint32_t* keys, uint32_t* vals, hipStream_t s);
// Alg. 1 through a repurposed map: out[s] = views[V[s]][src[s]][s mod 3].
hipError_t launch_interleave_sr(const uint8_t* V, const int32_t* src, const float* views, float* out, int W, int H,
                                hipStream_t s);
// out[s] = s / 3 (every subpixel's own pixel), [3 W H].
hipError_t launch_own_pixel(int32_t* out, int W, int H, hipStream_t s);

// ---- scans, radix sort, ranges (sort.hip) ----
int64_t scan_partial_count(int64_t n);
// exclusive scan of n uint32 (in may equal out); `partial` holds scan_partial_count(n) + 1 entries and
// receives the grand total in partial[scan_partial_count(n)].
// With n_dev, only the first min(n, n_mul * *n_dev) entries are scanned; the grand total of what was scanned lands in
// partial[scan_partial_count(n)] either way.  byte_sums: each input word counts as the sum of its four bytes.
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partial, hipStream_t s,
                              const uint32_t* n_dev = nullptr, int n_mul = 1, bool byte_sums = false);
int64_t radix_hist_size(int64_t seg_len, int n_seg);
// Stable partition of (key = digit < n_dig, value) pairs within each of n_seg segments given as device ranges
// [seg_start[s], seg_start[s + 1]) of one array (clamped to cap): afterwards every segment holds its values
// grouped by digit, in input order within a digit.  start[s * n_dig + d] receives the first position of
// digit d in segment s, start[n_seg * n_dig] the end.  Returns the buffer holding the partitioned values
// (v0 or v1); keys k0/k1 are scratch.  hist: tile_partition_hist_size(n_seg) entries; layout: the 2 n_seg + 1
// entries launch_chunk_setup wrote for these ranges; n_seg <= 256.
int64_t tile_partition_hist_size(int n_seg);
const uint32_t* tile_partition(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int n_seg,
                               const uint32_t* seg_start, uint32_t cap, int n_dig, uint32_t* hist, uint32_t* partial,
                               uint32_t* layout, uint32_t* start, hipStream_t s, hipError_t* err);
// Stable LSD sort of n_seg segments (static length seg_len, live length seg_n[s] clamped to cap when seg_n is
// given) of (key, value) pairs by key bits [bit_lo, bit_hi), each segment independently.  Ping-pongs between
// (k0, v0) and (k1, v1); returns true when the result ends in (k1, v1).
bool radix_sort_u64(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t seg_len, int n_seg,
                    const uint32_t* seg_n, uint32_t cap, int bit_lo, int bit_hi, uint32_t* hist, uint32_t* partial,
                    hipStream_t s, hipError_t* err);
// One stable pass over full segments [s seg_len, (s + 1) seg_len) of keys k0 that leaves out items whose key is
// drop_key and splits the rest into keys < thr[s] (first) and keys >= thr[s]; values are the items' positions in
// their segment.  Results in (k1, v1); n_vis[s] = items kept, n_front[s] = items below thr[s].  hist holds
// split_hist_size(seg_len, n_seg) entries.  With `live`, segments s with live[s] == 0 are left alone (nothing
// written, counts kept); with back_only, only the items >= thr[s] are written (at the same places).
int64_t split_hist_size(int64_t seg_len, int n_seg);
int split_waves_per_seg(int64_t seg_len, int n_seg);
bool radix_split_u64(uint64_t* k0, uint64_t* k1, uint32_t* v1, int64_t seg_len, int n_seg, const uint64_t* thr,
                     uint64_t drop_key, uint32_t* n_vis, uint32_t* n_front, uint32_t* hist, uint32_t* partial,
                     hipStream_t s, hipError_t* err, const uint32_t* live = nullptr, bool back_only = false);
// The front part of that split alone: thr[s] is picked from the sampled histogram `hist` as launch_front_select
// does, and each of the split's runs (split_waves_per_seg runs per segment) keeps its items that are not drop_key
// and below thr[s], in order, at the run's start in kout, each packed as key << 24 | position in the segment;
// cnt (split_hist_size entries) receives per run the count of those and of all kept items, [segment][2][run].
// Segments of at most kFrontSortMaxG items.
hipError_t launch_front_gather(const uint64_t* keys, uint64_t* kout, int64_t G, int N, const uint32_t* hist,
                               int key_bits, int64_t num, int64_t den, uint64_t* thr, uint64_t drop_key,
                               uint32_t* cnt, hipStream_t s);
// Stable LSD sort of each device range [lo[s], hi[s]) in place (n_seg <= 256), with the histogram layout that
// launch_depth_ranges wrote to `layout`; returns whether the result is in (k1, v1).  hist: depth_ranges_hist_size
// entries.
int64_t depth_ranges_hist_size(int64_t seg_len, int n_seg);
bool depth_ranges_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t seg_len, int n_seg,
                       const uint32_t* lo, const uint32_t* hi, int key_bits, uint32_t* hist, uint32_t* partial,
                       uint32_t* layout, hipStream_t s, hipError_t* err);
// The front of each view's depth order: thr[v] = the smallest bin boundary of the top kFrontBits key bits with at
// least a fraction num / den of the sampled visible keys below it, from hist ([view][2^kFrontBits] counts, which
// launch_project_keys fills: front_hist_size(N) entries, zero before it).
constexpr int kFrontBits = 12;
constexpr int kFrontSamplePeriod = 1024;  // Gaussians i with i mod kFrontSamplePeriod < kFrontSampleRun are sampled
constexpr int kFrontSampleRun = 64;
int64_t front_hist_size(int N);
hipError_t launch_front_select(int N, int key_bits, int64_t num, int64_t den, const uint32_t* hist, uint64_t* thr,
                               hipStream_t s);
// Ranges of the depth sorts: live == nullptr: the fronts [vG, vG + f); else the backs [vG + f, vG + n) of views
// with a live tile (empty otherwise); rank_hi = end rank of the range; layout (2N + 1 entries) for the sort.
// The fronts of the views sorted in LDS, front_sort_parts(N) workgroups per view (each a range of the key's top
// 12 bits, at quantiles of fhist, the projection's sampled histogram below thr[v]), from the runs that
// launch_front_gather left in `items` with its counts cnt: vals[v G, v G + n_front[v]) receives the front's
// Gaussian indices in depth order, n_vis[v] the view's kept items, rank_hi[v] = n_front[v].  A front of more
// than 12288 items is sorted by one workgroup after a cut at a bin of the key's top 12 bits, thr[v] lowered to
// that bin's start and n_front to the items below it; the rest belongs to the back (a back-only split with the
// lowered thr puts it after the front).  Usable when front_sort_fits(G, N): Gaussians per view at most
// kFrontSortMaxG.
constexpr int64_t kFrontSortMaxG = 400000;
constexpr int kFrontSortCap = 12288;  // the largest front sorted in LDS (larger ones are cut)
bool front_sort_fits(int64_t G, int N);
int front_sort_parts(int N);
hipError_t launch_front_sort(const uint64_t* items, uint32_t* vals, int64_t G, int N, const uint32_t* cnt,
                             const uint32_t* fhist, uint64_t* thr, uint32_t* n_vis, uint32_t* n_front,
                             uint32_t* rank_hi, hipStream_t s);
hipError_t launch_depth_ranges(int N, int64_t G, const uint32_t* n_vis, const uint32_t* n_front,
                               const uint32_t* live, uint32_t* lo, uint32_t* hi, uint32_t* rank_hi, uint32_t* layout,
                               hipStream_t s);
// Per depth chunk: start[v] = scanned[v * wstride] (v < N), start[N] = *total (saturated), *max_total =
// max(*max_total, *total), and the tile partition's layout (2N + 1 entries) over the ranges of start.
hipError_t launch_chunk_setup(const uint32_t* scanned, int64_t wstride, int N, const unsigned long long* total,
                              unsigned long long* max_total, uint32_t cap, uint32_t* start, uint32_t* layout,
                              hipStream_t s);
bool radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t seg_len, int n_seg,
                    const uint32_t* seg_n, uint32_t cap, int bit_lo, int bit_hi, uint32_t* hist, uint32_t* partial,
                    hipStream_t s, hipError_t* err);
// start[k] = first index j < n with keys[j] >= k << shift, for k in [0, n_keys]; n = min(*n_dev, cap) or n_static
hipError_t launch_lower_bounds(const uint32_t* keys, const uint32_t* n_dev, uint32_t cap, int64_t n_static,
                               uint32_t* start, int64_t n_keys, hipStream_t s, int shift = 0);
// Ray-list keys (view T + tile, or ~0u for none) widened by four bits, (key << 4) | block, where block =
// 4 (4 row / th) + (4 column / tw) is the ray's sub-block of its tile (4 x 4 sub-blocks; the local column and row
// are the entry's bits 0-11 and 12-23), so that a stable sort lists each (view, tile)'s rays block by block.
hipError_t launch_ray_key_blocks(uint32_t* keys, const uint32_t* vals, int64_t n, int tw, int th, hipStream_t s);

// ---- projection (project.hip) ----
hipError_t launch_project(const float* soa, const double* cams, const ProjConst& pc, float4* rec, uint64_t* keys,
                          uint32_t* vals, double* depth_out, hipStream_t s);
// Depth keys of every (view, Gaussian) and each Gaussian's block of view-independent terms (blocks[G][18]); the
// sampled visible keys are added to the front histogram fhist (see launch_front_select).
hipError_t launch_project_keys(const float* soa, const double* cams, const ProjConst& pc, float4* blocks,
                               uint64_t* keys, uint32_t* fhist, hipStream_t s);
// out[v][r] = record of (view v, Gaussian sorted[v][r]) for rank_lo[v] <= r < rank_hi[v] (rank_lo nullptr: 0),
// from the blocks, with the arithmetic of launch_project; max_ranks bounds rank_hi - rank_lo (sizes the grid)
hipError_t launch_project_ranks(const float4* blocks, const double* cams, const ProjConst& pc,
                                const uint32_t* sorted, const uint32_t* rank_lo, const uint32_t* rank_hi,
                                int64_t max_ranks, float4* out, hipStream_t s);
hipError_t launch_scene_transpose(const float* means, const float* log_scales, const float* quats,
                                  const float* logits, const float* sh, int64_t n, int64_t n_pad, float* soa,
                                  hipStream_t s);

// ---- binning (bin.hip) ----
// counts[v][i] = live tiles touched by the Gaussian of depth rank lo_c(v) + i of view v; *total += sum.
// `rec` holds the records in depth-rank order; emitted values are ranks.
// counts: one per wavefront of 64 ranks, [N][wstride]; live: live tiles per view (nullptr: all views live)
hipError_t launch_bin_count(const float4* rec, const uint32_t* vis_count, const uint32_t* live, const BlendConst& bc,
                            const ChunkArgs& ch, const uint8_t* alive, uint32_t* counts, unsigned long long* total,
                            hipStream_t s);
hipError_t launch_bin_emit(const float4* rec, const uint32_t* vis_count, const uint32_t* live, const BlendConst& bc,
                           const ChunkArgs& ch, const uint8_t* alive, const uint32_t* offsets, uint32_t* keys,
                           uint32_t* vals, hipStream_t s);
// Table form of the first chunk's binning (T <= kTableMaxTiles): no partition, ranks written into the final
// (view, tile) lists.  launch_table_setup: e0[v] = min(front[v], fcap) ends the first chunk (the second starts
// there), base[v] = T * sum_{u < v} ceil(e0[u] / kTableGroup), base[N] = table length (N <= 256).  Count writes
// the table [v][t][workgroup] from base[v], one word of four byte counts (its wavefronts' hits) per entry; after
// an exclusive scan of the base[N] words' byte sums into `scanned`, emit writes the ranks of chunk ranks
// [0, e0[v]) into vals (slots below cap), and launch_table_starts writes start[NT + 1] (list bounds clamped to
// cap, start[NT] = *grand, the scan's total) and raises *max_total to the key total.
constexpr int kTableMaxTiles = 1024;
constexpr int kTableWaveRanks = 32;                   // ranks (Gaussians) per wavefront slot of the table
constexpr int kTableGroup = 4 * kTableWaveRanks;      // ranks per workgroup of the table form
constexpr int kTableStage = 8192;  // hits of one emit workgroup staged in LDS (more: written directly)
hipError_t launch_table_setup(const uint32_t* front, int N, int T, uint32_t fcap, uint32_t* e0, uint32_t* base,
                              hipStream_t s);
hipError_t launch_bin_table_count(const float4* rec, const uint32_t* vis_count, const BlendConst& bc,
                                  const ChunkArgs& ch, const uint8_t* alive, const uint32_t* base, uint32_t* table,
                                  hipStream_t s);
hipError_t launch_bin_table_emit(const float4* rec, const uint32_t* vis_count, const BlendConst& bc,
                                 const ChunkArgs& ch, const uint8_t* alive, const uint32_t* base, uint32_t* table,
                                 const uint32_t* scanned, uint32_t* vals, hipStream_t s);
hipError_t launch_table_starts(const uint32_t* scanned, const uint32_t* base, const uint32_t* e0, int N, int T,
                               const uint32_t* grand, uint32_t cap, unsigned long long* max_total,
                               unsigned long long* host_total, uint32_t* start, hipStream_t s);
// live[v] = live tiles of view v; *total = 0 (for the next chunk)
hipError_t launch_view_live(const uint8_t* alive, int64_t T, int N, uint32_t* live, unsigned long long* total,
                            hipStream_t s);


// alive[i] = tile i has rays (ray_off nullptr: all); zero32[0, n_zero) = 0; totals[0, n_totals) = 0
// (cams given: cams[v kCamDoubles ...] = rig_camera(rig, v) for v < rig.n)
hipError_t launch_frame_init(uint8_t* alive, const uint32_t* ray_off, int64_t n, uint32_t* zero32, int64_t n_zero,
                             unsigned long long* totals, int n_totals, const CamRig& rig, double* cams,
                             hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s);

// ---- blending (blend.hip) ----
// DirectL: rays of (view, tile) from ray lists; writes owned channels of out[H][W][3]; per-ray state
// (signed transmittance, colour) carried between depth chunks in `state`.
hipError_t launch_blend_directl(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                const uint32_t* ray_off, const uint32_t* ray_ent, int max_rays,
                                const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state, float* out,
                                hipStream_t s);
// Standard: all pixels of each (view, tile); writes views[v][H][W][3].
hipError_t launch_blend_standard(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                 const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state, float* views,
                                 hipStream_t s);

// ---- ray-order rendering (bvh.hip, rayorder.hip) ----
// 8-wide BVH node: 64 floats = child boxes lo x[8], lo y[8], lo z[8], hi x[8], hi y[8], hi z[8], child refs
// (uint32 bits) [8], the node's own box (lo xyz, hi xyz) and 2 unused.  A ref is a node index, or
// kBvhLeafBit | (count - 1) << 28 | first Gaussian (in leaf order), or kBvhEmpty.
constexpr int kBvhNodeFloats = 64;
constexpr int kBvhLeafMax = 4;
constexpr uint32_t kBvhLeafBit = 0x80000000u;
constexpr uint32_t kBvhEmpty = 0xffffffffu;
constexpr int kBvhStackMax = 256;  // stack entries per lane the traversal supports
struct BvhHost {
  std::vector<float> nodes;   // n_nodes * kBvhNodeFloats, root first
  std::vector<float> rec;     // per Gaussian in leaf order: [mu, o], [a00 a01 a02 a11], [a12 a22 q_lim, index]
  std::vector<int32_t> perm;  // leaf order -> scene index
  int64_t n_prims = 0, n_nodes = 0, n_leaves = 0;
  int depth = 0, stack_bound = 1;
  double sah_cost = 0.0;
};
// Host build from the scene's structure-of-arrays rows (host copy); DL_ code, message in *why.
int bvh_build_host(const float* soa, int64_t n, int64_t n_pad, float q_cut, float alpha_min, BvhHost* out,
                   std::string* why);

struct RoConst {
  int W, H, N, T, tw, th, ntx;
  int sh_degree;
  int heap_cap;    // c_h
  int stack_cap;   // stack entries per lane (the BVH's bound)
  double focal, cx, cy;
  float z_near, alpha_max, t_min;
  float bg[3];
  const int32_t* tgt;  // repurposed panel's targets (see BlendConst::tgt), or nullptr
  unsigned long long* stats;  // optional: kStatSlots x {Gaussian tests, blends, rays}
};
// One ray per lane over the (view, tile) ray lists: BVH traversal, the c_h nearest hits by peak distance, their
// blend; writes the owned channels of out[H][W][3].
hipError_t launch_rayorder(const float* nodes, const float4* rec, const float4* sh, const double* cams,
                           const uint32_t* ray_off, const uint32_t* ray_ent, const RoConst& rc, float* out,
                           hipStream_t s);

// ---- backward (backward.hip) ----
// Replays the DirectL blend of one depth chunk and accumulates d loss / d (u, v, A, B, C, o, r, g, b) per
// (view, Gaussian) into acc[9][N * G]; fwd is the forward's encoded image, gout d loss / d image.
hipError_t launch_blend_backward(const float4* rec, const uint32_t* tile_start, const uint32_t* gidx,
                                 const uint32_t* sorted, const uint32_t* ray_off, const uint32_t* ray_ent,
                                 int max_rays, const BlendConst& bc, BlendChunk bk, uint8_t* alive, float4* state,
                                 const float* fwd, const float* gout, float* acc, hipStream_t s);
// Chains acc through the projection of every view; writes gradients in the user layouts (overwritten).
hipError_t launch_project_backward(const float* soa, const double* cams, const ProjConst& pc, const float* acc,
                                   float* g_means, float* g_log_scales, float* g_quats, float* g_logits, float* g_sh,
                                   hipStream_t s);

// ---- issue-rate probe (probe.hip) ----
// Synchronous, on the current device: out[0..6] = FMA lane-ops/s, exp lane-ops/s, (4 FMA + 1 exp) steps/s, blend
// pairs/s of one-channel and of three-channel rays (per lane), measured engine clock (Hz), compute units; out[7..10]
// = v_add_f32, v_fmac_f32, negated v_mul_f32, three-VGPR v_fma_f32 lane-ops/s; DL_ code, message in *why.
int probe_issue_rates(double* out, int n_out, std::string* why);

}  // namespace dl

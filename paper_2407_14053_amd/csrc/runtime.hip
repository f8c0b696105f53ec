// Host runtime of the light-field renderer: the C ABI of include/directl.h on top of the gfx950 kernels.
//
// Frame (both paths):
//   cameras (FP64, host) -> project (all views) -> per-view depth sort (segmented radix sort, 36-bit keys)
//   -> for each depth chunk, front to back: count keys of live (view, tile) pairs -> scan -> emit
//      (view, tile) keys -> stable radix partition by key -> list bounds -> blend (carrying per-ray state,
//      retiring tiles whose rays have all terminated)
//   ; the standard path then interlaces its N views (Alg. 1).
// Every launch has a static grid; data-dependent sizes (visible counts, key counts) stay on the device.  An
// eager frame synchronises with the host after the first depth chunk, to read the live tiles (later chunks with
// nothing left to blend are skipped) together with the key count; when later chunks run, or for the backward,
// a second synchronisation at the end of the frame checks that no chunk overflowed the key capacity.  A frame
// captured into a graph has neither.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "dl_internal.h"

using namespace dl;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                                  \
  do {                                                                                                 \
    hipError_t _e = (expr);                                                                            \
    if (_e != hipSuccess) return fail(DL_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

// Scratch of dl_project_noalloc: a fixed device array that every GPU the library runs on holds until the process
// ends (a HIP module's device variable), so that entry point allocates nothing.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address is taken once per device, with that device current,
// by scratch_setup (from dl_create), and only that address is ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[DL_NOALLOC_SCRATCH_BYTES];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices] = {};

int scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return fail(DL_EINVAL, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return DL_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(DL_EHIP, std::string("device address of the no-allocation scratch: ") + hipGetErrorString(e));
  g_scratch_dev[device] = p;
  return DL_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[device];
}

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  // grow-only; contents are not preserved
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    release();
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

int64_t gcd64(int64_t a, int64_t b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

bool reduce(dl_rational& r) {
  if (r.den <= 0) return false;
  int64_t g = gcd64(r.num, r.den);
  if (g == 0) g = 1;
  r.num /= g;
  r.den /= g;
  return true;
}

__int128 mod_floor(__int128 a, __int128 m) {
  __int128 r = a % m;
  return r < 0 ? r + m : r;
}

struct RayLists {
  int tw = 0, th = 0, ntx = 0, nty = 0, T = 0;
  DevBuf off;  // [N * T + 1] uint32
  DevBuf ent;  // [n_rays] uint32
  int max_rays = 0;
  int64_t n_rays = 0;
  bool single_channel = false;  // every ray fills exactly one channel
};

}  // namespace

struct dl_ctx {
  int device = 0;
  DevBuf live;    // live tiles per view after the last blended chunk
  DevBuf vstart;  // start of each view's tile keys in the current chunk [N + 1]
  DevBuf dord, thr, fhist;  // depth order: fronts and sort ranges, front thresholds, key histogram
  DevBuf cams, rec, srec, k64[2], v32[2], vis, counts, bk[2], bv[2], hist, partial, tstart, views, stats, alive,
      state, dtotal, gacc;
  uint32_t key_cap = 0;  // current per-chunk key capacity (grows on overflow)
  double* cams_host = nullptr;  // pinned staging, 255 * 16 doubles
  // pinned and coherent (kernels write it directly), read after the first depth chunk of eager frames: that
  // chunk's key count, whether a tile is still live, then (profiled frames) the visible Gaussians of each view
  // [256]; frame_dev is its device address
  unsigned long long* frame_host = nullptr;
  unsigned long long* frame_dev = nullptr;
  // profiling: 0 off, 1 HIP events around the blend launches, 2 around every stage, 3 every stage and the
  // blend's work counters
  int prof = 0;
  struct Mark {
    int stage, chunk;
    hipEvent_t a, b;
  };
  int chunk = 0;  // depth chunk of the marks being recorded
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<Mark> marks;
  int64_t keys = 0, visible = 0;
  int batches = 0, tile_w = 0, tile_h = 0, rpt = 0, lanes = 0;
  bool later_ran = false;  // the last eager frame had a live tile after its first depth chunk
  ~dl_ctx() {
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
  }
  hipEvent_t ev() {
    if (evused == evpool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      evpool.push_back(e);
    }
    return evpool[evused++];
  }
  void frame_begin() {
    evused = 0;
    chunk = 0;
    marks.clear();
    keys = visible = 0;
    batches = 0;
  }
  int begin(int stage, hipStream_t s) {
    if (!prof || (prof == 1 && stage != DL_STAGE_BLEND)) return -1;
    Mark m{stage, chunk, ev(), ev()};
    if (!m.a || !m.b) return -1;
    (void)hipEventRecord(m.a, s);
    marks.push_back(m);
    return (int)marks.size() - 1;
  }
  void end(int i, hipStream_t s) {
    if (i >= 0) (void)hipEventRecord(marks[i].b, s);
  }
};

struct dl_scene {
  dl_ctx* ctx = nullptr;
  int64_t n = 0, n_pad = 0;
  DevBuf soa;
};

struct dl_bvh {
  dl_ctx* ctx = nullptr;
  DevBuf nodes, rec, sh;  // wide nodes; records and SH [3][16] per Gaussian in leaf order
  dl_bvh_stats st{};
};

struct dl_display {
  dl_ctx* ctx = nullptr;
  dl_display_desc desc{};
  DevBuf V;
  DevBuf src, tgt;  // repurposed panels only: source pixel per subpixel, target subpixel per (ray, channel)
  int64_t n_rays = 0;
  std::map<std::pair<int, int>, RayLists*> lists;
  ~dl_display() {
    for (auto& kv : lists) delete kv.second;
  }
};

namespace {

int check_desc(const dl_display_desc* d, dl_display_desc& o) {
  if (!d) return fail(DL_EINVAL, "display descriptor is NULL");
  o = *d;
  if (o.width < 1 || o.height < 1 || o.width > 65536 || o.height > 65536)
    return fail(DL_EINVAL, "display width/height out of range");
  if (o.n_views < 1 || o.n_views > 255) return fail(DL_EINVAL, "n_views must be in [1, 255]");
  if (!reduce(o.tan_slant) || !reduce(o.pitch) || !reduce(o.offset))
    return fail(DL_EINVAL, "rational with non-positive denominator");
  if (o.pitch.num <= 0) return fail(DL_EINVAL, "pitch must be > 0");
  if (!(o.focal_px > 0) || !std::isfinite(o.focal_px)) return fail(DL_EINVAL, "focal_px must be finite and > 0");
  if (!(o.baseline >= 0) || !std::isfinite(o.baseline)) return fail(DL_EINVAL, "baseline must be finite and >= 0");
  if (o.repurpose_pw < 0 || o.repurpose_pw > 4096) return fail(DL_EINVAL, "repurpose_pw must be in [0, 4096]");
  return DL_OK;
}

// Cameras of the rig (Eq. (17) with a horizontal toe-in rig), FP64.
// The rig of a display and pose (rig_camera builds its cameras).
CamRig make_rig(const dl_display_desc& d, const dl_pose* pose) {
  CamRig r{};
  for (int k = 0; k < 16; ++k) r.c2w[k] = pose->c2w[k];
  r.converge_dist = pose->converge_dist;
  r.baseline = d.baseline;
  r.n = d.n_views;
  return r;
}

int make_cameras(const dl_display_desc& d, const dl_pose* pose, double* out) {
  if (!pose) return fail(DL_EINVAL, "pose is NULL");
  const double* m = pose->c2w;
  for (int k = 0; k < 16; ++k)
    if (!std::isfinite(m[k])) return fail(DL_EINVAL, "pose has non-finite entries");
  if (!(pose->converge_dist > 0) || !std::isfinite(pose->converge_dist))
    return fail(DL_EINVAL, "converge_dist must be finite and > 0");
  const CamRig r = make_rig(d, pose);
  for (int v = 0; v < d.n_views; ++v)
    if (rig_camera(r, v, out + v * kCamDoubles))
      return fail(DL_EINVAL, "degenerate rig (camera at the convergence point, or forward parallel to down)");
  return DL_OK;
}

int check_opts(const dl_render_opts* o, dl_render_opts& out) {
  if (o) out = *o;
  else dl_default_opts(&out);
  if (!(out.z_near > 0) || !(out.q_cut > 0) || !(out.alpha_min > 0) || !(out.alpha_max > 0) || !(out.t_min >= 0) ||
      !(out.dilation >= 0))
    return fail(DL_EINVAL, "render options out of range");
  if (out.sh_degree < 0 || out.sh_degree > 3) return fail(DL_EINVAL, "sh_degree must be in [0, 3]");
  if (out.tile_w < 0 || out.tile_h < 0 || out.tile_w > 4096 || out.tile_h > 4096)
    return fail(DL_EINVAL, "tile size out of range");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(out.bg[k])) return fail(DL_EINVAL, "background must be finite");
  return DL_OK;
}

void auto_tile_directl(const dl_display_desc& d, int64_t n_rays, int& tw, int& th) {
  // A view owns about r/N of a tile's pixels (r = rays per pixel: 3 without repurposing).  Tiles of about 900
  // owned rays (3-4 per lane of a 256-lane workgroup) amortise each LDS-staged record over many rays and keep
  // the tile-key count low, while the extra per-ray evaluations of a larger tile stay small next to the splat
  // sizes; with fewer rays per pixel the best side grows only as (3 / r)^(1/4) (measured: the evaluations per
  // ray grow with the tile).  On large panels the tiles grow until a view has at most 1024 of them, so that
  // the first chunk's binning takes the table form.
  const double r = n_rays > 0 ? std::min(3.0, (double)n_rays / ((double)d.width * d.height)) : 3.0;
  const double side = std::sqrt(300.0 * d.n_views) * std::pow(3.0 / r, 0.25);
  int s = (int)std::floor(side / 8.0) * 8;
  s = std::max(8, std::min(s, 256));
  auto tiles = [&](int t) { return (int64_t)((d.width + t - 1) / t) * ((d.height + t - 1) / t); };
  while (tiles(s) > 1024 && s < 256) s += 8;
  tw = th = s;
}

int build_ray_lists(dl_display* D, int tw, int th, hipStream_t s, RayLists** out) {
  auto key = std::make_pair(tw, th);
  auto it = D->lists.find(key);
  if (it != D->lists.end()) {
    *out = it->second;
    return DL_OK;
  }
  const dl_display_desc& d = D->desc;
  RayLists* L = new RayLists();
  L->tw = tw;
  L->th = th;
  L->ntx = (d.width + tw - 1) / tw;
  L->nty = (d.height + th - 1) / th;
  L->T = L->ntx * L->nty;
  const int64_t NT = (int64_t)d.n_views * L->T;
  if (NT >= (1ll << 31)) {
    delete L;
    return fail(DL_EINVAL, "too many (view, tile) lists");
  }
  const int64_t n = (int64_t)3 * d.width * d.height;
  DevBuf k0, v0, k1, v1, hist, part;
  int bits = 1;
  while ((1ll << bits) - 1 < NT) ++bits;
  auto cleanup_fail = [&](int code, const std::string& m) {
    delete L;
    return fail(code, m);
  };
  if (k0.ensure(n * 4) || v0.ensure(n * 4) || k1.ensure(n * 4) || v1.ensure(n * 4))
    return cleanup_fail(DL_ENOMEM, "ray list buffers");
  const int64_t hs = radix_hist_size(n, 1);
  if (hist.ensure(hs * 4) || part.ensure((scan_partial_count(hs) + 2) * 4) || L->off.ensure((NT + 1) * 4))
    return cleanup_fail(DL_ENOMEM, "ray list buffers");
  hipError_t e = D->tgt.p ? launch_rays_emit_sr(D->V.as<uint8_t>(), D->tgt.as<int32_t>(), d.width, d.height, tw, th,
                                                L->ntx, L->T, k0.as<uint32_t>(), v0.as<uint32_t>(), s)
                          : launch_rays_emit(D->V.as<uint8_t>(), d.width, d.height, tw, th, L->ntx, L->T,
                                             k0.as<uint32_t>(), v0.as<uint32_t>(), s);
  if (e != hipSuccess) return cleanup_fail(DL_EHIP, hipGetErrorString(e));
  // each list's rays block by block (4 x 4 sub-blocks of the tile, row-major within a block), so that the blend's
  // 64-ray slots cover compact areas (more records that no ray of a slot accepts, and rays that end together)
  const int shift = bits + 4 <= 32 ? 4 : 0;
  if (shift) {
    e = launch_ray_key_blocks(k0.as<uint32_t>(), v0.as<uint32_t>(), n, tw, th, s);
    if (e != hipSuccess) return cleanup_fail(DL_EHIP, hipGetErrorString(e));
  }
  bool fl = radix_sort_u32(k0.as<uint32_t>(), v0.as<uint32_t>(), k1.as<uint32_t>(), v1.as<uint32_t>(), n, 1, nullptr,
                           0, 0, bits + shift, hist.as<uint32_t>(), part.as<uint32_t>(), s, &e);
  if (e != hipSuccess) return cleanup_fail(DL_EHIP, hipGetErrorString(e));
  uint32_t* sk = fl ? k1.as<uint32_t>() : k0.as<uint32_t>();
  DevBuf& sv = fl ? v1 : v0;
  e = launch_lower_bounds(sk, nullptr, 0, n, L->off.as<uint32_t>(), NT, s, shift);
  if (e != hipSuccess) return cleanup_fail(DL_EHIP, hipGetErrorString(e));
  std::vector<uint32_t> off(NT + 1);
  e = hipMemcpyAsync(off.data(), L->off.p, (NT + 1) * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup_fail(DL_EHIP, hipGetErrorString(e));
  L->n_rays = off[NT];
  int mx = 0;
  for (int64_t k = 0; k < NT; ++k) mx = std::max<int>(mx, (int)(off[k + 1] - off[k]));
  L->max_rays = mx;
  {
    uint32_t multi = 0;
    e = hipMemsetAsync(part.p, 0, 4, s);
    if (e == hipSuccess) e = launch_count_multichannel(sv.as<uint32_t>(), L->n_rays, part.as<uint32_t>(), s);
    if (e == hipSuccess) e = hipMemcpyAsync(&multi, part.p, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup_fail(DL_EHIP, hipGetErrorString(e));
    L->single_channel = multi == 0;
  }
  // keep the sorted entries (first n_rays values)
  std::swap(L->ent.p, sv.p);
  std::swap(L->ent.cap, sv.cap);
  D->lists[key] = L;
  *out = L;
  return DL_OK;
}

struct Tiles {
  int tw, th, ntx, nty, T;
};

Tiles make_tiles(const dl_display_desc& d, int tw, int th) {
  Tiles t;
  t.tw = tw;
  t.th = th;
  t.ntx = (d.width + tw - 1) / tw;
  t.nty = (d.height + th - 1) / th;
  t.T = t.ntx * t.nty;
  return t;
}

// Depth chunks (fractions of each view's visible depth ranks, in 1/1024): the front (about 1/32, chosen on a
// sampled histogram of the depth keys), the ranks up to 1/8, then the rest.  An eager frame skips the later
// chunks when no tile is live after the front (a plan whose probe frame finished there holds the front alone);
// when tiles stay live, the middle chunk gives them a second chance to saturate before the whole back is binned.
// A front too small for the scene's rays to saturate costs the sort of every live view's back (measured on 300k
// Gaussians at 3840x2160 N=45: 1/64 leaves tiles live, 3.6 ms per frame; 1/32 none, 1.91 ms; 1/16 1.99 ms; a
// front of 1/43 was 1% faster there but left tiles live at some poses of 500k Gaussians at 1920x1080 N=16 and
// 7680x4320 N=60, where 1/32 does not).
constexpr int kChunkDen = 1024;
constexpr int kChunkBounds[] = {0, 32, 128, 1024};
constexpr int kChunks = sizeof(kChunkBounds) / sizeof(kChunkBounds[0]) - 1;
constexpr uint32_t kMaxKeyCap = 0x7fffffffu;

int depth_key_e0(float z_near) {
  uint64_t b;
  const double z = (double)z_near;
  std::memcpy(&b, &z, 8);
  return (int)(b >> 52);
}

// Item slots per view of chunk c (a bound on its ranks): the first chunk is the view's front (at most all G
// ranks), the second runs from the front's end to a rank fraction, the others between two rank fractions of the
// visible Gaussians.
int64_t chunk_stride(int64_t G, int c) {
  if (c == 0) return G + 1;
  if (c == 1) return G * kChunkBounds[2] / kChunkDen + 1;  // starts at the front's end, which may be rank 0
  return G * (kChunkBounds[c + 1] - kChunkBounds[c]) / kChunkDen + 1;
}

// The first chunk uses the table form of binning (no tile partition) when a view has at most kTableMaxTiles
// tiles; its table holds one byte count per (view, tile, wavefront slot of kTableWaveRanks ranks), four to a
// word, at most kTableMaxEntries counts, so the first chunk of each view is capped at fcap ranks (the second
// chunk starts where it ended).  0: partition form.
constexpr int64_t kTableMaxEntries = 64ll << 20;
uint32_t table_fcap(int N, int64_t G, int64_t T) {
  if (T > kTableMaxTiles || N <= 0 || T <= 0) return 0;
  const int64_t waves = std::max<int64_t>(1, kTableMaxEntries / (T * N));
  return (uint32_t)std::min<int64_t>(std::max<int64_t>(G, 1), (int64_t)kTableWaveRanks * waves);
}
int64_t table_entries(int N, int64_t G, int64_t T) {
  const uint32_t f = table_fcap(N, G, T);
  return f ? T * N * (((int64_t)f + kTableGroup - 1) / kTableGroup) : 0;  // one word per workgroup slot
}

// Device bytes of every per-frame buffer, in the order render_frame ensures them.
constexpr int kFrameBufs = 26;
struct FrameSizes {
  size_t bytes[kFrameBufs];
  int64_t max_wstride;
  size_t total() const {
    size_t t = 0;
    for (size_t b : bytes) t += b;
    return t;
  }
};

FrameSizes frame_sizes(int N, int64_t G, int64_t NT, int64_t nstate, uint32_t cap, bool stats, bool bwd) {
  FrameSizes z{};
  const int64_t NG = (int64_t)N * G;
  int64_t max_stride = 0;
  for (int c = 0; c < kChunks; ++c) max_stride = std::max(max_stride, chunk_stride(G, c) + 64);
  z.max_wstride = (max_stride + 63) / 64;
  const int64_t tab = table_entries(N, G, N ? NT / N : 0);
  const int64_t ncounts = std::max<int64_t>((int64_t)N * z.max_wstride, 2 * tab + 1);
  const int64_t hs = std::max(std::max(std::max(radix_hist_size(G, N), depth_ranges_hist_size(G, N)),
                                        tile_partition_hist_size(N)),
                               split_hist_size(G, N));
  const size_t v[kFrameBufs] = {
      (size_t)N * kCamDoubles * 8,                    // cameras
      (size_t)G * kGaussBlockF4 * 16,                 // per-Gaussian blocks of the projection
      (size_t)NG * kRecF4 * 16,                       // records, depth order
      (size_t)NG * 8, (size_t)NG * 8,                 // depth keys (double-buffered)
      (size_t)NG * 4, (size_t)NG * 4,                 // Gaussian indices (double-buffered)
      256 * 4,                                        // visible counts
      (size_t)ncounts * 4,                            // per-wavefront key counts, or the first chunk's table, scanned
      (size_t)N * 4,                                  // live tiles per view
      (size_t)(3 * N + 2) * 4,                        // view key ranges and the partition layout
      (size_t)(8 * N + 2) * 4,                        // fronts, sort ranges, rank ends, sort layout, table layout
      (size_t)N * 8,                                  // front thresholds
      (size_t)front_hist_size(N) * 4,                 // front histogram
      (size_t)cap * 4, (size_t)cap * 4,               // tile keys (double-buffered)
      (size_t)cap * 4, (size_t)cap * 4,               // tile values (double-buffered)
      (size_t)(NT + 1) * 4,                           // list starts
      (size_t)NT,                                     // live tiles
      (size_t)std::max<int64_t>(nstate, 1) * 16,      // ray state
      3 * 8,                                          // key totals: chunk, largest, later chunk needed
      (size_t)hs * 4,                                 // radix histograms
      (size_t)(scan_partial_count(std::max<int64_t>(hs, ncounts)) + 2) * 4,  // scan partials
      stats ? (size_t)kStatSlots * 3 * 8 : 0,         // work counters
      bwd ? (size_t)NG * 9 * 4 : 0};                  // backward accumulators
  for (int b = 0; b < kFrameBufs; ++b) z.bytes[b] = v[b];
  return z;
}

// How a frame is issued: eager frames upload their cameras and end with the overflow check; a frame being
// captured into a graph does neither (the plan uploads the cameras before each launch and reads the overflow
// flag after completion).
struct FrameMode {
  bool upload = true;
  bool finish = true;
  bool keep_max = false;  // keep the largest chunk total of earlier frames (a plan's overflow status is sticky)
  // the first depth chunk only (a plan whose probe frame finished in it): a tile still live after it sets the
  // third key total, so that the caller learns the frame's image is incomplete
  bool first_only = false;
};

// Backward inputs/outputs of a frame (DirectL only).
struct BwdArgs {
  const float* fwd;   // forward encoded image
  const float* gout;  // d loss / d image
  float *g_means, *g_log_scales, *g_quats, *g_logits, *g_sh;
};

// One frame of either path: cameras, projection, depth sort, then per depth chunk: count live (view, tile)
// keys, scan, emit, partition by (view, tile), list bounds, blend.  Returns DL_ECAP (with *need set) if a
// chunk produced more keys than the capacity; the caller grows it and renders again.
int render_frame(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose, const dl_render_opts& o,
                 const Tiles& tl, bool standard, const RayLists* L, float* out, hipStream_t s,
                 unsigned long long* need, const BwdArgs* bwd, FrameMode mode = FrameMode()) {
  const dl_display_desc& d = D->desc;
  const int N = d.n_views;
  const int64_t G = S->n;
  if (mode.upload) {
    int rc = make_cameras(d, pose, C->cams_host);
    if (rc) return rc;
  }
  const int64_t NG = (int64_t)N * G;
  if (NG >= (1ll << 32) - 1) return fail(DL_EINVAL, "views x Gaussians exceeds 2^32");
  const int64_t NT = (int64_t)N * tl.T;
  if (NT >= (1ll << 31)) return fail(DL_EINVAL, "too many (view, tile) lists");
  if (C->key_cap == 0) C->key_cap = (uint32_t)std::min<int64_t>(kMaxKeyCap, std::max<int64_t>(1 << 22, 2 * NG));
  const uint32_t cap = C->key_cap;
  const int64_t nstate = standard ? (int64_t)N * d.width * d.height : L->n_rays;
  const FrameSizes z = frame_sizes(N, G, NT, nstate, cap, C->prof >= 3, bwd != nullptr);
  DevBuf* bufs[] = {&C->cams,   &C->rec,   &C->srec,  &C->k64[0], &C->k64[1], &C->v32[0], &C->v32[1],
                    &C->vis,    &C->counts, &C->live, &C->vstart, &C->dord,   &C->thr,    &C->fhist,
                    &C->bk[0],  &C->bk[1], &C->bv[0], &C->bv[1],  &C->tstart, &C->alive,  &C->state,
                    &C->dtotal, &C->hist,  &C->partial, &C->stats, &C->gacc};
  static_assert(sizeof(bufs) / sizeof(bufs[0]) == kFrameBufs, "one size per frame buffer");
  for (int b = 0; b < kFrameBufs; ++b)
    if (z.bytes[b]) HIP_TRY(bufs[b]->ensure(z.bytes[b]));
  if (bwd) HIP_TRY(hipMemsetAsync(C->gacc.p, 0, (size_t)NG * 9 * 4, s));

  C->frame_begin();
  int mk = C->begin(DL_STAGE_UPLOAD, s);
  if (C->prof >= 3) HIP_TRY(launch_fill_u64(C->stats.as<unsigned long long>(), kStatSlots * 3, 0ull, s));
  // an eager frame's cameras are built by the frame's first kernel from the pose (the host has validated the same
  // cameras above); a captured frame's are uploaded by its plan before every launch
  HIP_TRY(launch_frame_init(C->alive.as<uint8_t>(), standard ? nullptr : L->off.as<uint32_t>(), NT,
                            C->fhist.as<uint32_t>(), front_hist_size(N), C->dtotal.as<unsigned long long>(),
                            mode.keep_max ? 1 : 3, mode.upload ? make_rig(d, pose) : CamRig{},
                            mode.upload ? C->cams.as<double>() : nullptr, s));
  C->end(mk, s);

  ProjConst pc{};
  pc.G = G;
  pc.n_pad = S->n_pad;
  pc.N = N;
  pc.W = d.width;
  pc.H = d.height;
  pc.sh_degree = o.sh_degree;
  pc.focal = d.focal_px;
  pc.cx = d.width / 2.0;
  pc.cy = d.height / 2.0;
  pc.z_near = o.z_near;
  pc.q_cut = o.q_cut;
  pc.alpha_min = o.alpha_min;
  pc.alpha_max = o.alpha_max;
  pc.dilation = o.dilation;
  pc.key_e0 = depth_key_e0(o.z_near);
  mk = C->begin(DL_STAGE_PROJECT, s);
  HIP_TRY(launch_project_keys(S->soa.as<float>(), C->cams.as<double>(), pc, C->rec.as<float4>(),
                              C->k64[0].as<uint64_t>(), C->fhist.as<uint32_t>(), s));
  C->end(mk, s);
  hipError_t e;
  // Depth order.  The first chunk is each view's front (the nearest ~1/32 of its visible Gaussians, chosen on a
  // histogram of the keys' top bits).  Scenes of at most kFrontSortMaxG Gaussians: one pass gathers the fronts
  // (culled items dropped; each of its workgroups picks its view's threshold) and a few workgroups per view sort
  // its front in LDS, each a range of the keys' top bits; the backs are split off and sorted
  // after the first chunk, only for views that still have a live tile.  Larger scenes: one stable pass drops the
  // culled items and puts each front before its back, and device passes sort the fronts now and the live backs
  // later.  Every view's ranks end in one buffer.
  mk = C->begin(DL_STAGE_DEPTH_SORT, s);
  uint32_t* vis = C->vis.as<uint32_t>();
  uint32_t* front = C->dord.as<uint32_t>();
  uint32_t* rlo = front + N;
  uint32_t* rhi = rlo + N;
  uint32_t* rank_hi = rhi + N;
  uint32_t* dlayout = rank_hi + N;  // 2N + 1
  uint64_t* thr = C->thr.as<uint64_t>();
  bool fl = false;
  const bool lds_front = front_sort_fits(G, N);
  if (lds_front) {
    HIP_TRY(launch_front_gather(C->k64[0].as<uint64_t>(), C->k64[1].as<uint64_t>(), G, N, C->fhist.as<uint32_t>(),
                                kDepthKeyBits, kChunkBounds[1], kChunkDen, thr, kDepthCulled, C->hist.as<uint32_t>(),
                                s));
    HIP_TRY(launch_front_sort(C->k64[1].as<uint64_t>(), C->v32[1].as<uint32_t>(), G, N, C->hist.as<uint32_t>(),
                              C->fhist.as<uint32_t>(), thr, vis, front, rank_hi, s));
  } else {
    HIP_TRY(launch_front_select(N, kDepthKeyBits, kChunkBounds[1], kChunkDen, C->fhist.as<uint32_t>(), thr, s));
    radix_split_u64(C->k64[0].as<uint64_t>(), C->k64[1].as<uint64_t>(), C->v32[1].as<uint32_t>(), G, N, thr,
                    kDepthCulled, vis, front, C->hist.as<uint32_t>(), C->partial.as<uint32_t>(), s, &e);
    if (e != hipSuccess) return fail(DL_EHIP, std::string("depth split: ") + hipGetErrorString(e));
    HIP_TRY(launch_depth_ranges(N, G, vis, front, nullptr, rlo, rhi, rank_hi, dlayout, s));
    fl = depth_ranges_sort(C->k64[1].as<uint64_t>(), C->v32[1].as<uint32_t>(), C->k64[0].as<uint64_t>(),
                           C->v32[0].as<uint32_t>(), G, N, rlo, rhi, kDepthKeyBits, C->hist.as<uint32_t>(),
                           C->partial.as<uint32_t>(), dlayout, s, &e);
    if (e != hipSuccess) return fail(DL_EHIP, std::string("depth sort: ") + hipGetErrorString(e));
  }
  const uint32_t* sorted = fl ? C->v32[0].as<uint32_t>() : C->v32[1].as<uint32_t>();
  HIP_TRY(launch_project_ranks(C->rec.as<float4>(), C->cams.as<double>(), pc, sorted, nullptr, rank_hi,
                               lds_front ? kFrontSortCap : G, C->srec.as<float4>(), s));
  // the first chunk's end per view (the table form caps it) and the table layout
  const uint32_t fcap = table_fcap(N, G, tl.T);
  const int64_t tab_n = table_entries(N, G, tl.T);
  uint32_t* e0 = dlayout + 2 * N + 1;
  uint32_t* tbase = e0 + N;
  if (fcap) HIP_TRY(launch_table_setup(front, N, tl.T, fcap, e0, tbase, s));
  const uint32_t* chunk_front = fcap ? e0 : front;
  C->end(mk, s);

  BlendConst bc{};
  bc.W = d.width;
  bc.H = d.height;
  bc.tw = tl.tw;
  bc.th = tl.th;
  bc.ntx = tl.ntx;
  bc.nty = tl.nty;
  bc.T = tl.T;
  bc.N = N;
  bc.G = G;
  bc.q_cut = (float)(0.72134752044448170368 * (double)o.q_cut);  // log2(e)/2 scale of the record's conic
  bc.alpha_min = o.alpha_min;
  bc.alpha_max = o.alpha_max;
  bc.t_min = o.t_min;
  bc.log2_alpha_min = (float)std::log2((double)o.alpha_min);
  for (int k = 0; k < 3; ++k) bc.bg[k] = o.bg[k];
  bc.stats = C->prof >= 3 ? C->stats.as<unsigned long long>() : nullptr;
  bc.tgt = (!standard && D->tgt.p) ? D->tgt.as<int32_t>() : nullptr;
  bc.single_channel = (!standard && L && L->single_channel) ? 1 : 0;
  unsigned long long* total = C->dtotal.as<unsigned long long>();
  // an eager frame's first-chunk status words in host memory start at zero (the frame before has finished)
  if (mode.finish) C->frame_host[0] = C->frame_host[1] = 0;
  for (int c = 0; c < kChunks; ++c) {
    C->chunk = c;
    // after the first chunk an eager frame reads its key count and whether a tile is still live
    const bool readback = c == 0 && kChunks > 1 && mode.finish;
    ChunkArgs ch{};
    // the second chunk starts where the front ended, whatever fraction the front took
    ch.num_lo = c == 1 ? 0 : kChunkBounds[c];
    ch.num_hi = kChunkBounds[c + 1];
    ch.den = kChunkDen;
    ch.front = chunk_front;
    ch.first = c == 0;
    ch.stride = chunk_stride(G, c);
    ch.wstride = (ch.stride + 63) / 64;
    ch.cap = cap;
    // the first chunk's ranks per view: the LDS-sorted front (at most kFrontSortCap), within the table's cap
    ch.front_max = fcap ? (lds_front ? std::min<int64_t>(kFrontSortCap, fcap) : (int64_t)fcap) : 0;
    const int64_t ncount = (int64_t)N * ch.wstride;
    // views with no live tile left produce no keys in this chunk (the first chunk has every tile live)
    const uint32_t* live = c > 0 ? C->live.as<uint32_t>() : nullptr;
    const uint32_t* svals;
    if (c == 0 && fcap) {
      // table form: counts per (view, tile, wavefront), scan, ranks written into the final lists; the scanned
      // table follows the counts
      uint32_t* table = C->counts.as<uint32_t>();
      uint32_t* scanned = table + tab_n;
      mk = C->begin(DL_STAGE_BIN_COUNT, s);
      // every tile with rays is live in the first chunk (tiles without rays have empty blend work)
      HIP_TRY(launch_bin_table_count(C->srec.as<float4>(), C->vis.as<uint32_t>(), bc, ch, nullptr, tbase, table, s));
      C->end(mk, s);
      mk = C->begin(DL_STAGE_SCAN, s);
      HIP_TRY(exclusive_scan_u32(table, scanned, tab_n, C->partial.as<uint32_t>(), s, tbase + N, 1, true));
      C->end(mk, s);
      mk = C->begin(DL_STAGE_BIN_EMIT, s);
      HIP_TRY(launch_bin_table_emit(C->srec.as<float4>(), C->vis.as<uint32_t>(), bc, ch, nullptr, tbase, table,
                                    scanned, C->bv[0].as<uint32_t>(), s));
      C->end(mk, s);
      mk = C->begin(DL_STAGE_TILE_SORT, s);
      HIP_TRY(launch_table_starts(scanned, tbase, e0, N, tl.T, C->partial.as<uint32_t>() + scan_partial_count(tab_n),
                                  cap, total + 1, readback ? C->frame_dev : nullptr, C->tstart.as<uint32_t>(),
                                  s));
      C->end(mk, s);
      svals = C->bv[0].as<uint32_t>();
    } else {
      mk = C->begin(DL_STAGE_BIN_COUNT, s);
      HIP_TRY(launch_bin_count(C->srec.as<float4>(), C->vis.as<uint32_t>(), live, bc, ch, C->alive.as<uint8_t>(),
                               C->counts.as<uint32_t>(), total, s));
      C->end(mk, s);
      mk = C->begin(DL_STAGE_SCAN, s);
      HIP_TRY(exclusive_scan_u32(C->counts.as<uint32_t>(), C->counts.as<uint32_t>(), ncount, C->partial.as<uint32_t>(),
                                 s));
      C->end(mk, s);
      mk = C->begin(DL_STAGE_BIN_EMIT, s);
      HIP_TRY(launch_bin_emit(C->srec.as<float4>(), C->vis.as<uint32_t>(), live, bc, ch, C->alive.as<uint8_t>(),
                              C->counts.as<uint32_t>(), C->bk[0].as<uint32_t>(), C->bv[0].as<uint32_t>(), s));
      C->end(mk, s);
      mk = C->begin(DL_STAGE_TILE_SORT, s);
      HIP_TRY(launch_chunk_setup(C->counts.as<uint32_t>(), ch.wstride, N, total, total + 1, cap,
                                 C->vstart.as<uint32_t>(), C->vstart.as<uint32_t>() + (N + 1), s));
      svals = tile_partition(C->bk[0].as<uint32_t>(), C->bv[0].as<uint32_t>(), C->bk[1].as<uint32_t>(),
                             C->bv[1].as<uint32_t>(), N, C->vstart.as<uint32_t>(), cap, tl.T, C->hist.as<uint32_t>(),
                             C->partial.as<uint32_t>(), C->vstart.as<uint32_t>() + (N + 1), C->tstart.as<uint32_t>(),
                             s, &e);
      if (e != hipSuccess) return fail(DL_EHIP, std::string("tile partition: ") + hipGetErrorString(e));
      C->end(mk, s);
    }
    // the blend's workgroups raise the later-chunk flag: in host memory for an eager frame, as the status of a
    // first-chunk plan
    BlendChunk bk{c == 0, c == kChunks - 1,
                  readback ? C->frame_dev + 1 : (c == 0 && mode.first_only) ? total + 2 : nullptr};
    mk = C->begin(DL_STAGE_BLEND, s);
    if (bwd) {
      HIP_TRY(launch_blend_backward(C->srec.as<float4>(), C->tstart.as<uint32_t>(), svals, sorted,
                                    L->off.as<uint32_t>(), L->ent.as<uint32_t>(), L->max_rays, bc, bk,
                                    C->alive.as<uint8_t>(), C->state.as<float4>(), bwd->fwd, bwd->gout,
                                    C->gacc.as<float>(), s));
    } else if (standard) {
      HIP_TRY(launch_blend_standard(C->srec.as<float4>(), C->tstart.as<uint32_t>(), svals, bc, bk,
                                    C->alive.as<uint8_t>(), C->state.as<float4>(), out, s));
    } else {
      HIP_TRY(launch_blend_directl(C->srec.as<float4>(), C->tstart.as<uint32_t>(), svals, L->off.as<uint32_t>(),
                                   L->ent.as<uint32_t>(), L->max_rays, bc, bk, C->alive.as<uint8_t>(),
                                   C->state.as<float4>(), out, s));
    }
    // the live tiles per view for the next chunk (an eager frame counts them only once it knows a later chunk
    // runs; a first-chunk plan has none)
    if (c + 1 < kChunks && !readback && !mode.first_only)
      HIP_TRY(launch_view_live(C->alive.as<uint8_t>(), tl.T, N, C->live.as<uint32_t>(), total, s));
    C->end(mk, s);
    if (mode.first_only) break;
    if (readback) {
      // an eager frame (its caller waits for it anyway) reads whether a tile is still live after the first chunk:
      // when every tile's rays have terminated, every tile has written its pixels and the later chunks would only
      // launch empty kernels, so they are skipped (a captured frame keeps them: its launches are fixed).  It also
      // reads the first chunk's key count: a frame that skips the later chunks is complete here, and its overflow
      // check needs nothing more (a backward frame goes on to the projection's backward).  The blend and (table
      // form) the list-bounds kernel wrote both words into host memory; the partition form's count comes by copy,
      // and profiled frames copy the views' visible counts.
      volatile unsigned long long* rb = C->frame_host;
      uint32_t* vis_host = reinterpret_cast<uint32_t*>(C->frame_host + 2);
      if (!fcap) HIP_TRY(hipMemcpyAsync(C->frame_host, total + 1, 8, hipMemcpyDeviceToHost, s));
      if (C->prof) HIP_TRY(hipMemcpyAsync(vis_host, vis, (size_t)N * 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (rb[0] > cap) {
        // the first chunk overflowed: its blend saw truncated lists, so the live tiles (and the later chunks'
        // key counts) mean nothing; grow to what this chunk needs and render again
        *need = rb[0];
        return DL_ECAP;
      }
      C->later_ran = rb[1] != 0;
      if (!C->later_ran) {
        if (bwd) break;
        C->keys = (int64_t)rb[0];
        if (C->prof)
          for (int v = 0; v < N; ++v) C->visible += vis_host[v];
        return DL_OK;
      }
      HIP_TRY(launch_view_live(C->alive.as<uint8_t>(), tl.T, N, C->live.as<uint32_t>(), total, s));
    }
    if (c == 0 && kChunks > 1) {
      // the backs of the views that still have a live tile (split off the projection's keys first when only the
      // fronts were gathered)
      mk = C->begin(DL_STAGE_DEPTH_SORT, s);
      if (lds_front) {
        radix_split_u64(C->k64[0].as<uint64_t>(), C->k64[1].as<uint64_t>(), C->v32[1].as<uint32_t>(), G, N, thr,
                        kDepthCulled, vis, front, C->hist.as<uint32_t>(), C->partial.as<uint32_t>(), s, &e,
                        C->live.as<uint32_t>(), true);
        if (e != hipSuccess) return fail(DL_EHIP, std::string("depth split: ") + hipGetErrorString(e));
      }
      HIP_TRY(launch_depth_ranges(N, G, vis, front, C->live.as<uint32_t>(), rlo, rhi, rank_hi, dlayout, s));
      const bool fl2 = depth_ranges_sort(C->k64[1].as<uint64_t>(), C->v32[1].as<uint32_t>(), C->k64[0].as<uint64_t>(),
                                         C->v32[0].as<uint32_t>(), G, N, rlo, rhi, kDepthKeyBits,
                                         C->hist.as<uint32_t>(), C->partial.as<uint32_t>(), dlayout, s, &e);
      if (e != hipSuccess) return fail(DL_EHIP, std::string("depth sort: ") + hipGetErrorString(e));
      if (fl2 != fl) return fail(DL_EHIP, "depth sorts ended in different buffers");
      HIP_TRY(launch_project_ranks(C->rec.as<float4>(), C->cams.as<double>(), pc, sorted, front, rank_hi, G,
                                   C->srec.as<float4>(), s));
      C->end(mk, s);
    }
  }
  if (bwd) {
    mk = C->begin(DL_STAGE_PROJECT, s);
    HIP_TRY(launch_project_backward(S->soa.as<float>(), C->cams.as<double>(), pc, C->gacc.as<float>(), bwd->g_means,
                                    bwd->g_log_scales, bwd->g_quats, bwd->g_logits, bwd->g_sh, s));
    C->end(mk, s);
  }
  if (!mode.finish) return DL_OK;
  unsigned long long mx = 0;
  std::vector<uint32_t> vis_host(N, 0);
  HIP_TRY(hipMemcpyAsync(&mx, total + 1, 8, hipMemcpyDeviceToHost, s));
  if (C->prof) HIP_TRY(hipMemcpyAsync(vis_host.data(), C->vis.p, (size_t)N * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  C->keys = (int64_t)mx;
  for (int v = 0; v < N; ++v) C->visible += vis_host[v];
  if (mx > cap) {
    *need = mx;
    return DL_ECAP;
  }
  return DL_OK;
}

// Render with the context's key buffers, growing them once if a depth chunk overflowed.
int render_grow(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose, const dl_render_opts& o,
                const Tiles& tl, bool standard, const RayLists* L, float* out, hipStream_t s,
                const BwdArgs* bwd = nullptr) {
  for (int attempt = 0; attempt < 3; ++attempt) {
    unsigned long long need = 0;
    int rc = render_frame(C, S, D, pose, o, tl, standard, L, out, s, &need, bwd);
    if (rc != DL_ECAP) return rc;
    if (need > kMaxKeyCap) return fail(DL_ENOMEM, "a depth chunk needs more than 2^31 tile keys");
    const unsigned long long want = std::min<unsigned long long>(kMaxKeyCap, need + need / 4 + 1024);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
      const size_t have = C->bk[0].cap + C->bk[1].cap + C->bv[0].cap + C->bv[1].cap;
      if ((size_t)want * 16 > fr + have) return fail(DL_ENOMEM, "tile key buffers do not fit in device memory");
    }
    C->key_cap = (uint32_t)want;
  }
  return fail(DL_ECAP, "tile key capacity kept overflowing");
}

// Projection constants of a scene on a display under options o.
ProjConst proj_const(const dl_scene* S, const dl_display_desc& d, const dl_render_opts& o) {
  ProjConst pc{};
  pc.G = S->n;
  pc.n_pad = S->n_pad;
  pc.N = d.n_views;
  pc.W = d.width;
  pc.H = d.height;
  pc.sh_degree = o.sh_degree;
  pc.focal = d.focal_px;
  pc.cx = d.width / 2.0;
  pc.cy = d.height / 2.0;
  pc.z_near = o.z_near;
  pc.q_cut = o.q_cut;
  pc.alpha_min = o.alpha_min;
  pc.alpha_max = o.alpha_max;
  pc.dilation = o.dilation;
  pc.key_e0 = depth_key_e0(o.z_near);
  return pc;
}

int check_common(dl_ctx* C, const dl_scene* S, const dl_display* D) {
  if (!C || !S || !D) return fail(DL_EINVAL, "NULL context, scene or display");
  if (S->ctx->device != C->device || D->ctx->device != C->device)
    return fail(DL_EINVAL, "scene/display live on another device");
  return DL_OK;
}

}  // namespace

extern "C" {

void dl_default_opts(dl_render_opts* o) {
  if (!o) return;
  o->z_near = 0.2f;
  o->q_cut = 9.0f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
  o->dilation = 0.3f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
  o->sh_degree = 3;
  o->tile_w = 0;
  o->tile_h = 0;
}

const char* dl_last_error(void) { return g_err.c_str(); }

int dl_create(int device, dl_ctx** out) {
  if (!out) return fail(DL_EINVAL, "out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DL_EINVAL, "no such HIP device");
  HIP_TRY(hipSetDevice(device));
  int rc = scratch_setup(device);
  if (rc) return rc;
  dl_ctx* c = new dl_ctx();
  c->device = device;
  if (hipHostMalloc((void**)&c->cams_host, 256 * kCamDoubles * 8, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->frame_host, 2 * 8 + 256 * 4, hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&c->frame_dev, c->frame_host, 0) != hipSuccess) {
    if (c->cams_host) (void)hipHostFree(c->cams_host);
    if (c->frame_host) (void)hipHostFree(c->frame_host);
    delete c;
    return fail(DL_ENOMEM, "pinned camera staging");
  }
  *out = c;
  return DL_OK;
}

void dl_destroy(dl_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->cams_host) (void)hipHostFree(c->cams_host);
  if (c->frame_host) (void)hipHostFree(c->frame_host);
  delete c;
}

static int scene_fill(dl_scene* sc, const float* means, const float* log_scales, const float* quats,
                      const float* logits, const float* sh, int on_dev, hipStream_t s) {
  if (!means || !log_scales || !quats || !logits || !sh) return fail(DL_EINVAL, "NULL scene array");
  const int64_t n = sc->n, np = sc->n_pad;
  if (on_dev) {
    HIP_TRY(launch_scene_transpose(means, log_scales, quats, logits, sh, n, np, sc->soa.as<float>(), s));
    return DL_OK;
  }
  std::vector<float> h((size_t)kSceneRows * np, 0.0f);
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) h[(kRowMean + k) * np + i] = means[i * 3 + k];
    for (int k = 0; k < 3; ++k) h[(kRowLogScale + k) * np + i] = log_scales[i * 3 + k];
    for (int k = 0; k < 4; ++k) h[(kRowQuat + k) * np + i] = quats[i * 4 + k];
    h[kRowLogit * np + i] = logits[i];
    for (int k = 0; k < 48; ++k) h[(kRowSH + k) * np + i] = sh[i * 48 + k];
  }
  HIP_TRY(hipMemcpyAsync(sc->soa.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DL_OK;
}

int dl_scene_create(dl_ctx* ctx, int64_t n, const float* means, const float* log_scales, const float* quats,
                    const float* opacity_logits, const float* sh, int src_on_device, void* stream,
                    dl_scene** out) {
  if (!ctx || !out) return fail(DL_EINVAL, "NULL context or out");
  if (n < 1 || n >= (1ll << 31)) return fail(DL_EINVAL, "scene size must be in [1, 2^31)");
  dl_scene* sc = new dl_scene();
  sc->ctx = ctx;
  sc->n = n;
  sc->n_pad = (n + 63) / 64 * 64;
  if (sc->soa.ensure((size_t)kSceneRows * sc->n_pad * 4) != hipSuccess) {
    delete sc;
    return fail(DL_ENOMEM, "scene buffer");
  }
  int rc = scene_fill(sc, means, log_scales, quats, opacity_logits, sh, src_on_device, (hipStream_t)stream);
  if (rc) {
    delete sc;
    return rc;
  }
  *out = sc;
  return DL_OK;
}

int dl_scene_update(dl_scene* sc, const float* means, const float* log_scales, const float* quats,
                    const float* opacity_logits, const float* sh, int src_on_device, void* stream) {
  if (!sc) return fail(DL_EINVAL, "NULL scene");
  return scene_fill(sc, means, log_scales, quats, opacity_logits, sh, src_on_device, (hipStream_t)stream);
}

int64_t dl_scene_size(const dl_scene* sc) { return sc ? sc->n : -1; }

void dl_scene_free(dl_scene* sc) { delete sc; }

int dl_display_create(dl_ctx* ctx, const dl_display_desc* desc, void* stream, dl_display** out) {
  if (!ctx || !out) return fail(DL_EINVAL, "NULL context or out");
  dl_display_desc d;
  int rc = check_desc(desc, d);
  if (rc) return rc;
  // Q = b c p; As = b c q mod Q; Ax = 3 a c q mod Q; C = -r b q mod Q (floored)
  const __int128 a = d.tan_slant.num, b = d.tan_slant.den, p = d.pitch.num, q = d.pitch.den, r = d.offset.num,
                 c = d.offset.den;
  const __int128 Q = b * c * p;
  const __int128 lim = (__int128)1 << 62;
  // the device reduces each product modulo Q on its own when the direct sum would not fit (below 2^61 and with
  // row and column indices below 2^20, see view_map_kernel); N rho < N Q must fit as well
  if (Q <= 0 || Q >= ((__int128)1 << 61)) return fail(DL_ERANGE, "view map modulus b*c*p out of range");
  if (Q * d.n_views >= lim || 3 * (int64_t)d.width >= (1 << 20) || d.height >= (1 << 20))
    return fail(DL_ERANGE, "view map exceeds 64-bit exact arithmetic");
  const __int128 As = mod_floor(b * c * q, Q), Ax = mod_floor(3 * a * c * q, Q), Cc = mod_floor(-r * b * q, Q);
  const int wide = Q * (__int128)(3 * (int64_t)d.width + d.height + 1) >= lim ? 1 : 0;
  dl_display* D = new dl_display();
  D->ctx = ctx;
  D->desc = d;
  hipStream_t s = (hipStream_t)stream;
  const size_t nV = (size_t)3 * d.width * d.height;
  if (D->V.ensure(nV) != hipSuccess) {
    delete D;
    return fail(DL_ENOMEM, "view map buffer");
  }
  hipError_t e = launch_view_map(D->V.as<uint8_t>(), d.width, d.height, d.n_views, (int64_t)As, (int64_t)Ax,
                                 (int64_t)Cc, (int64_t)Q, wide, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete D;
    return fail(DL_EHIP, std::string("view map: ") + hipGetErrorString(e));
  }
  if (d.repurpose_pw > 0) {
    // subpixel repurposing (Alg. 2) on the host from the view map, then the rays' targets on the device
    const size_t nsub = nV;
    std::vector<uint8_t> Vh(nsub);
    std::vector<int32_t> srch(nsub);
    e = hipMemcpy(Vh.data(), D->V.p, nsub, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      delete D;
      return fail(DL_EHIP, std::string("view map copy: ") + hipGetErrorString(e));
    }
    std::string why;
    rc = repurpose_sources(d, d.repurpose_pw, Vh.data(), srch.data(), &why);
    if (rc) {
      delete D;
      return fail(rc, why);
    }
    DevBuf err;
    if (D->src.ensure(nsub * 4) || D->tgt.ensure(nsub * 3 * 4) || err.ensure(4)) {
      delete D;
      return fail(DL_ENOMEM, "repurposing buffers");
    }
    int32_t errh = 0;
    e = hipMemcpyAsync(D->src.p, srch.data(), nsub * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = launch_tgt_build(D->V.as<uint8_t>(), D->src.as<int32_t>(), d.width, d.height, D->tgt.as<int32_t>(),
                           err.as<int32_t>(), s);
    if (e == hipSuccess) e = hipMemcpyAsync(&errh, err.p, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || errh) {
      delete D;
      return fail(DL_EHIP, e != hipSuccess ? std::string("repurposing: ") + hipGetErrorString(e)
                                           : std::string("repurposing: a source pixel does not show its view"));
    }
  }
  // number of distinct rays via the ray lists of a 64x64 tiling (cached for later use)
  RayLists* L = nullptr;
  rc = build_ray_lists(D, 64, 64, s, &L);
  if (rc) {
    delete D;
    return rc;
  }
  D->n_rays = L->n_rays;
  *out = D;
  return DL_OK;
}

void dl_display_free(dl_display* D) { delete D; }

int dl_display_view_map(const dl_display* D, uint8_t* out_dev, void* stream) {
  if (!D || !out_dev) return fail(DL_EINVAL, "NULL display or output");
  const size_t n = (size_t)3 * D->desc.width * D->desc.height;
  HIP_TRY(hipMemcpyAsync(out_dev, D->V.p, n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return DL_OK;
}

int64_t dl_display_num_rays(const dl_display* D) { return D ? D->n_rays : -1; }

int dl_display_source_map(const dl_display* D, int32_t* out_dev, void* stream) {
  if (!D || !out_dev) return fail(DL_EINVAL, "NULL display or output");
  const size_t n = (size_t)3 * D->desc.width * D->desc.height;
  if (D->src.p)
    HIP_TRY(hipMemcpyAsync(out_dev, D->src.p, n * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  else
    HIP_TRY(launch_own_pixel(out_dev, D->desc.width, D->desc.height, (hipStream_t)stream));
  return DL_OK;
}

int dl_cameras(const dl_display* D, const dl_pose* pose, double* out_host) {
  if (!D || !out_host) return fail(DL_EINVAL, "NULL display or output");
  return make_cameras(D->desc, pose, out_host);
}

int dl_project(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose, const dl_render_opts* opts,
               float* out_dev, double* depth_dev, void* stream) {
  int rc = check_common(C, S, D);
  if (rc) return rc;
  if (!out_dev || !depth_dev) return fail(DL_EINVAL, "NULL output");
  dl_render_opts o;
  if ((rc = check_opts(opts, o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const dl_display_desc& d = D->desc;
  const int N = d.n_views;
  const int64_t NG = (int64_t)N * S->n;
  if ((rc = make_cameras(d, pose, C->cams_host))) return rc;
  HIP_TRY(C->cams.ensure((size_t)N * kCamDoubles * 8));
  HIP_TRY(C->k64[0].ensure((size_t)NG * 8));
  HIP_TRY(C->v32[0].ensure((size_t)NG * 4));
  HIP_TRY(C->vis.ensure(256 * 4));
  HIP_TRY(hipMemcpyAsync(C->cams.p, C->cams_host, (size_t)N * kCamDoubles * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(C->vis.p, 0, 256 * 4, s));
  HIP_TRY(hipMemsetAsync(out_dev, 0, (size_t)NG * 48, s));
  const ProjConst pc = proj_const(S, d, o);
  HIP_TRY(launch_project(S->soa.as<float>(), C->cams.as<double>(), pc, (float4*)out_dev, C->k64[0].as<uint64_t>(),
                         C->v32[0].as<uint32_t>(), depth_dev, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DL_OK;
}

int dl_project_noalloc(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose,
                       const dl_render_opts* opts, float* out_dev, double* depth_dev, void* stream) {
  int rc = check_common(C, S, D);
  if (rc) return rc;
  if (!out_dev || !depth_dev) return fail(DL_EINVAL, "NULL output");
  dl_render_opts o;
  if ((rc = check_opts(opts, o))) return rc;
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != C->device) return fail(DL_EINVAL, "the context's device is not the current device");
  const dl_display_desc& d = D->desc;
  const int N = d.n_views;
  const int64_t NG = (int64_t)N * S->n;
  // scratch layout: the N cameras, then the N x G depth keys the projection kernel writes (read by nobody here)
  const size_t cam_bytes = ((size_t)N * kCamDoubles * 8 + 255) / 256 * 256;
  const unsigned long long need = (unsigned long long)cam_bytes + (unsigned long long)NG * 8ull;
  if (need > (unsigned long long)DL_NOALLOC_SCRATCH_BYTES)
    return fail(DL_ERANGE, "projection of " + std::to_string(NG) + " (view, Gaussian) pairs needs " +
                               std::to_string(need) + " bytes of scratch, more than the fixed " +
                               std::to_string((long long)DL_NOALLOC_SCRATCH_BYTES));
  unsigned char* base = static_cast<unsigned char*>(scratch_of(C->device));
  if (!base) return fail(DL_EHIP, "no scratch address for this device");
  if ((rc = make_cameras(d, pose, C->cams_host))) return rc;
  hipStream_t s = (hipStream_t)stream;
  double* cams = reinterpret_cast<double*>(base);
  uint64_t* keys = reinterpret_cast<uint64_t*>(base + cam_bytes);
  HIP_TRY(hipMemcpyAsync(cams, C->cams_host, (size_t)N * kCamDoubles * 8, hipMemcpyHostToDevice, s));
  const ProjConst pc = proj_const(S, d, o);
  // every (view, Gaussian) record and depth is written by the kernel (culled records as zeros): nothing to clear
  HIP_TRY(launch_project(S->soa.as<float>(), cams, pc, (float4*)out_dev, keys, nullptr, depth_dev, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DL_OK;
}

int dl_render(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose, const dl_render_opts* opts,
              float* out_dev, void* stream) {
  int rc = check_common(C, S, D);
  if (rc) return rc;
  if (!out_dev) return fail(DL_EINVAL, "NULL output");
  dl_render_opts o;
  if ((rc = check_opts(opts, o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int tw = o.tile_w, th = o.tile_h;
  if (tw == 0 || th == 0) auto_tile_directl(D->desc, D->n_rays, tw, th);
  RayLists* L = nullptr;
  if ((rc = build_ray_lists(const_cast<dl_display*>(D), tw, th, s, &L))) return rc;
  if (L->max_rays > 16 * 256) return fail(DL_EINVAL, "tile too large: more than 4096 rays of one view");
  Tiles tl = make_tiles(D->desc, tw, th);
  C->tile_w = tw;
  C->tile_h = th;
  C->rpt = L->max_rays <= 1024 ? (L->max_rays + 255) / 256 : (L->max_rays + 511) / 512;
  C->lanes = L->max_rays <= 1024 ? 256 : 512;
  return render_grow(C, S, D, pose, o, tl, false, L, out_dev, s);
}

int dl_render_multiview(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose,
                        const dl_render_opts* opts, int32_t view_w, int32_t view_h, float* out_dev, float* views_dev,
                        void* stream) {
  int rc = check_common(C, S, D);
  if (rc) return rc;
  if (!out_dev) return fail(DL_EINVAL, "NULL output");
  if (view_w < 1 || view_h < 1 || view_w > 65536 || view_h > 65536) return fail(DL_EINVAL, "view size out of range");
  dl_render_opts o;
  if ((rc = check_opts(opts, o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int tw = o.tile_w ? o.tile_w : 32, th = o.tile_h ? o.tile_h : 32;
  if (tw * th > 16 * 256) return fail(DL_EINVAL, "standard tile larger than 4096 pixels");
  const dl_display_desc& d = D->desc;
  // the views: the same rig and vertical field of view at view_w x view_h pixels
  dl_display Dv;
  Dv.ctx = D->ctx;
  Dv.desc = d;
  Dv.desc.width = view_w;
  Dv.desc.height = view_h;
  Dv.desc.focal_px = d.focal_px * (double)view_h / (double)d.height;
  float* views = views_dev;
  if (!views) {
    HIP_TRY(C->views.ensure((size_t)d.n_views * view_w * view_h * 12));
    views = C->views.as<float>();
  }
  Tiles tl = make_tiles(Dv.desc, tw, th);
  C->tile_w = tw;
  C->tile_h = th;
  C->rpt = tw * th <= 1024 ? (tw * th + 255) / 256 : (tw * th + 511) / 512;
  C->lanes = tw * th <= 1024 ? 256 : 512;
  if ((rc = render_grow(C, S, &Dv, pose, o, tl, true, nullptr, views, s))) return rc;
  int mk = C->begin(DL_STAGE_INTERLEAVE, s);
  HIP_TRY(launch_interleave_resize(D->V.as<uint8_t>(), D->src.p ? D->src.as<int32_t>() : nullptr, views, out_dev,
                                   d.width, d.height, view_w, view_h, s));
  C->end(mk, s);
  return DL_OK;
}

}  // extern "C"

struct dl_plan {
  dl_ctx* C = nullptr;  // private frame buffers
  const dl_scene* S = nullptr;
  const dl_display* D = nullptr;
  dl_render_opts o{};
  Tiles tl{};
  RayLists* L = nullptr;
  float* out = nullptr;  // caller's [H][W][3] image
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t copied = nullptr;                // after the last camera upload: the staging may be rewritten
  hipEvent_t done = nullptr;                  // after the last launch's status copy
  // pinned: largest chunk key total of the plan's frames so far, and whether one of them needed a later chunk
  unsigned long long* status_host = nullptr;
  bool first_only = false;  // the graphs hold the first depth chunk only (the probe frame finished in it)
  // batched launches: graphs of 1..batch_max frames in a row, frame k reading camera set k of batch_cams and
  // writing batch_out[k]; the camera sets of a launch are uploaded together from pinned staging
  int batch_max = 0;
  std::vector<float*> batch_out;
  std::vector<hipGraph_t> batch_graph;
  std::vector<hipGraphExec_t> batch_exec;
  DevBuf batch_cams;
  double* batch_cams_host = nullptr;
  ~dl_plan() {
    if (copied) {
      (void)hipEventSynchronize(copied);
      (void)hipEventDestroy(copied);
    }
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    for (hipGraphExec_t x : batch_exec) (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : batch_graph) (void)hipGraphDestroy(g);
    if (batch_cams_host) (void)hipHostFree(batch_cams_host);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (status_host) (void)hipHostFree(status_host);
    dl_destroy(C);
  }
};

namespace {
size_t ctx_bytes(const dl_ctx* C) {
  const DevBuf* b[] = {&C->cams, &C->rec, &C->srec, &C->k64[0], &C->k64[1], &C->v32[0], &C->v32[1], &C->vis,
                       &C->counts, &C->bk[0], &C->bk[1], &C->bv[0], &C->bv[1], &C->hist, &C->partial, &C->tstart,
                       &C->views, &C->stats, &C->alive, &C->state, &C->dtotal, &C->gacc, &C->live, &C->vstart, &C->dord, &C->thr, &C->fhist};
  size_t t = 0;
  for (const DevBuf* x : b) t += x->cap;
  return t;
}
// Record one frame of the plan into a graph (cameras are uploaded outside it, before every launch).
int plan_capture(dl_plan* P, hipStream_t s) {
  unsigned long long need = 0;
  FrameMode m;
  m.upload = false;
  m.finish = false;
  m.keep_max = true;
  m.first_only = P->first_only;
  HIP_TRY(launch_fill_u64(P->C->dtotal.as<unsigned long long>(), 3, 0ull, s));  // status of the plan's frames
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = render_frame(P->C, P->S, P->D, nullptr, P->o, P->tl, false, P->L, P->out, s, &need, nullptr, m);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(DL_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  P->graph = g;
  HIP_TRY(hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0));
  return DL_OK;
}

// Record n frames of the plan in a row into one graph: frame k copies camera set k into the frame's camera buffer
// (a device-to-device copy node), then runs the captured frame into batch_out[k].
int plan_capture_batch(dl_plan* P, int n, hipStream_t s, hipGraph_t* graph, hipGraphExec_t* exec) {
  unsigned long long need = 0;
  FrameMode m;
  m.upload = false;
  m.finish = false;
  m.keep_max = true;
  m.first_only = P->first_only;
  const size_t cam_bytes = (size_t)P->D->desc.n_views * kCamDoubles * 8;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = DL_OK;
  hipError_t ce = hipSuccess;
  for (int k = 0; k < n && rc == DL_OK && ce == hipSuccess; ++k) {
    ce = hipMemcpyAsync(P->C->cams.p, static_cast<char*>(P->batch_cams.p) + k * cam_bytes, cam_bytes,
                        hipMemcpyDeviceToDevice, s);
    if (ce == hipSuccess)
      rc = render_frame(P->C, P->S, P->D, nullptr, P->o, P->tl, false, P->L, P->batch_out[k], s, &need, nullptr, m);
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : fail(DL_EHIP, std::string("batch camera copy: ") + hipGetErrorString(ce));
  }
  if (e != hipSuccess) return fail(DL_EHIP, std::string("batch graph capture: ") + hipGetErrorString(e));
  *graph = g;
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) return fail(DL_EHIP, std::string("batch graph instantiate: ") + hipGetErrorString(e));
  return DL_OK;
}
}  // namespace

extern "C" {

int dl_plan_create(dl_ctx* ctx, const dl_scene* S, const dl_display* D, const dl_render_opts* opts,
                   const dl_pose* probe_pose, int64_t min_key_capacity, float* out_dev, void* stream,
                   dl_plan** out) {
  int rc = check_common(ctx, S, D);
  if (rc) return rc;
  if (!out || !probe_pose || !out_dev) return fail(DL_EINVAL, "NULL argument");
  if (min_key_capacity < 0 || min_key_capacity > (int64_t)kMaxKeyCap) return fail(DL_EINVAL, "key capacity range");
  dl_render_opts o;
  if ((rc = check_opts(opts, o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(DL_EINVAL, "plans are captured on a created stream, not the null stream");
  dl_plan* P = new dl_plan();
  if ((rc = dl_create(ctx->device, &P->C))) {
    delete P;
    return rc;
  }
  P->S = S;
  P->D = D;
  P->o = o;
  P->out = out_dev;
  int tw = o.tile_w, th = o.tile_h;
  if (tw == 0 || th == 0) auto_tile_directl(D->desc, D->n_rays, tw, th);
  P->tl = make_tiles(D->desc, tw, th);
  // first guess of the per-chunk key capacity; the probe grows it to what the pose needs
  P->C->key_cap = (uint32_t)std::min<int64_t>(1 << 22, std::max<int64_t>(1 << 16, (int64_t)D->desc.n_views * S->n / 2));
  if ((rc = build_ray_lists(const_cast<dl_display*>(D), tw, th, s, &P->L))) {
    delete P;
    return rc;
  }
  if (P->L->max_rays > 16 * 256) {
    delete P;
    return fail(DL_EINVAL, "tile too large: more than 4096 rays of one view");
  }
  if (hipHostMalloc((void**)&P->status_host, 16, hipHostMallocDefault) != hipSuccess) {
    delete P;
    return fail(DL_ENOMEM, "plan status word");
  }
  // size every buffer with an eager frame at the probe pose, then refit the key buffers to the largest chunk
  // total seen plus 30% headroom (buffers are grow-only, so release those that depend on the capacity)
  if ((rc = render_grow(P->C, S, D, probe_pose, o, P->tl, false, P->L, P->out, s))) {
    delete P;
    return rc;
  }
  const unsigned long long k = (unsigned long long)P->C->keys;
  P->C->key_cap = (uint32_t)std::min<unsigned long long>(
      kMaxKeyCap, std::max<unsigned long long>((unsigned long long)min_key_capacity, k + k * 3 / 10 + 4096));
  for (DevBuf* b : {&P->C->bk[0], &P->C->bk[1], &P->C->bv[0], &P->C->bv[1], &P->C->hist, &P->C->partial})
    b->release();
  if ((rc = render_grow(P->C, S, D, probe_pose, o, P->tl, false, P->L, P->out, s))) {
    delete P;
    return rc;
  }
  if (hipEventCreateWithFlags(&P->copied, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->done, hipEventDisableTiming) != hipSuccess) {
    delete P;
    return fail(DL_EHIP, "plan event");
  }
  // a probe frame that finished in its first depth chunk gives a plan of that chunk alone
  P->first_only = kChunks > 1 && !P->C->later_ran;
  if ((rc = plan_capture(P, s))) {
    delete P;
    return rc;
  }
  P->status_host[0] = P->status_host[1] = 0;
  *out = P;
  return DL_OK;
}

int64_t dl_plan_bytes(const dl_plan* P) { return P ? (int64_t)ctx_bytes(P->C) : -1; }

int64_t dl_plan_estimate_bytes(const dl_scene* S, const dl_display* D, const dl_render_opts* opts,
                               int64_t key_capacity) {
  if (!S || !D || key_capacity < 0) return -1;
  dl_render_opts o;
  if (check_opts(opts, o)) return -1;
  int tw = o.tile_w, th = o.tile_h;
  if (tw == 0 || th == 0) auto_tile_directl(D->desc, D->n_rays, tw, th);
  const Tiles tl = make_tiles(D->desc, tw, th);
  const int N = D->desc.n_views;
  const uint32_t cap = (uint32_t)std::min<int64_t>(kMaxKeyCap, std::max<int64_t>(key_capacity, 1));
  return (int64_t)frame_sizes(N, S->n, (int64_t)N * tl.T, D->n_rays, cap, false, false).total();
}

int dl_plan_render(dl_plan* P, const dl_pose* pose, void* stream) {
  if (!P) return fail(DL_EINVAL, "NULL plan");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(DL_EINVAL, "plans are launched on a created stream, not the null stream");
  dl_ctx* C = P->C;
  const int N = P->D->desc.n_views;
  HIP_TRY(hipEventSynchronize(P->copied));  // the previous launch's upload has left the staging buffer
  int rc = make_cameras(P->D->desc, pose, C->cams_host);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(C->cams.p, C->cams_host, (size_t)N * kCamDoubles * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(P->copied, s));
  HIP_TRY(hipGraphLaunch(P->exec, s));
  HIP_TRY(hipMemcpyAsync(P->status_host, C->dtotal.as<unsigned long long>() + 1, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(P->done, s));
  return DL_OK;
}

int dl_plan_check(const dl_plan* P, int64_t* need) {
  if (!P) return fail(DL_EINVAL, "NULL plan");
  const unsigned long long mx = P->status_host[0];
  if (need) *need = (int64_t)mx;
  if (mx > P->C->key_cap) return fail(DL_ECAP, "a depth chunk overflowed the plan's key capacity");
  if (P->status_host[1]) return fail(DL_ELATER, "a frame of a first-chunk plan needed a later depth chunk");
  return DL_OK;
}

int dl_plan_first_chunk_only(const dl_plan* P) { return P ? (P->first_only ? 1 : 0) : DL_EINVAL; }

int dl_plan_use_all_chunks(dl_plan* P, void* stream) {
  if (!P) return fail(DL_EINVAL, "NULL plan");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(DL_EINVAL, "plans are captured on a created stream, not the null stream");
  if (!P->first_only) return DL_OK;
  // the plan's graphs are replaced once its last launch has completed
  HIP_TRY(hipEventSynchronize(P->done));
  P->first_only = false;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->exec = nullptr;
  P->graph = nullptr;
  int rc = plan_capture(P, s);
  if (rc) return rc;
  for (int n = 1; n <= P->batch_max; ++n) {
    (void)hipGraphExecDestroy(P->batch_exec[n - 1]);
    (void)hipGraphDestroy(P->batch_graph[n - 1]);
    P->batch_exec[n - 1] = nullptr;
    P->batch_graph[n - 1] = nullptr;
    if ((rc = plan_capture_batch(P, n, s, &P->batch_graph[n - 1], &P->batch_exec[n - 1]))) return rc;
  }
  HIP_TRY(hipStreamSynchronize(s));  // the status reset of the capture has run
  P->status_host[0] = P->status_host[1] = 0;
  return DL_OK;
}

int dl_plan_batch_prepare(dl_plan* P, int32_t max_frames, float* const* outs_dev, void* stream) {
  if (!P || !outs_dev) return fail(DL_EINVAL, "NULL plan or outputs");
  if (P->batch_max) return fail(DL_EINVAL, "the plan's batched launches are already prepared");
  if (max_frames < 1 || max_frames > DL_MAX_BATCH) return fail(DL_EINVAL, "max_frames must be in [1, DL_MAX_BATCH]");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(DL_EINVAL, "plans are captured on a created stream, not the null stream");
  for (int k = 0; k < max_frames; ++k)
    if (!outs_dev[k]) return fail(DL_EINVAL, "NULL output image");
  const size_t cam_bytes = (size_t)P->D->desc.n_views * kCamDoubles * 8;
  HIP_TRY(P->batch_cams.ensure(cam_bytes * max_frames));
  if (hipHostMalloc((void**)&P->batch_cams_host, cam_bytes * max_frames, hipHostMallocDefault) != hipSuccess) {
    P->batch_cams_host = nullptr;
    return fail(DL_ENOMEM, "pinned batch camera staging");
  }
  P->batch_out.assign(outs_dev, outs_dev + max_frames);
  P->batch_graph.assign(max_frames, nullptr);
  P->batch_exec.assign(max_frames, nullptr);
  for (int n = 1; n <= max_frames; ++n) {
    int rc = plan_capture_batch(P, n, s, &P->batch_graph[n - 1], &P->batch_exec[n - 1]);
    if (rc) return rc;
  }
  P->batch_max = max_frames;
  return DL_OK;
}

int dl_plan_render_batch(dl_plan* P, const dl_pose* poses, int32_t n, void* stream) {
  if (!P || !poses) return fail(DL_EINVAL, "NULL plan or poses");
  if (!P->batch_max) return fail(DL_EINVAL, "batched launches not prepared (dl_plan_batch_prepare)");
  if (n < 1 || n > P->batch_max) return fail(DL_EINVAL, "n must be in [1, the prepared max_frames]");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(DL_EINVAL, "plans are launched on a created stream, not the null stream");
  const int N = P->D->desc.n_views;
  const size_t cam_doubles = (size_t)N * kCamDoubles;
  HIP_TRY(hipEventSynchronize(P->copied));  // the previous launch's upload has left the staging buffers
  for (int k = 0; k < n; ++k) {
    int rc = make_cameras(P->D->desc, &poses[k], P->batch_cams_host + k * cam_doubles);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpyAsync(P->batch_cams.p, P->batch_cams_host, n * cam_doubles * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(P->copied, s));
  HIP_TRY(hipGraphLaunch(P->batch_exec[n - 1], s));
  HIP_TRY(hipMemcpyAsync(P->status_host, P->C->dtotal.as<unsigned long long>() + 1, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(P->done, s));
  return DL_OK;
}

void dl_plan_free(dl_plan* P) { delete P; }

int dl_set_key_capacity(dl_ctx* C, int64_t keys) {
  if (!C) return fail(DL_EINVAL, "NULL context");
  if (keys < 1 || keys > (int64_t)kMaxKeyCap) return fail(DL_EINVAL, "key capacity must be in [1, 2^31)");
  C->key_cap = (uint32_t)keys;
  return DL_OK;
}

int64_t dl_key_capacity(const dl_ctx* C) { return C ? (int64_t)C->key_cap : -1; }

int dl_probe_issue_rates(int device, double* out, int n_out) {
  if (!out || n_out < 1) return fail(DL_EINVAL, "out is NULL or n_out < 1");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DL_EINVAL, "no such device");
  HIP_TRY(hipSetDevice(device));
  std::string why;
  const int rc = probe_issue_rates(out, n_out, &why);
  if (rc != DL_OK) return fail(rc, why);
  return DL_OK;
}

int dl_set_profiling(dl_ctx* C, int level) {
  if (!C) return fail(DL_EINVAL, "NULL context");
  if (level < 0 || level > 3) return fail(DL_EINVAL, "profiling level is 0, 1, 2 or 3");
  C->prof = level;
  return DL_OK;
}

int dl_frame_stats_get(dl_ctx* C, dl_frame_stats* out) {
  if (!C || !out) return fail(DL_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  if (!C->prof) return fail(DL_EINVAL, "profiling is off");
  for (const auto& m : C->marks) {
    HIP_TRY(hipEventSynchronize(m.b));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, m.a, m.b));
    if (m.stage >= 0 && m.stage < DL_NSTAGES) {
      out->stage_ms[m.stage] += ms;
      out->stage_launches[m.stage] += 1;
      if (m.chunk >= 0 && m.chunk < DL_MAX_CHUNKS) out->chunk_ms[m.chunk][m.stage] += ms;
    }
  }
  unsigned long long st[3] = {0, 0, 0};
  if (C->prof >= 3 && C->stats.p) {
    std::vector<unsigned long long> sl((size_t)kStatSlots * 3);
    HIP_TRY(hipMemcpy(sl.data(), C->stats.p, sl.size() * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < kStatSlots; ++i)
      for (int k = 0; k < 3; ++k) st[k] += sl[(size_t)i * 3 + k];
  }
  out->chunks = kChunks;
  out->keys = C->keys;
  out->visible = C->visible;
  out->evaluations = (int64_t)st[0];
  out->blends = (int64_t)st[1];
  out->rays = (int64_t)st[2];
  out->batches = C->batches;
  out->tile_w = C->tile_w;
  out->tile_h = C->tile_h;
  out->rays_per_lane = C->rpt;
  out->lanes = C->lanes;
  return DL_OK;
}

int dl_render_backward(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose,
                       const dl_render_opts* opts, const float* out_dev, const float* grad_out_dev, float* g_means,
                       float* g_log_scales, float* g_quats, float* g_opacity_logits, float* g_sh, void* stream) {
  int rc = check_common(C, S, D);
  if (rc) return rc;
  if (!out_dev || !grad_out_dev || !g_means || !g_log_scales || !g_quats || !g_opacity_logits || !g_sh)
    return fail(DL_EINVAL, "NULL buffer");
  dl_render_opts o;
  if ((rc = check_opts(opts, o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int tw = o.tile_w, th = o.tile_h;
  if (tw == 0 || th == 0) auto_tile_directl(D->desc, D->n_rays, tw, th);
  RayLists* L = nullptr;
  if ((rc = build_ray_lists(const_cast<dl_display*>(D), tw, th, s, &L))) return rc;
  if (L->max_rays > 16 * 256) return fail(DL_EINVAL, "tile too large: more than 4096 rays of one view");
  Tiles tl = make_tiles(D->desc, tw, th);
  C->tile_w = tw;
  C->tile_h = th;
  C->rpt = L->max_rays <= 1024 ? (L->max_rays + 255) / 256 : (L->max_rays + 511) / 512;
  C->lanes = L->max_rays <= 1024 ? 256 : 512;
  BwdArgs b{out_dev, grad_out_dev, g_means, g_log_scales, g_quats, g_opacity_logits, g_sh};
  return render_grow(C, S, D, pose, o, tl, false, L, nullptr, s, &b);
}

int dl_interleave(const dl_display* D, const float* views_dev, float* out_dev, void* stream) {
  if (!D || !views_dev || !out_dev) return fail(DL_EINVAL, "NULL argument");
  if (D->src.p)
    HIP_TRY(launch_interleave_sr(D->V.as<uint8_t>(), D->src.as<int32_t>(), views_dev, out_dev, D->desc.width,
                                 D->desc.height, (hipStream_t)stream));
  else
    HIP_TRY(launch_interleave(D->V.as<uint8_t>(), views_dev, out_dev, D->desc.width, D->desc.height,
                              (hipStream_t)stream));
  return DL_OK;
}

int dl_render_standard(dl_ctx* C, const dl_scene* S, const dl_display* D, const dl_pose* pose,
                       const dl_render_opts* opts, float* out_dev, float* views_dev, void* stream) {
  int rc = check_common(C, S, D);
  if (rc) return rc;
  if (!out_dev) return fail(DL_EINVAL, "NULL output");
  dl_render_opts o;
  if ((rc = check_opts(opts, o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int tw = o.tile_w ? o.tile_w : 32, th = o.tile_h ? o.tile_h : 32;
  if (tw * th > 16 * 256) return fail(DL_EINVAL, "standard tile larger than 4096 pixels");
  const dl_display_desc& d = D->desc;
  float* views = views_dev;
  if (!views) {
    HIP_TRY(C->views.ensure((size_t)d.n_views * d.width * d.height * 12));
    views = C->views.as<float>();
  }
  Tiles tl = make_tiles(d, tw, th);
  C->tile_w = tw;
  C->tile_h = th;
  C->rpt = tw * th <= 1024 ? (tw * th + 255) / 256 : (tw * th + 511) / 512;
  C->lanes = tw * th <= 1024 ? 256 : 512;
  if ((rc = render_grow(C, S, D, pose, o, tl, true, nullptr, views, s))) return rc;
  int mk = C->begin(DL_STAGE_INTERLEAVE, s);
  if (D->src.p)
    HIP_TRY(launch_interleave_sr(D->V.as<uint8_t>(), D->src.as<int32_t>(), views, out_dev, d.width, d.height, s));
  else
    HIP_TRY(launch_interleave(D->V.as<uint8_t>(), views, out_dev, d.width, d.height, s));
  C->end(mk, s);
  return DL_OK;
}

int dl_bvh_build(dl_ctx* C, const dl_scene* S, const dl_render_opts* opts, void* stream, dl_bvh** out) {
  if (!C || !S || !out) return fail(DL_EINVAL, "NULL context, scene or out");
  if (S->ctx->device != C->device) return fail(DL_EINVAL, "scene lives on another device");
  dl_render_opts o;
  int rc = check_opts(opts, o);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t np = S->n_pad;
  std::vector<float> h((size_t)kSceneRows * np);
  HIP_TRY(hipMemcpyAsync(h.data(), S->soa.p, h.size() * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  BvhHost bh;
  std::string why;
  if ((rc = bvh_build_host(h.data(), S->n, np, o.q_cut, o.alpha_min, &bh, &why))) return fail(rc, why);
  if (bh.stack_bound > kBvhStackMax) return fail(DL_ERANGE, "BVH needs a traversal stack deeper than 256");
  const int64_t m = bh.n_prims;
  std::vector<float> sh((size_t)m * 48);
  for (int64_t r = 0; r < m; ++r)
    for (int c = 0; c < 3; ++c)
      for (int l = 0; l < 16; ++l) sh[((size_t)r * 3 + c) * 16 + l] = h[(size_t)(kRowSH + 3 * l + c) * np + bh.perm[r]];
  dl_bvh* B = new dl_bvh();
  B->ctx = C;
  if (B->nodes.ensure(bh.nodes.size() * 4) || B->rec.ensure(bh.rec.size() * 4) || B->sh.ensure(sh.size() * 4)) {
    delete B;
    return fail(DL_ENOMEM, "BVH buffers");
  }
  hipError_t e = hipMemcpyAsync(B->nodes.p, bh.nodes.data(), bh.nodes.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m)
    e = hipMemcpyAsync(B->rec.p, bh.rec.data(), bh.rec.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m) e = hipMemcpyAsync(B->sh.p, sh.data(), sh.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete B;
    return fail(DL_EHIP, hipGetErrorString(e));
  }
  B->st.n_gaussians = S->n;
  B->st.n_prims = m;
  B->st.n_nodes = bh.n_nodes;
  B->st.n_leaves = bh.n_leaves;
  B->st.depth = bh.depth;
  B->st.stack_bound = bh.stack_bound;
  B->st.sah_cost = bh.sah_cost;
  B->st.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = B;
  return DL_OK;
}

int dl_bvh_get_stats(const dl_bvh* B, dl_bvh_stats* out) {
  if (!B || !out) return fail(DL_EINVAL, "NULL argument");
  *out = B->st;
  return DL_OK;
}

void dl_bvh_free(dl_bvh* B) { delete B; }

int dl_render_rayorder(dl_ctx* C, const dl_bvh* B, const dl_display* D, const dl_pose* pose,
                       const dl_render_opts* opts, int32_t heap_cap, float* out_dev, void* stream) {
  if (!C || !B || !D) return fail(DL_EINVAL, "NULL context, BVH or display");
  if (B->ctx->device != C->device || D->ctx->device != C->device)
    return fail(DL_EINVAL, "BVH/display live on another device");
  if (!out_dev) return fail(DL_EINVAL, "NULL output");
  if (heap_cap < 1 || heap_cap > (1 << 24)) return fail(DL_EINVAL, "heap_cap must be in [1, 2^24]");
  dl_render_opts o;
  int rc = check_opts(opts, o);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const dl_display_desc& d = D->desc;
  int tw = o.tile_w, th = o.tile_h;
  if (tw == 0 || th == 0) {
    // about 128 rays of one view per (view, tile) list: two batches of a 64-lane workgroup
    const double r = D->n_rays > 0 ? std::min(3.0, (double)D->n_rays / ((double)d.width * d.height)) : 3.0;
    int side = (int)std::ceil(std::sqrt(128.0 * d.n_views / r) / 8.0) * 8;
    tw = th = std::max(8, std::min(side, 256));
  }
  RayLists* L = nullptr;
  if ((rc = build_ray_lists(const_cast<dl_display*>(D), tw, th, s, &L))) return rc;
  C->frame_begin();
  C->tile_w = tw;
  C->tile_h = th;
  C->rpt = 1;
  C->lanes = 64;
  if ((rc = make_cameras(d, pose, C->cams_host))) return rc;
  HIP_TRY(C->cams.ensure((size_t)d.n_views * kCamDoubles * 8));
  HIP_TRY(hipMemcpyAsync(C->cams.p, C->cams_host, (size_t)d.n_views * kCamDoubles * 8, hipMemcpyHostToDevice, s));
  RoConst rcs{};
  rcs.W = d.width;
  rcs.H = d.height;
  rcs.N = d.n_views;
  rcs.T = L->T;
  rcs.tw = tw;
  rcs.th = th;
  rcs.ntx = L->ntx;
  rcs.sh_degree = o.sh_degree;
  rcs.heap_cap = heap_cap;
  rcs.stack_cap = B->st.stack_bound;
  rcs.focal = d.focal_px;
  rcs.cx = d.width / 2.0;
  rcs.cy = d.height / 2.0;
  rcs.z_near = o.z_near;
  rcs.alpha_max = o.alpha_max;
  rcs.t_min = o.t_min;
  for (int k = 0; k < 3; ++k) rcs.bg[k] = o.bg[k];
  rcs.tgt = D->tgt.p ? D->tgt.as<int32_t>() : nullptr;
  rcs.stats = nullptr;
  if (C->prof >= 3) {
    HIP_TRY(C->stats.ensure((size_t)kStatSlots * 3 * 8));
    HIP_TRY(launch_fill_u64(C->stats.as<unsigned long long>(), kStatSlots * 3, 0ull, s));
    rcs.stats = C->stats.as<unsigned long long>();
  }
  const int mk = C->begin(DL_STAGE_BLEND, s);
  HIP_TRY(launch_rayorder(B->nodes.as<float>(), B->rec.as<float4>(), B->sh.as<float4>(), C->cams.as<double>(),
                          L->off.as<uint32_t>(), L->ent.as<uint32_t>(), rcs, out_dev, s));
  C->end(mk, s);
  return DL_OK;
}


}  // extern "C"

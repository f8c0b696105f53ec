/* directl.h — C ABI of the MI355X (gfx950) light-field renderer.
 *
 * Renders the interleaved ("encoded") image of a slanted-lenticular autostereoscopic panel directly from a
 * 3D Gaussian splatting scene (DirectL, arXiv 2407.14053): every subpixel (row x, column y, channel k) is
 * owned by exactly one view v = V(x, 3y + k) (Eq. (1)-(3)), and is the ray of camera v through pixel (x, y)
 * (Sec. 5); each view's Gaussians are projected (Eq. (8)-(9)), binned into that view's tiles, depth-sorted
 * and alpha-composited (Eq. (5), (10)) only into the subpixels that view owns.  The standard paradigm
 * (render all N views, then interlace with Alg. 1) is provided on the same kernels for comparison.
 *
 * Conventions shared by every entry point:
 *  - Return value: DL_OK (0) or a negative DL_E* code; dl_last_error() (thread-local) holds a message.
 *    No C++ exception crosses this boundary.  On error nothing has been enqueued unless stated otherwise.
 *  - Pointers named *_dev are device (HBM) pointers owned by the caller; the library never frees them and
 *    does not keep them after the call returns, except that enqueued work reads/writes them in stream order.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).  All device work is
 *    enqueued on it asynchronously.  Some calls also synchronise the stream (documented per call).
 *  - Layouts are row-major.  Images are float32 [H][W][3] (channel-minor), linear, unclamped.
 *  - Scene arrays (user layout): means[G][3], log_scales[G][3], quats[G][4] as (w, x, y, z),
 *    opacity_logits[G], sh[G][16][3] (coefficient-major, channel-minor, DC first; real spherical
 *    harmonics without the Condon-Shortley phase, index l*l + l + m, m = -l..l).
 *  - Camera axes are OpenCV's (x right, y down, z forward).  Pixel (x, y) has its centre at image
 *    coordinates (y + 1/2, x + 1/2); the principal point is (W/2, H/2).
 *  - Objects are not thread-safe: one thread at a time per dl_ctx (the serving loop serialises host calls).
 */
#ifndef DIRECTL_H
#define DIRECTL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DL_OK = 0,
  DL_EINVAL = -1, /* invalid argument or descriptor */
  DL_ERANGE = -2, /* exact view-map integer arithmetic would overflow */
  DL_ENOMEM = -3, /* device or host allocation failed */
  DL_EHIP = -4,   /* a HIP runtime call failed */
  DL_ECAP = -5,   /* a fixed-capacity plan overflowed (nothing valid was written to the output) */
  DL_ELATER = -6  /* a frame of a first-chunk plan needed a later depth chunk (its image is incomplete) */
};

typedef struct dl_ctx dl_ctx;
typedef struct dl_scene dl_scene;
typedef struct dl_display dl_display;
typedef struct dl_plan dl_plan;
typedef struct dl_bvh dl_bvh;

/* Exact rational num/den, den > 0. */
typedef struct {
  int64_t num, den;
} dl_rational;

/* Lenticular panel (Sec. 3.1 "Interlacing and Display", Eq. (1)-(3); parameters of the display table).
 * width/height: panel pixels (each has 3 subpixels, R G B left to right).  n_views: N in [1, 255].
 * tan_slant: tan(alpha) of the lens tilt (clockwise positive).  pitch: line count L_x in subpixel widths
 * (> 0).  offset: K_offset in subpixel widths.  baseline: distance between the outermost cameras (world
 * units, >= 0).  focal_px: focal length in pixels (> 0), square pixels.
 * repurpose_pw: 0 = every subpixel shows its own pixel of its view (Alg. 1, the identity map); P_w >= 1 =
 * subpixel repurposing (Sec. "Subpixel Repurposing", Alg. 2) in areas of P_w grating units: a subpixel may show
 * its channel of a nearby pixel of its view, so fewer rays are rendered (dl_display_num_rays, dl_display_
 * source_map).  At most 4096. */
typedef struct {
  int32_t width, height, n_views;
  int32_t repurpose_pw;
  dl_rational tan_slant, pitch, offset;
  double baseline;
  double focal_px;
} dl_display_desc;

/* Light-field centre camera (the extrinsic L_0 of Eq. (17)): camera-to-world 4x4 row-major, OpenCV
 * axes.  View v sits at eye_0 + s_v * right_0 with s_v = baseline * (v / (N - 1) - 1/2) (s_0 = 0 when
 * N = 1) and is aimed at eye_0 + converge_dist * forward_0, with down_0 as its reference down axis
 * (evenly spaced cameras converging on the centre, Sec. 3.1). */
typedef struct {
  double c2w[16];
  double converge_dist; /* > 0 */
} dl_pose;

/* Rasterizer constants (the paper fixes none; these are the 3D Gaussian splatting conventions):
 * a Gaussian contributes to a ray iff its camera depth z > z_near, q = d^T Sigma'^{-1} d <= q_cut at the
 * pixel centre and alpha = min(alpha_max, o exp(-q/2)) >= alpha_min (Eq. (10)); contributions are blended
 * front to back by depth (ties by Gaussian index) and the walk stops before a Gaussian whose blend would take
 * the transmittance below t_min (Eq. (5)-(6)).  dilation is added to the diagonal of Sigma' (Eq. (9)).
 * bg is the background colour weighted by the final transmittance.  sh_degree in [0, 3].
 * tile_w/tile_h: screen tile of the blend (0 = automatic: about 900 owned rays per tile for dl_render,
 * 32x32 for dl_render_standard). */
typedef struct {
  float z_near, q_cut, alpha_min, alpha_max, t_min, dilation;
  float bg[3];
  int32_t sh_degree;
  int32_t tile_w, tile_h;
} dl_render_opts;

/* Defaults: z_near 0.2, q_cut 9, alpha_min 1/255, alpha_max 0.99, t_min 1e-4, dilation 0.3, bg 0,
 * sh_degree 3, automatic tiles. */
void dl_default_opts(dl_render_opts* opts);

/* Message of the last error on this thread ("" if none).  Owned by the library. */
const char* dl_last_error(void);

/* Create a context on HIP device `device` (made current for the calling thread). */
int dl_create(int device, dl_ctx** out);
/* Destroy the context (synchronises the device; frees every library-owned buffer of the context). */
void dl_destroy(dl_ctx* ctx);

/* Scene upload (Sec. 3.3: mean, covariance via scale and rotation, opacity, SH colour).  The library keeps
 * its own structure-of-arrays copy in HBM (row-major [59][n_pad] float32).  src_on_device selects whether
 * the five arrays are device pointers (copied with a device transpose on `stream`) or host pointers (the
 * call synchronises `stream`).  n >= 1.  Arrays must be finite. */
int dl_scene_create(dl_ctx* ctx, int64_t n, const float* means, const float* log_scales, const float* quats,
                    const float* opacity_logits, const float* sh, int src_on_device, void* stream,
                    dl_scene** out);
/* Overwrite the parameters of an existing scene with the same n (e.g. after an optimiser step). */
int dl_scene_update(dl_scene* scene, const float* means, const float* log_scales, const float* quats,
                    const float* opacity_logits, const float* sh, int src_on_device, void* stream);
int64_t dl_scene_size(const dl_scene* scene);
void dl_scene_free(dl_scene* scene);

/* Display: validates the descriptor and builds the view map V[H][3W] (uint8) on the device by exact
 * integer arithmetic on the rationals (Eq. (1)-(3) with the floored modulo of Eq. (2)).  Returns DL_ERANGE if
 * the exact arithmetic would not fit 64-bit integers: with tan(alpha) = a/b, L_x = p/q, K_offset = r/c in
 * lowest terms, Q = b c p must be below 2^61, N Q below 2^62, 3W and H below 2^20.  Synchronises `stream`. */
int dl_display_create(dl_ctx* ctx, const dl_display_desc* desc, void* stream, dl_display** out);
void dl_display_free(dl_display* display);
/* Copy V[H][3W] (uint8, view of subpixel column 3y + k in row x) into out_dev. */
int dl_display_view_map(const dl_display* display, uint8_t* out_dev, void* stream);
/* Number of distinct rays (v, x, y) the panel needs (Sec. 5: wh <= n <= 3wh). */
int64_t dl_display_num_rays(const dl_display* display);
/* Source pixel of every subpixel (the index matrix M_i of Alg. 2 without its view and channel, which are
 * V(x, 3y + k) and k): out_dev[(x W + y) 3 + k] = x' W + y' (int32), the pixel of view V(x, 3y + k) whose
 * channel k the subpixel shows; its own pixel unless the panel repurposes subpixels.  Stream-ordered. */
int dl_display_source_map(const dl_display* display, int32_t* out_dev, void* stream);

/* Per-view cameras of the rig for `pose` (Eq. (17)), in FP64 on the host: out_host[N][16] =
 * world-to-camera rotation rows (9), translation (3), camera centre (3), 0. */
int dl_cameras(const dl_display* display, const dl_pose* pose, double* out_host);

/* Projection only (Eq. (8)-(9) and the SH colour), for inspection: out_dev[N][n][12] float32 (all zeros where
 * the Gaussian is culled in that view) =
 * (u, v, A, B, C, Q_limit, ext_x, ext_y, opacity, r, g, b) where (u, v) is the projected mean in image
 * coordinates and A = a log2(e)/2, B = b log2(e), C = c log2(e)/2 for the conic [[a, b], [b, c]] = Sigma'^-1
 * (so that exp(-q/2) = 2^-(A dx^2 + B dx dy + C dy^2)); Q_limit is the tile-test cutoff on the same scale
 * and (ext_x, ext_y) the half extents of that ellipse in pixels; depth_dev[N][n] float64 = camera z, or NaN when
 * the Gaussian cannot reach any pixel centre of that view (behind z_near, alpha always below alpha_min, or
 * its cutoff ellipse misses the screen). */
int dl_project(dl_ctx* ctx, const dl_scene* scene, const dl_display* display, const dl_pose* pose,
               const dl_render_opts* opts, float* out_dev, double* depth_dev, void* stream);

/* Bytes of the fixed device array behind dl_project_noalloc (held on every device the library runs on until the
 * process ends). */
#define DL_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* dl_project without any allocation, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same records out_dev[N][n][12] and depths
 * depth_dev[N][n] as dl_project, from the same kernel; its scratch (the N cameras, 256-byte aligned, then the
 * N x n depth keys, 8 bytes each) lives in a fixed device array of DL_NOALLOC_SCRATCH_BYTES per device, whose
 * address dl_create takes.  Calls no hipMalloc, hipFree or other allocating routine; the cameras are staged
 * through the context's pinned buffer (allocated by dl_create).  Errors: DL_ERANGE (nothing launched) when
 * round_up(128 N, 256) + 8 N n exceeds DL_NOALLOC_SCRATCH_BYTES; DL_EINVAL for NULL arguments or when the
 * context's device is not the current device; DL_EHIP.  Every call on a device shares that device's array and
 * finds the previous call's contents there (nothing in it needs to start at zero): calls that overlap on one
 * device (other streams, other threads) race; calls ordered on one stream do not.  Synchronises `stream`. */
int dl_project_noalloc(dl_ctx* ctx, const dl_scene* scene, const dl_display* display, const dl_pose* pose,
                       const dl_render_opts* opts, float* out_dev, double* depth_dev, void* stream);

/* DirectL forward: the encoded image out_dev[H][W][3] (every subpixel written).  The visible Gaussians of
 * each view are binned and blended in depth chunks, front to back; tiles whose rays have all terminated take
 * no further keys.  Synchronises `stream` at the end of the frame to check the library-owned key buffers
 * (grown, and the frame rendered again, if a chunk overflowed them). */
int dl_render(dl_ctx* ctx, const dl_scene* scene, const dl_display* display, const dl_pose* pose,
              const dl_render_opts* opts, float* out_dev, void* stream);

/* Standard paradigm on the same kernels and chunking: render all N full views (views_dev[N][H][W][3] if
 * non-NULL, else a library buffer), then interlace them with Alg. 1 into out_dev[H][W][3].  Synchronises
 * `stream`. */
int dl_render_standard(dl_ctx* ctx, const dl_scene* scene, const dl_display* display, const dl_pose* pose,
                       const dl_render_opts* opts, float* out_dev, float* views_dev, void* stream);

/* The paper's multi-view baselines (Alg. 1 with its Resize): the N views rendered at view_w x view_h pixels
 * (the panel's rig and vertical field of view: focal_px scaled by view_h / height), each upsampled to the
 * panel by bilinear interpolation (half-pixel centres, edges clamped), then interlaced into out_dev[H][W][3]
 * (through the source map on a repurposed panel).  The LR and MR rows of the paper's comparison; with the
 * panel's own size the views are the standard paradigm's.  views_dev: NULL or [N][view_h][view_w][3] to keep
 * the views.  tile_w/tile_h of opts as for dl_render_standard. */
int dl_render_multiview(dl_ctx* ctx, const dl_scene* scene, const dl_display* display, const dl_pose* pose,
                        const dl_render_opts* opts, int32_t view_w, int32_t view_h, float* out_dev,
                        float* views_dev, void* stream);

/* Backward of dl_render (the paper names backpropagation as future work, Sec. 9; here the rasterized
 * DirectL forward is differentiated): given the forward's encoded image out_dev[H][W][3] for the same scene,
 * display, pose and options, and grad_out_dev = d loss / d out_dev, writes d loss / d parameters in the
 * user layouts g_means[G][3], g_log_scales[G][3], g_quats[G][4] (w.r.t. the unnormalised quaternion),
 * g_opacity_logits[G], g_sh[G][16][3] (device buffers, overwritten).  The forward's tile lists are recomputed
 * (no per-pixel blend state is stored); threshold and termination decisions are the forward's and carry no
 * gradient, and neither does the colour clamp at 0 nor the opacity clamp at alpha_max.  Per-Gaussian
 * gradients are accumulated with floating-point atomics (summation order is not deterministic).
 * Synchronises `stream`. */
int dl_render_backward(dl_ctx* ctx, const dl_scene* scene, const dl_display* display, const dl_pose* pose,
                       const dl_render_opts* opts, const float* out_dev, const float* grad_out_dev, float* g_means,
                       float* g_log_scales, float* g_quats, float* g_opacity_logits, float* g_sh, void* stream);

/* Alg. 1 alone: out_dev[x][y][k] = views_dev[V(x, 3y + k)][x][y][k]. */
int dl_interleave(const dl_display* display, const float* views_dev, float* out_dev, void* stream);

/* ---- ray-order 3DGS (Sec. "Ray-Order 3DGS", Alg. 3, Eq. (21)-(23)) ----
 * A second renderer for the same rays as dl_render: every ray (its view's camera centre o, unit direction d
 * through the pixel centre) is cast through a BVH over the Gaussians; a Gaussian is hit where its response
 * along the ray peaks, t_j = (mu - o)^T Sigma^-1 d / (d^T Sigma^-1 d) (Eq. (22)), if there t_j >= z_near,
 * q_j <= q_cut and alpha_j = o_j G(o + t_j d) >= alpha_min (Eq. (23)); the c_h hits of smallest (t_j, j) are
 * blended front to back (alpha clamped at alpha_max, stop before the transmittance would fall below t_min,
 * background with the final transmittance) with SH colours in direction d.  This computes a different image
 * from the rasterizer (peak response along the ray instead of the projected 2D Gaussian). */
typedef struct {
  int64_t n_gaussians;  /* scene size */
  int64_t n_prims;      /* Gaussians in the BVH (opacity >= alpha_min) */
  int64_t n_nodes;      /* 8-wide nodes */
  int64_t n_leaves;     /* leaf children (at most 4 Gaussians each) */
  int32_t depth;        /* wide levels */
  int32_t stack_bound;  /* traversal stack entries per ray */
  double sah_cost;      /* Eq. (21) of the binary SAH tree, c_node = c_prim = 1, areas relative to the root */
  double build_ms;      /* host build time (copy-back, build, upload) */
} dl_bvh_stats;

/* Build the BVH of a scene (Eq. (21): binned SAH, collapsed to 8-wide nodes) on the host from the scene's
 * current parameters; q_cut and alpha_min of opts (NULL: defaults) fix the hit rule's bounds, baked into the
 * boxes.  The BVH holds its own copy of what it needs (records and SH in leaf order): later dl_scene_update calls
 * do not reach it (build again).  Synchronises `stream`.  DL_ERANGE if the tree needs a traversal stack deeper
 * than 256 entries. */
int dl_bvh_build(dl_ctx* ctx, const dl_scene* scene, const dl_render_opts* opts, void* stream, dl_bvh** out);
int dl_bvh_get_stats(const dl_bvh* bvh, dl_bvh_stats* out);
void dl_bvh_free(dl_bvh* bvh);

/* Render the display's rays (repurposed panels included) in ray order with heap capacity heap_cap = c_h in
 * [1, 2^24] into out_dev[H][W][3] (every subpixel written).  opts: z_near, alpha_max, t_min, bg, sh_degree;
 * tile_w/tile_h choose the (view, tile) ray lists that a 64-lane workgroup walks (0: about 128 rays per list);
 * q_cut and alpha_min are the BVH's.  Asynchronous on `stream`; profiling level >= 1 records the kernel as the
 * blend stage, level 3 counts Gaussian tests (evaluations), blends and rays. */
int dl_render_rayorder(dl_ctx* ctx, const dl_bvh* bvh, const dl_display* display, const dl_pose* pose,
                       const dl_render_opts* opts, int32_t heap_cap, float* out_dev, void* stream);

/* ---- plans: fixed-buffer frames replayed as HIP graphs (serving) ----
 * A plan owns every per-frame buffer of one (scene, display, options) at fixed capacity, sized by an eager
 * DirectL frame at probe_pose: the per-chunk tile-key capacity is the larger of min_key_capacity and the probe's
 * largest depth chunk plus 30%.  Scene and display
 * may be shared by many plans and contexts of the same device; both must outlive the plan, and the scene keeps
 * its size.  out_dev: caller-owned device image [H][W][3] float32 that every launch of the plan writes; it must
 * outlive the plan.
 * The frame is captured into a HIP graph on `stream` when the plan is created.  dl_plan_render uploads the
 * cameras of `pose`, then launches that graph on `stream`; it does not synchronise.  Streams must not be the
 * null stream.  Launches of one plan must be
 * ordered (one stream, or the previous frame completed): they share the plan's buffers.  After a launch has
 * completed, dl_plan_check returns DL_OK if no frame of the plan so far overflowed its capacity, else DL_ECAP
 * (sticky: the overflowing frame's image, and any later one, is invalid) with *need = the most keys a depth
 * chunk required — render those requests eagerly or with a new plan.  Many frames may be launched back to back
 * and checked once after the last.
 * Depth chunks (as for dl_render: each view's nearest Gaussians first, the rest only for tiles whose rays are
 * still live): when the probe frame finished in its first chunk, the plan's graphs
 * hold that chunk alone, which saves the later chunk's (then empty) launches.  A frame that leaves a tile live
 * after it is incomplete; dl_plan_check then returns DL_ELATER (sticky, after any DL_ECAP) — the caller renders
 * that pose eagerly, or calls dl_plan_use_all_chunks and launches it again.  dl_plan_first_chunk_only: 1 for
 * such a plan, 0 otherwise (DL_EINVAL for NULL).  dl_plan_use_all_chunks recaptures the plan's graphs (the
 * batched ones too) with every chunk and clears its status; it waits for the plan's last launch; DL_OK at once
 * for a plan that has every chunk.
 * dl_plan_bytes: device bytes the plan holds.  dl_plan_free waits for the plan's work to finish. */
int dl_plan_create(dl_ctx* ctx, const dl_scene* scene, const dl_display* display, const dl_render_opts* opts,
                   const dl_pose* probe_pose, int64_t min_key_capacity, float* out_dev, void* stream,
                   dl_plan** out);
int dl_plan_render(dl_plan* plan, const dl_pose* pose, void* stream);
int dl_plan_check(const dl_plan* plan, int64_t* need);
int dl_plan_first_chunk_only(const dl_plan* plan);
int dl_plan_use_all_chunks(dl_plan* plan, void* stream);
int64_t dl_plan_bytes(const dl_plan* plan);
/* Device bytes a plan of (scene, display, opts) would hold with a per-chunk tile-key capacity of key_capacity
 * (a plan sizes its own capacity with its probe frame), for admission decisions before creating one; -1 on a
 * NULL argument or invalid options. */
int64_t dl_plan_estimate_bytes(const dl_scene* scene, const dl_display* display, const dl_render_opts* opts,
                               int64_t key_capacity);
void dl_plan_free(dl_plan* plan);

/* Batched launches (serving several requests of one plan's (scene, display, options) with one launch):
 * dl_plan_batch_prepare captures, once per plan, graphs of 1..max_frames frames in a row (max_frames <=
 * DL_MAX_BATCH) on the plan's buffers, frame k writing outs_dev[k] ([H][W][3] float32, caller-owned, must outlive
 * the plan); the plan's own out_dev is not written by them.  dl_plan_render_batch uploads the cameras of
 * poses[0..n) together (one copy from pinned staging) and launches the n-frame graph on `stream` (not the null
 * stream); frame k of the batch is pose k.  Frames of a batch run one after another, so a batch takes n single
 * frames' time minus their per-launch costs (camera uploads, graph launches, status copies).  Ordering and
 * overflow status as for dl_plan_render (dl_plan_check after the launch completed; a frame of the batch that
 * overflowed makes the status sticky).  Errors: DL_EINVAL (NULL arguments, n outside [1, max_frames], batches not
 * prepared or prepared twice), DL_ENOMEM, DL_EHIP. */
#define DL_MAX_BATCH 16
int dl_plan_batch_prepare(dl_plan* plan, int32_t max_frames, float* const* outs_dev, void* stream);
int dl_plan_render_batch(dl_plan* plan, const dl_pose* poses, int32_t n, void* stream);

/* Per-depth-chunk capacity of the context's tile-key buffers (0 until the first frame sizes it).  A frame
 * whose chunk needs more keys grows the buffers and renders again; setting a smaller value is allowed (the
 * buffers shrink lazily only in the sense that the value bounds new growth decisions). */
int dl_set_key_capacity(dl_ctx* ctx, int64_t keys);
int64_t dl_key_capacity(const dl_ctx* ctx);

/* ---- measurement ---- */
enum {
  DL_STAGE_UPLOAD = 0,     /* camera upload and counter clears */
  DL_STAGE_PROJECT = 1,    /* projection + SH of all views */
  DL_STAGE_DEPTH_SORT = 2, /* per-view depth sort */
  DL_STAGE_BIN_COUNT = 3,  /* tiles per (view, Gaussian) */
  DL_STAGE_SCAN = 4,       /* key offsets */
  DL_STAGE_BIN_EMIT = 5,   /* (view, tile) keys */
  DL_STAGE_TILE_SORT = 6,  /* partition of the keys by (view, tile) */
  DL_STAGE_BOUNDS = 7,     /* list bounds */
  DL_STAGE_BLEND = 8,      /* compositing */
  DL_STAGE_INTERLEAVE = 9, /* Alg. 1 (standard path only) */
  DL_NSTAGES = 10
};

/* Per-frame measurements of the last dl_render / dl_render_standard made with profiling on.
 * stage_ms: summed HIP-event durations per stage on the render stream; stage_launches: occurrences.
 * keys: the largest number of (view, tile) list entries of one depth chunk; visible: (view, Gaussian) pairs
 * that reach the screen;
 * evaluations: (ray, list entry) pairs the blend examined; blends: pairs composited; rays: rays rendered
 * (these three are zero unless profiling is at level 3); stages without events read 0. */
#define DL_MAX_CHUNKS 8
typedef struct {
  double stage_ms[DL_NSTAGES];
  int32_t stage_launches[DL_NSTAGES];
  int64_t keys, visible, evaluations, blends, rays;
  int32_t batches, tile_w, tile_h, rays_per_lane;
  int32_t chunks;                               /* depth chunks of the frame */
  double chunk_ms[DL_MAX_CHUNKS][DL_NSTAGES];   /* stage_ms split by depth chunk (frame-level stages in 0) */
  int32_t lanes;                                /* blend workgroup size (rays_per_lane rays per lane) */
} dl_frame_stats;

/* Profiling of subsequent frames of this context: 0 off; 1 HIP events around the blend launches only (the
 * dominant kernel; two events per depth chunk); 2 events around every stage (each event adds a few microseconds
 * between kernels); 3 every stage plus the blend's work counters (evaluations, blends, rays), which cost
 * atomics in the blend kernel — time with level 1, break down with level 2, count with level 3.  Other levels:
 * DL_EINVAL. */
int dl_set_profiling(dl_ctx* ctx, int level);
/* Read the measurements of the last profiled frame (synchronises on its events). */
int dl_frame_stats_get(dl_ctx* ctx, dl_frame_stats* out);

/* Vector-ALU issue rates of the device (the ceilings against which the blend's arithmetic is measured): short
 * kernels of independent dependent-chain steps, 8 wavefronts per SIMD on every compute unit, timed with HIP
 * events (best of three after one warm-up launch).  Synchronous; makes `device` current.  Writes
 * min(n_out, 16) doubles: [0] v_fma_f32 lane operations per second, [1] v_exp_f32 lane operations per second,
 * [2] steps of (4 v_fma_f32 + 1 v_exp_f32) per second and lane, [3] (ray, record) pairs per second of the
 * blend's per-pair instruction sequence for a ray that fills one channel (lanes), [4] the same for a ray that
 * fills three channels, with the clamp at alpha_max, [5] the engine clock measured over the FMA kernel (Hz,
 * shader clock counter against the 100 MHz constant clock), [6] compute units, [7]-[10] lane operations per
 * second of single instruction classes: v_add_f32, v_fmac_f32, v_mul_f32 with a negated operand, v_fma_f32 with
 * three VGPR operands, [11] v_cndmask_b32 with an SGPR-pair mask, [12] steps of (v_cmp_gt_f32 into an SGPR pair
 * + v_add_f32), [13] v_fmac_f32 with three distinct registers, [14] v_fma_f32 with an SGPR operand, [15] steps of
 * (1 v_exp_f32 + 4 independent v_fma_f32).  Errors: DL_EINVAL (out NULL, n_out < 1, no such device), DL_EHIP. */
int dl_probe_issue_rates(int device, double* out, int n_out);

#ifdef __cplusplus
}
#endif

#endif /* DIRECTL_H */

// Tile binning of the depth-sorted projected Gaussians of each view, one depth chunk at a time (gfx950).
//
// Input order is (view, depth rank), so emitting (key = tile, value = rank) pairs in that order — each view's
// pairs in one contiguous range — and then partitioning every view's range by tile with a stable radix pass
// yields every (view, tile) list already in front-to-back order: the depth digits were sorted before the
// Gaussians were duplicated into tiles.
//
// Depth chunks: chunk c of view v holds the visible Gaussians of depth rank [n_v lo_c, n_v hi_c) / den.
// Chunks are binned and blended front to back; a tile whose rays have all terminated is marked dead by the
// blend and receives no keys from later chunks, so keys behind opaque regions are never produced.
//
// A Gaussian is listed in a tile when its cutoff ellipse (q <= q_limit) reaches at least one pixel centre of
// the tile.  The test is conservative (margins above FP32 error), so that the per-pixel rule in the blend
// alone decides what each ray composites and the image does not depend on the tile size or the chunks.
#include "dl_internal.h"

namespace dl {
namespace {

struct TileRange {
  int tx0, tx1, ty0, ty1;
};

__device__ inline bool tile_range(const float* r, const BlendConst& bc, TileRange& tr) {
  // columns y whose centre y + 0.5 lies within [u - ext_x, u + ext_x], widened by one pixel
  const float u = r[0], v = r[1], ex = r[6], ey = r[7];
  int y0 = (int)ceilf(u - ex - 0.5f), y1 = (int)floorf(u + ex - 0.5f);
  int x0 = (int)ceilf(v - ey - 0.5f), x1 = (int)floorf(v + ey - 0.5f);
  y0 = max(y0 - 1, 0); y1 = min(y1 + 1, bc.W - 1);
  x0 = max(x0 - 1, 0); x1 = min(x1 + 1, bc.H - 1);
  if (y0 > y1 || x0 > x1) return false;
  tr.tx0 = y0 / bc.tw; tr.tx1 = y1 / bc.tw;
  tr.ty0 = x0 / bc.th; tr.ty1 = x1 / bc.th;
  return true;
}

// Minimum over the tile's pixel centres (a rectangle) of Q = A dx^2 + B dx dy + C dy^2 about (u, v).
// Zero when the centre lies inside.  Otherwise the minimum of the convex quadratic lies on an edge that faces
// the centre — the nearer of the two vertical edges or the nearer of the two horizontal ones — where it is a
// 1D quadratic minimised at the clamped stationary point (-B dx / 2C along a vertical edge, -B dy / 2A along a
// horizontal one).  Evaluating both facing edges (one may not face the centre: its value is still a value of
// Q on the rectangle) gives the minimum without branches.  hA = 1 / 2A and hC = 1 / 2C per Gaussian.
__device__ inline bool tile_touch(float u, float v, float A, float B, float C, float qlim, float hA, float hC,
                                  float xlo, float xhi, float ylo, float yhi) {
  const float dxl = xlo - u, dxh = xhi - u, dyl = ylo - v, dyh = yhi - v;
  const bool inside = (dxl <= 0.0f) & (dxh >= 0.0f) & (dyl <= 0.0f) & (dyh >= 0.0f);
  const float ex = dxl > 0.0f ? dxl : dxh;  // the facing vertical edge
  const float ey = dyl > 0.0f ? dyl : dyh;  // the facing horizontal edge
  const float dy1 = fminf(fmaxf(-B * ex * hC, dyl), dyh);
  const float q1 = A * ex * ex + B * ex * dy1 + C * dy1 * dy1;
  const float dx2 = fminf(fmaxf(-B * ey * hA, dxl), dxh);
  const float q2 = A * dx2 * dx2 + B * dx2 * ey + C * ey * ey;
  return inside | (fminf(q1, q2) <= qlim * 1.001f + 1e-3f);
}

// The geometric half of a record: u, v, A, B, C, Q_limit, ext_x, ext_y.
__device__ inline void load_rec_geom(const float4* rec, float* r) {
  const float4 A = rec[0], B = rec[1];
  r[0] = A.x; r[1] = A.y; r[2] = A.z; r[3] = A.w;
  r[4] = B.x; r[5] = B.y; r[6] = B.z; r[7] = B.w;
}

__device__ inline uint32_t wave_incl_scan_u32(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Per-wavefront staging of its 64 Gaussians.
template <int GPW>
struct WaveBin {
  float u[GPW], v[GPW], A[GPW], B[GPW], C[GPW], qlim[GPW], hA[GPW], hC[GPW], rw[GPW];
  int tx0[GPW], ty0[GPW], wr[GPW];
  uint32_t pre[GPW], nt[GPW];
  int mark[128];  // per pair of a two-step window: the lane of the Gaussian whose pairs start there, or -1
};

// Orders the wavefront's LDS accesses: what a lane wrote before is seen by every lane of the wavefront after
// (without it the compiler may take a lane's own earlier store as the value of its load).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive maximum over lanes 0..lane of the wavefront: DPP row shifts within each row of 16 lanes, then
// the maxima of the rows below, read from lanes 15, 31 and 47; values are >= -1.
__device__ inline int wave_max_scan(int x, int lane) {
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false));  // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false));  // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false));  // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false));  // row_shr:8
  const int r0 = __builtin_amdgcn_readlane(x, 15);
  const int r1 = max(r0, __builtin_amdgcn_readlane(x, 31));
  const int r2 = max(r1, __builtin_amdgcn_readlane(x, 47));
  return max(x, lane >= 48 ? r2 : lane >= 32 ? r1 : lane >= 16 ? r0 : -1);
}

// Each wavefront takes 64 consecutive depth ranks of one view (one per lane), computes every Gaussian's
// tile rectangle, and then walks the flattened list of (Gaussian, tile of its rectangle) pairs 64 at a time,
// so that a large splat is shared by all lanes instead of stalling one.  Pairs are visited Gaussian by
// Gaussian in rank order, and the hits of each step are compacted with a ballot, so the wavefront's keys come
// out in rank order within every tile.  A view none of whose tiles is live (`live`, chunks after the first)
// produces no keys and reads no records.
//
// Two ways to turn the hits into (view, tile) lists:
//   !TABLE: COUNT stores the number of keys of each wavefront; EMIT writes (tile, rank) pairs from the
//           wavefront's scanned offset, in emission order, and a stable partition by tile follows.
//   TABLE:  COUNT stores, for every workgroup (group of four wavefronts) g and tile t of view v, the numbers of
//           its four wavefronts' hits in t, one byte each (at most kTableWaveRanks), in the word
//           table[base_v + t * ng_v + g] (ng_v = groups of the view, base_v = T * sum of ng over earlier views);
//           the exclusive scan of the words' byte sums in that order gives each group its first slot in every
//           tile's final list, and the bytes its wavefronts' slots after it, so EMIT writes the ranks straight
//           into the lists: no partition.  Lanes of one step that hit the same tile take consecutive slots in
//           lane order, which is rank order, since every Gaussian's tiles are distinct.  The tile counters of
//           the four wavefronts of a workgroup live in LDS as [tile][wavefront] (T <= kTableMaxTiles).
static_assert(kTableWaveRanks <= 255, "a wavefront's hits in one tile fit the table's byte");

template <bool EMIT, bool TABLE>
__global__ __launch_bounds__(256) void bin_kernel(const float4* __restrict__ rec, const uint32_t* __restrict__ vis_count,
                                                  const uint32_t* __restrict__ live, BlendConst bc, ChunkArgs ch,
                                                  const uint8_t* __restrict__ alive, uint32_t* __restrict__ counts,
                                                  unsigned long long* __restrict__ total,
                                                  const uint32_t* __restrict__ offsets, uint32_t* __restrict__ keys,
                                                  uint32_t* __restrict__ vals, const uint32_t* __restrict__ tab_base) {
  // Gaussians per wavefront: the table form takes 32 (lanes 32-63 own none; the pair walk still runs 64 pairs a
  // step), so that the first chunk's few hundred Gaussians per view spread over twice the wavefronts and each
  // wavefront's serial walk is half as long
  constexpr int GPW = TABLE ? kTableWaveRanks : 64;
  constexpr int GPG = 4 * GPW;  // per workgroup (a group)
  __shared__ WaveBin<GPW> wb[4];
  __shared__ unsigned long long part[4];
  // TABLE (dynamic LDS, sized by the launch): the tile counters, [T] x 16 bytes; for EMIT also each tile's
  // first slot of the workgroup's run in the lists, [T] x 4 bytes, and the workgroup's hits staged in list order
  // as ranks relative to its first rank (below GPG), kTableStage bytes, copied out run by run per group
  extern __shared__ __align__(16) uint8_t bin_dyn[];
  uint4* tcnt_s = reinterpret_cast<uint4*>(bin_dyn);
  uint32_t* ppos = reinterpret_cast<uint32_t*>(bin_dyn + 16 * bc.T);
  uint8_t* stage = bin_dyn + 20 * bc.T;
  __shared__ uint32_t ssum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  WaveBin<GPW>& W = wb[w];
  uint32_t* tc = reinterpret_cast<uint32_t*>(tcnt_s);  // tc[4 t + w]: wavefront w's counter of tile t
  // TABLE: a one-dimensional grid in which all workgroups of view v have the same index modulo 8, so that they
  // run on one XCD (workgroups are handed to the 8 XCDs in turn) and the view's table and lists are touched by
  // one L2.  Otherwise blockIdx.y is the view.
  int v, bx, gx;
  if (TABLE) {
    gx = (int)ch.tgx;
    const int slot = (int)(blockIdx.x >> 3), q = slot / gx;
    bx = slot - q * gx;
    v = (int)(blockIdx.x & 7) + 8 * q;
    if (v >= bc.N) return;
  } else {
    v = blockIdx.y;
    bx = blockIdx.x;
    gx = gridDim.x;
  }
  const int64_t nv = vis_count[v];
  const int64_t fv = ch.front ? (int64_t)ch.front[v] : 0;
  int64_t lo, hi;
  if (ch.front && ch.first) {
    lo = 0;
    hi = fv;
  } else {
    lo = max(fv, nv * ch.num_lo / ch.den);
    hi = max(lo, nv * ch.num_hi / ch.den);
  }
  hi = min(hi, lo + ch.stride);  // the host sizes the stride to cover every chunk; never write past its slots
  const bool view_live = !live || live[v] != 0;
  // groups of GPG consecutive ranks of this chunk (none for a view without live tiles)
  const int64_t groups = view_live ? (hi - lo + GPG - 1) / GPG : 0;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint8_t* al = alive ? alive + (int64_t)v * bc.T : nullptr;
  const int T = bc.T;
  const int64_t ng = groups;  // TABLE: group slots of this view
  const int64_t tbase = TABLE ? (int64_t)tab_base[v] : 0;
  int tbits = 0;
  while ((1 << tbits) < T) ++tbits;
  if (!EMIT && !TABLE)  // the count pass owes a zero to every wavefront slot no group covers
    for (int64_t j = groups * 4 + (int64_t)bx * 256 + threadIdx.x; j < ch.wstride; j += (int64_t)gx * 256)  // GPG = 256
      counts[(int64_t)v * ch.wstride + j] = 0;
  unsigned long long block_sum = 0;

  // Pair p of the wavefront's flattened (Gaussian, tile) list, owned by the Gaussian of lane i: its tile t
  // (column tx, row ty of the Gaussian's rectangle, row-major), and whether the Gaussian's cutoff ellipse
  // reaches a pixel centre of the (live) tile.  Branch-free, so that the two pairs of a step are computed side
  // by side; pairs beyond the list are misses.
  auto locate = [&](uint32_t p, int i, uint32_t S, int& t, int& tx, int& ty) -> bool {
    const uint32_t q = p - W.pre[i];
    const int wr = W.wr[i];
    // row = q / wr from the rounded reciprocal, then one correction step
    int row = (int)(((float)q + 0.5f) * W.rw[i]);
    const int rem0 = (int)q - row * wr;
    row += (rem0 >= wr ? 1 : 0) - (rem0 < 0 ? 1 : 0);
    tx = W.tx0[i] + ((int)q - row * wr);
    ty = W.ty0[i] + row;
    const bool valid = (p < S) & (q < W.nt[i]);
    t = valid ? ty * bc.ntx + tx : 0;
    const float xlo = tx * bc.tw + 0.5f, xhi = min((tx + 1) * bc.tw, bc.W) - 0.5f;
    const float ylo = ty * bc.th + 0.5f, yhi = min((ty + 1) * bc.th, bc.H) - 0.5f;
    bool hit = valid & tile_touch(W.u[i], W.v[i], W.A[i], W.B[i], W.C[i], W.qlim[i], W.hA[i], W.hC[i], xlo, xhi,
                                  ylo, yhi);
    if (al) hit = hit && al[t];
    return hit;
  };
  // this lane's Gaussian's rectangle (first column and row, width), first pair and pair count, for other lanes
  // to read with readlane
  int g_tx0 = 0, g_ty0 = 0, g_wr = 1;
  uint32_t g_pre = 0, g_nt = 0;
  // One step's hits in lane order: keys (!TABLE) or ranks into the lists (TABLE EMIT), or counts.
  uint32_t pos = 0;  // !TABLE: next key of this wavefront
  auto record = [&](bool hit, int i, int t, int tx, int ty, uint32_t s0, uint32_t S, int64_t r, bool staged) {
    const uint64_t bal = __ballot(hit);
    if (TABLE) {
      if (!EMIT) {
        if (hit) atomicAdd(&tc[4 * t + w], 1u);
      } else if (bal) {
        // k = hits of this step in the same tile on earlier lanes.  Those belong to earlier Gaussians of the
        // step; when the step spans few Gaussians, each is tested for holding this tile within the step (its
        // pair index and hit bit), else lanes are matched on the tile index, one ballot per bit.
        uint32_t k = 0;
        const int ia = __builtin_amdgcn_readlane(i, 0), ib = __builtin_amdgcn_readlane(i, 63);
        if (ib - ia <= 4) {
          for (int j = ia; j < ib; ++j) {
            const int wrj = __builtin_amdgcn_readlane(g_wr, j);
            const int dx = tx - __builtin_amdgcn_readlane(g_tx0, j), dy = ty - __builtin_amdgcn_readlane(g_ty0, j);
            const uint32_t prej = __builtin_amdgcn_readlane(g_pre, j);
            const uint32_t ntj = __builtin_amdgcn_readlane(g_nt, j);
            const uint32_t q = (uint32_t)dy * (uint32_t)wrj + (uint32_t)dx;
            const uint32_t pp = prej + q - s0;  // the step offset of pair (j, this tile)
            k += (j < i && (uint32_t)dx < (uint32_t)wrj && q < ntj && pp < 64u && ((bal >> (pp & 63u)) & 1ull))
                     ? 1u : 0u;
          }
        } else {
          uint64_t m = bal;
          for (int b = 0; b < tbits; ++b) {
            const bool bit = (t >> b) & 1;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
          }
          k = (uint32_t)__popcll(m & below);
        }
        if (hit) {
          const uint32_t at = tc[4 * t + w] + k;
          if (staged) stage[at] = (uint8_t)(GPW * w + i);  // the Gaussian in lane i, relative to the group
          else if (at < ch.cap) vals[at] = (uint32_t)(r - lane + i);  // depth rank of the Gaussian in lane i
          atomicAdd(&tc[4 * t + w], 1u);  // after every lane's read: the tile's slots advance by its hits
        }
      }
    } else {
      if (EMIT && hit) {
        const uint32_t at = pos + (uint32_t)__popcll(bal & below);
        if (at < ch.cap) {
          keys[at] = (uint32_t)t;  // the view is the segment: keys of view v lie in its scanned range
          vals[at] = (uint32_t)(r - lane + i);  // depth rank of the Gaussian in lane i
        }
      }
      pos += (uint32_t)__popcll(bal);
    }
  };

  // the chunk's groups, strided over the view's workgroups
  for (int64_t grp = bx; grp < groups; grp += gx) {
    const int64_t idx = grp * GPG + (int64_t)w * GPW + lane;  // this lane's rank in the chunk (lanes < GPW)
    const int64_t wv = grp * 4 + w;  // wavefront index within the view's chunk
    const int64_t wslot = (int64_t)v * ch.wstride + wv;
    const bool wave_in = wv < ch.wstride;
    const int64_t r = lo + idx;
    uint32_t nt = 0;
    if (lane < GPW && r < hi) {
      float rr[8];
      load_rec_geom(rec + ((int64_t)v * bc.G + r) * kRecF4, rr);
      TileRange tr;
      if (tile_range(rr, bc, tr)) {
        W.u[lane] = rr[0];
        W.v[lane] = rr[1];
        W.A[lane] = rr[2];
        W.B[lane] = rr[3];
        W.C[lane] = rr[4];
        W.qlim[lane] = rr[5];
        W.hA[lane] = 0.5f / rr[2];
        W.hC[lane] = 0.5f / rr[4];
        W.tx0[lane] = tr.tx0;
        W.ty0[lane] = tr.ty0;
        W.wr[lane] = tr.tx1 - tr.tx0 + 1;
        W.rw[lane] = 1.0f / (float)(tr.tx1 - tr.tx0 + 1);
        nt = (uint32_t)((tr.tx1 - tr.tx0 + 1) * (tr.ty1 - tr.ty0 + 1));
        g_tx0 = tr.tx0;
        g_ty0 = tr.ty0;
        g_wr = tr.tx1 - tr.tx0 + 1;
      }
    }
    const uint32_t incl = wave_incl_scan_u32(nt, lane);
    const uint32_t my_pre = incl - nt;
    if (lane < GPW) {
      W.pre[lane] = my_pre;
      W.nt[lane] = nt;
    }
    g_pre = my_pre;
    g_nt = nt;
    const uint32_t S = __shfl(incl, 63, 64);
    bool staged = false;
    if (TABLE && !EMIT) {
      // the workgroup's counters, 16 bytes per tile
      for (int tt = threadIdx.x; tt < T; tt += 256) tcnt_s[tt] = make_uint4(0, 0, 0, 0);
    }
    if (TABLE && EMIT) {
      // The workgroup's four wavefronts own consecutive slots of every tile's list: its run, which starts at the
      // scanned offset and holds the counts of the table word, wavefront after wavefront.  When all runs fit in
      // LDS they are laid out back to back there (local slots), else the counters hold the list slots themselves.
      const int64_t at = tbase + grp;
      uint32_t cnt[4];
      uint32_t mine = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tt = 4 * (int)threadIdx.x + q;
        cnt[q] = 0;
        if (tt < T) {
          const uint32_t c = counts[at + (int64_t)tt * ng], o = offsets[at + (int64_t)tt * ng];
          const uint32_t c0 = c & 255u, c1 = (c >> 8) & 255u, c2 = (c >> 16) & 255u, c3 = c >> 24;
          tcnt_s[tt] = make_uint4(o, o + c0, o + c0 + c1, o + c0 + c1 + c2);
          ppos[tt] = o;
          cnt[q] = c0 + c1 + c2 + c3;
        }
        mine += cnt[q];
      }
      const uint32_t inc = wave_incl_scan_u32(mine, lane);
      if (lane == 63) ssum[w] = inc;
      __syncthreads();
      uint32_t run = inc - mine, total = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < w) run += ssum[q];
        total += ssum[q];
      }
      staged = total <= (uint32_t)kTableStage;
      if (staged) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int tt = 4 * (int)threadIdx.x + q;
          if (tt < T) {
            const uint4 o = tcnt_s[tt];
            tcnt_s[tt] = make_uint4(run, run + (o.y - o.x), run + (o.z - o.x), run + (o.w - o.x));
          }
          run += cnt[q];
        }
      }
    }
    __syncthreads();

    if (!TABLE) pos = EMIT && wave_in && S ? offsets[wslot] : 0u;
    int carry = 0;  // owner of the pair before the window
    for (uint32_t s0 = 0; s0 < S; s0 += 128) {
      // two steps of 64 pairs side by side, recorded in order.  Owners: each Gaussian marks the pair where its
      // list starts, and a running maximum over the window's pairs carries it to the pairs that follow.
      wave_lds_sync();  // the previous window's reads of the marks are done
      W.mark[lane] = -1;
      W.mark[64 + lane] = -1;
      wave_lds_sync();
      if (nt > 0 && my_pre - s0 < 128u) W.mark[my_pre - s0] = lane;
      wave_lds_sync();
      const int i0 = max(wave_max_scan(W.mark[lane], lane), carry);
      const int i1 = max(wave_max_scan(W.mark[64 + lane], lane), __builtin_amdgcn_readlane(i0, 63));
      carry = __builtin_amdgcn_readlane(i1, 63);
      int t0, x0, y0, t1, x1, y1;
      const bool h0 = locate(s0 + (uint32_t)lane, i0, S, t0, x0, y0);
      const bool h1 = locate(s0 + 64 + (uint32_t)lane, i1, S, t1, x1, y1);
      record(h0, i0, t0, x0, y0, s0, S, r, staged);
      if (s0 + 64 < S) record(h1, i1, t1, x1, y1, s0 + 64, S, r, staged);
    }
    if (!TABLE && !EMIT && lane == 0) {
      if (wave_in) counts[wslot] = pos;
      block_sum += pos;
    }
    __syncthreads();  // the counters are complete; the wavefront staging is rewritten by the next group
    if (TABLE && EMIT && staged) {
      // copy the runs out: tile t's run is [end of tile t - 1's, the last wavefront's counter of tile t).  Sixteen
      // lanes copy one run, consecutive lanes to consecutive slots, so that the list lines are written in pieces
      // of up to 64 bytes, not word by word.
      const uint32_t rank0 = (uint32_t)(lo + grp * GPG);
      const int sub = lane >> 4, sl = lane & 15;
      for (int tb = 4 * w; tb < T; tb += 16) {
        const int tt = tb + sub;
        uint32_t a = 0u, b = 0u, p0 = 0u;
        if (tt < T) {
          a = tt ? tc[4 * (tt - 1) + 3] : 0u;
          b = tc[4 * tt + 3];
          p0 = ppos[tt];
        }
        for (uint32_t k = a + (uint32_t)sl; k < b; k += 16u)
          if (p0 + (k - a) < ch.cap) vals[p0 + (k - a)] = rank0 + stage[k];
      }
      __syncthreads();
    }
    if (TABLE && !EMIT) {
      const int64_t at = tbase + grp;
      for (int tt = threadIdx.x; tt < T; tt += 256) {
        const uint4 c = tcnt_s[tt];
        counts[at + (int64_t)tt * ng] = c.x | (c.y << 8) | (c.z << 16) | (c.w << 24);
      }
      __syncthreads();
    }
  }
  if (!TABLE && !EMIT) {
    if (lane == 0) part[w] = block_sum;
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long sum = part[0] + part[1] + part[2] + part[3];
      if (sum) atomicAdd(total, sum);
    }
  }
}

// Chunk-0 layout of the table form: e0[v] = min(front[v], fcap) (the first chunk's end, where the second
// starts), base[v] = T * sum over earlier views of ng = ceil(e0 / kTableGroup) (workgroup slots), base[N] = the
// table's length.
__global__ __launch_bounds__(256) void table_setup_kernel(const uint32_t* __restrict__ front, int N, int T,
                                                          uint32_t fcap, uint32_t* __restrict__ e0,
                                                          uint32_t* __restrict__ base) {
  __shared__ uint32_t wsum[4];
  const int v = threadIdx.x, lane = v & 63, w = v >> 6;
  const uint32_t e = v < N ? min(front[v], fcap) : 0u;
  const uint32_t ng = (e + kTableGroup - 1) / kTableGroup;
  const uint32_t inc = wave_incl_scan_u32(ng, lane);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (int i = 0; i < 4; ++i) {
    if (i < w) before += wsum[i];
    tot += wsum[i];
  }
  if (v < N) {
    e0[v] = e;
    base[v] = (uint32_t)T * (before + inc - ng);
  }
  if (v == 0) base[N] = (uint32_t)T * tot;
}

// List starts from the scanned table: start[v T + t] = scanned[base_v + t ng_v] (the slot of the view's first
// group in tile t), start[N T] = the key total; *max_total = max(*max_total, key total), and *host_total = the key
// total when given (a word of host memory the host reads after synchronising).  Starts are clamped
// to the key capacity, as emission drops keys beyond it: a frame that overflows reads only written slots (and
// is reported and rendered again).
__global__ __launch_bounds__(256) void table_starts_kernel(const uint32_t* __restrict__ scanned,
                                                           const uint32_t* __restrict__ base,
                                                           const uint32_t* __restrict__ e0, int N, int T,
                                                           const uint32_t* __restrict__ grand, uint32_t cap,
                                                           unsigned long long* __restrict__ max_total,
                                                           unsigned long long* host_total,
                                                           uint32_t* __restrict__ start) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t NT = (int64_t)N * T;
  if (i > NT) return;
  const uint32_t g = *grand;
  if (i == NT) {
    start[NT] = min(g, cap);
    if (g > *max_total) *max_total = g;
    if (host_total) *host_total = g;
    return;
  }
  const int v = (int)(i / T), t = (int)(i - (int64_t)v * T);
  const int64_t ng = ((int64_t)e0[v] + kTableGroup - 1) / kTableGroup;
  const int64_t k = (int64_t)base[v] + t * ng;
  start[i] = min(k < (int64_t)base[N] ? scanned[k] : g, cap);
}

// Live tiles of each view (one workgroup per view), read by the binning of the next depth chunk.
__global__ __launch_bounds__(256) void view_live_kernel(const uint8_t* __restrict__ alive, int64_t T,
                                                         uint32_t* __restrict__ live,
                                                         unsigned long long* __restrict__ total) {
  __shared__ uint32_t part[4];
  const int v = blockIdx.x;
  if (v == 0 && threadIdx.x == 0) *total = 0;  // the next chunk's key count starts from zero
  uint32_t c = 0;
  for (int64_t t = threadIdx.x; t < T; t += 256) c += alive[(int64_t)v * T + t];
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) live[v] = part[0] + part[1] + part[2] + part[3];
}

// Start of a frame: every (view, tile) with rays is live, the front histogram and the first n_totals frame totals
// (the chunk's key count, the frame's largest, whether a later chunk is needed) are zero, and (cams given) the
// rig's cameras are built.
__global__ __launch_bounds__(256) void frame_init_kernel(uint8_t* __restrict__ alive,
                                                         const uint32_t* __restrict__ ray_off, int64_t n,
                                                         uint32_t* __restrict__ zero32, int64_t n_zero,
                                                         unsigned long long* __restrict__ totals, int n_totals,
                                                         CamRig rig, double* __restrict__ cams) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) alive[i] = ray_off ? (uint8_t)(ray_off[i + 1] > ray_off[i]) : (uint8_t)1;
  if (i < n_zero) zero32[i] = 0;
  if (i < n_totals) totals[i] = 0;
  if (cams && i < rig.n) (void)rig_camera(rig, (int)i, cams + i * kCamDoubles);
}

__global__ void fill_u64_kernel(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// Workgroups per view: enough to fill the chip for one chunk of a large scene, few enough that a chunk whose
// views are dead costs little more than its launch.
unsigned bin_blocks(const ChunkArgs& ch) { return (unsigned)std::min<int64_t>((ch.stride + 255) / 256, 96); }
// workgroups per view of the table form: one per group of the largest first chunk a view can have
unsigned table_blocks(const ChunkArgs& ch) {
  const int64_t m = ch.front_max > 0 ? ch.front_max : ch.stride;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + kTableGroup - 1) / kTableGroup, 256));
}

hipError_t launch_bin_count(const float4* rec, const uint32_t* vis_count, const uint32_t* live, const BlendConst& bc,
                            const ChunkArgs& ch, const uint8_t* alive, uint32_t* counts, unsigned long long* total,
                            hipStream_t s) {
  const dim3 grid(bin_blocks(ch), (unsigned)bc.N);
  hipLaunchKernelGGL((bin_kernel<false, false>), grid, dim3(256), 0, s, rec, vis_count, live, bc, ch, alive, counts,
                     total, nullptr, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_bin_emit(const float4* rec, const uint32_t* vis_count, const uint32_t* live, const BlendConst& bc,
                           const ChunkArgs& ch, const uint8_t* alive, const uint32_t* offsets, uint32_t* keys,
                           uint32_t* vals, hipStream_t s) {
  const dim3 grid(bin_blocks(ch), (unsigned)bc.N);
  hipLaunchKernelGGL((bin_kernel<true, false>), grid, dim3(256), 0, s, rec, vis_count, live, bc, ch, alive, nullptr,
                     nullptr, offsets, keys, vals, nullptr);
  return hipGetLastError();
}

hipError_t launch_table_setup(const uint32_t* front, int N, int T, uint32_t fcap, uint32_t* e0, uint32_t* base,
                              hipStream_t s) {
  if (N > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(table_setup_kernel, dim3(1), dim3(256), 0, s, front, N, T, fcap, e0, base);
  return hipGetLastError();
}

hipError_t launch_bin_table_count(const float4* rec, const uint32_t* vis_count, const BlendConst& bc,
                                  const ChunkArgs& ch, const uint8_t* alive, const uint32_t* base, uint32_t* table,
                                  hipStream_t s) {
  if (bc.T > kTableMaxTiles || !ch.first || !ch.front) return hipErrorInvalidValue;
  ChunkArgs c = ch;
  c.tgx = table_blocks(ch);
  const dim3 grid((unsigned)(8 * ((bc.N + 7) / 8) * c.tgx));
  hipLaunchKernelGGL((bin_kernel<false, true>), grid, dim3(256), (size_t)16 * bc.T, s, rec, vis_count, nullptr, bc, c,
                     alive, table, nullptr, nullptr, nullptr, nullptr, base);
  return hipGetLastError();
}

hipError_t launch_bin_table_emit(const float4* rec, const uint32_t* vis_count, const BlendConst& bc,
                                 const ChunkArgs& ch, const uint8_t* alive, const uint32_t* base, uint32_t* table,
                                 const uint32_t* scanned, uint32_t* vals, hipStream_t s) {
  if (bc.T > kTableMaxTiles || !ch.first || !ch.front) return hipErrorInvalidValue;
  ChunkArgs c = ch;
  c.tgx = table_blocks(ch);
  const dim3 grid((unsigned)(8 * ((bc.N + 7) / 8) * c.tgx));
  hipLaunchKernelGGL((bin_kernel<true, true>), grid, dim3(256), (size_t)20 * bc.T + kTableStage, s, rec, vis_count,
                     nullptr, bc, c, alive, table, nullptr, scanned, nullptr, vals, base);
  return hipGetLastError();
}

hipError_t launch_table_starts(const uint32_t* scanned, const uint32_t* base, const uint32_t* e0, int N, int T,
                               const uint32_t* grand, uint32_t cap, unsigned long long* max_total,
                               unsigned long long* host_total, uint32_t* start, hipStream_t s) {
  const int64_t n = (int64_t)N * T + 1;
  hipLaunchKernelGGL(table_starts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, scanned, base, e0, N, T,
                     grand, cap, max_total, host_total, start);
  return hipGetLastError();
}

hipError_t launch_view_live(const uint8_t* alive, int64_t T, int N, uint32_t* live, unsigned long long* total,
                            hipStream_t s) {
  hipLaunchKernelGGL(view_live_kernel, dim3((unsigned)N), dim3(256), 0, s, alive, T, live, total);
  return hipGetLastError();
}

hipError_t launch_frame_init(uint8_t* alive, const uint32_t* ray_off, int64_t n, uint32_t* zero32, int64_t n_zero,
                             unsigned long long* totals, int n_totals, const CamRig& rig, double* cams,
                             hipStream_t s) {
  const int64_t m = std::max<int64_t>(std::max<int64_t>(std::max<int64_t>(n, n_zero), n_totals), cams ? rig.n : 0);
  hipLaunchKernelGGL(frame_init_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, alive, ray_off, n, zero32,
                     n_zero, totals, n_totals, rig, cams);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace dl

// splat.hip -- per-bucket splat of wave-particle pairs and the blend epilogue.
//
// Each particle of bucket b is a crest +A at its position p and a trough -A
// one radius behind it, p - r_b u (the positive-negative pair of Fig 1);
// both use the separable raised cosine K(d) = w(d_x) w(d_y),
// w(d) = 1/2 (1 + cos(pi d / r_b)) = cos^2(pi d / (2 r_b)) for |d| < r_b
// (Sec 4.2: per-bucket layers smoothed by separable x and y passes; here
// evaluated at the exact particle position).  The layers are summed into the
// patch height, which is then blended with the background,
//   h = s h_WP + (1 - s) bilinear(H),  s = smoothstep(edge distance / band)
// (Sec 3.1 local replacement, smooth distance weights of Sec 4.2).
//
// Work decomposition.  The output of every patch is cut into 64x64 tiles.
// The particle scatter adds a weighted crest count per tile (cost weight per
// bucket ~ footprint area); k_splat_plan turns these loads into a number of
// parts per tile (about equal load per part, within a total item budget) and
// a prefix of work items.  k_splat is a persistent grid over the items: an
// item is one part of one tile, i.e. one of `nparts` interleaved shares of
// the particles that can reach that tile.  For each bucket it walks the
// particle bins whose crests lie within 2 r_b of the tile, which are
// contiguous runs of the bin-sorted particle buffer:
//   * small and medium radii: a group of G lanes (G ~ footprint width, a
//     power of two) takes one crest or trough; its lanes write the row
//     weights to a per-wave scratch, then own columns and add
//     A w(d_x) w(d_y) into the LDS tile with LDS float atomics;
//   * large radii (r >= dense_rc cells): the tile is a rank-K update,
//     H += W_y^T (A W_x), over batches of 32 crests/troughs whose weight
//     vectors are staged in LDS; each thread keeps a 4x4 block of the tile in
//     registers (16 FMA per item, two 16-byte LDS reads).
// A tile with one part is blended and written straight from LDS.  Parts of a
// split tile store their partial tile; k_splat_reduce (the next launch, so
// every store is visible on every XCD) sums them and runs the blend.
#include "hwo_dev.h"

namespace hwo {

namespace {

constexpr int kBatch = 16;   // dense-path items (crests + troughs) per batch
constexpr int kPad = kTile + 1;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raised cosine w(t r) for t = d / r: cos^2(pi t / 2) on |t| < 1, else 0.
// v_cos_f32 takes its argument in revolutions: cos(pi t / 2) = cos(2 pi t / 4).
__device__ __forceinline__ float wcos(float t) {
  const float c = __builtin_amdgcn_cosf(0.25f * t);
  return (fabsf(t) < 1.f) ? c * c : 0.f;
}

struct TileGeom {
  int p, i0, j0, tw, th;
  float Ab;            // boundary amplitude of the bucket being splatted
  int64_t X0, Y0;      // first cell centre (position units)
  float inv_dxu;
};

// Decode particle k: crest centre in tile cell coordinates, amplitude, direction.
template <class Rec>
__device__ __forceinline__ bool load_item(const Dev &d, const Rec *__restrict__ S, int k, int64_t n, int b,
                                          const TileGeom &T, float &cx, float &cy, float &A, float2 &u) {
  const Part q = RecIO<Rec>::load(S, k, n);
  if ((int)m_bucket(q.meta) != b || (int)m_patch(q.meta) != T.p) return false;
  const int2 v = d.V[b * kNCode + q.code];
  const int64_t px = (int64_t)q.ox + (((int64_t)q.age * v.x) >> 12);
  const int64_t py = (int64_t)q.oy + (((int64_t)q.age * v.y) >> 12);
  cx = (float)(px - T.X0) * T.inv_dxu;
  cy = (float)(py - T.Y0) * T.inv_dxu;
  A = (RecIO<Rec>::kHasAmp || m_kind(q.meta) != 0) ? particle_amp<Rec>(d, q) : T.Ab;
  u = d.UC[q.code];
  return true;
}

}  // namespace

namespace {

__device__ __forceinline__ int patch_of_tile(const Dev &d, int tile) {
  int lo = 0, hi = d.np - 1;   // last patch with tile0 <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.patches[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void tile_geom(const Dev &d, int tile, int p, TileGeom &T) {
  const PatchDev &P = d.patches[p];
  const StepPatch &W = d.sp[p];
  T.p = p;
  const int lt = tile - P.tile0;
  T.i0 = (lt % P.ntx) * kTile;
  T.j0 = (lt / P.ntx) * kTile;
  T.tw = min(kTile, P.nx - T.i0);
  T.th = min(kTile, P.ny - T.j0);
  T.X0 = ((int64_t)W.wx + T.i0) * P.dxu + P.dxu / 2;
  T.Y0 = ((int64_t)W.wy + T.j0) * P.dxu + P.dxu / 2;
  T.inv_dxu = 1.0f / (float)P.dxu;
}

// Blend one cell (tile-local i, j) and store the raw and blended heights.
__device__ __forceinline__ void blend_store(const Dev &d, const PatchDev &P, const StepPatch &W, const TileGeom &T,
                                            int i, int j, float h, float *__restrict__ raw_out,
                                            float *__restrict__ blend_out, int64_t out_off) {
  const int ci = T.i0 + i, cj = T.j0 + j;
  const size_t o = (size_t)(P.cell0 - out_off) + (size_t)cj * P.nx + ci;
  raw_out[o] = h;
  if (!blend_out) return;
  const int N = d.N;
  const float dx = (float)P.dx;
  const float dd = fminf(fminf((float)ci + 0.5f, (float)P.nx - (float)ci - 0.5f),
                         fminf((float)cj + 0.5f, (float)P.ny - (float)cj - 0.5f)) * dx;
  const float t = fminf(dd / P.band, 1.f);
  const float s = t * t * (3.f - 2.f * t);
  const float uu = W.fx0 + (float)ci * P.ratio, vv = W.fy0 + (float)cj * P.ratio;
  const float fu = floorf(uu), fv = floorf(vv);
  const float a = uu - fu, bb = vv - fv;
  const int x0 = (W.gx0 + (int)fu) & (N - 1), y0 = (W.gy0 + (int)fv) & (N - 1);
  const int x1 = (x0 + 1) & (N - 1), y1 = (y0 + 1) & (N - 1);
  const float *Hr0 = d.H + (size_t)y0 * N, *Hr1 = d.H + (size_t)y1 * N;
  const float hb = (1.f - bb) * ((1.f - a) * Hr0[x0] + a * Hr0[x1]) + bb * ((1.f - a) * Hr1[x0] + a * Hr1[x1]);
  blend_out[o] = s * h + (1.f - s) * hb;
}

}  // namespace

// ---------------------------------------------------------------- load
// One wavefront per output tile: weighted count of the particles whose bin
// origin lies in the tile (every bin belongs to exactly one tile; bins in the
// margins go to the edge tiles), read from the bin offsets of this step.
__global__ __launch_bounds__(kThreads) void k_splat_load(Dev d, int t0, int nt) {
  const int t = (int)blockIdx.x * (kThreads / 64) + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= nt) return;
  const int tile = t0 + t;
  const int p = d.tile_patch[tile];
  const PatchDev &P = d.patches[p];
  const int lt = tile - P.tile0;
  const int tx = lt % P.ntx, ty = lt / P.ntx;
  const int64_t span = (int64_t)kTile * P.dxu;
  uint64_t load = 0;
  for (int b = 0; b < d.nb; ++b) {
    const int64_t m = d.margin[b], binu = P.binu[b];
    // first bin whose origin (bin * binu - m, window frame) is at or past x
    auto first_bin = [&](int64_t x) { return (int)((x + m + binu - 1) / binu); };
    const int bx0 = tx == 0 ? 0 : min(P.nbx[b], first_bin(tx * span));
    const int bx1 = tx == P.ntx - 1 ? P.nbx[b] : min(P.nbx[b], first_bin((tx + 1) * span));
    const int by0 = ty == 0 ? 0 : min(P.nby[b], first_bin(ty * span));
    const int by1 = ty == P.nty - 1 ? P.nby[b] : min(P.nby[b], first_bin((ty + 1) * span));
    if (bx1 <= bx0) continue;
    uint32_t cnt = 0;
    for (int by = by0 + lane; by < by1; by += 64) {
      const int rb = P.binbase[b] + by * P.nbx[b];
      cnt += (uint32_t)(d.off[rb + bx1] - d.off[rb + bx0]);
    }
    load += (uint64_t)cnt * d.bcost[b];
  }
  for (int o = 32; o > 0; o >>= 1) load += __shfl_xor(load, o);
  if (lane == 0) d.tile_load[tile] = (uint32_t)min<uint64_t>(load, 0xFFFFFFFFull);
}

// ---------------------------------------------------------------- plan
// One block: parts per tile from the loads, prefix of work items.
constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void k_splat_plan(Dev d, int t0, int nt, int items_target) {
  __shared__ uint32_t s_red[kPlanThreads / 64];
  __shared__ int32_t s_cnt[kPlanThreads / 64];
  __shared__ uint32_t s_chunk;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (nt + kPlanThreads - 1) / kPlanThreads;
  const int beg = tid * per, end = min(nt, beg + per);
  uint64_t mine = 0;
  for (int t = beg; t < end; ++t) mine += d.tile_load[t0 + t];
  uint64_t tot = mine;
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
  if (lane == 0) s_red[wv] = (uint32_t)min<uint64_t>(tot, 0xFFFFFFFFull);
  __syncthreads();
  if (tid == 0) {
    uint64_t all = 0;
    for (int w = 0; w < kPlanThreads / 64; ++w) all += s_red[w];
    // sum over tiles of (1 + load / chunk) must stay within the item budget
    const int64_t room = (int64_t)d.max_items - nt;
    uint64_t chunk = d.chunk_load;
    const uint64_t by_target = (all + (uint64_t)items_target - 1) / (uint64_t)max(items_target, 1);
    if (by_target > chunk) chunk = by_target;
    if (room > 0) {
      const uint64_t by_room = (all + (uint64_t)room - 1) / (uint64_t)room;
      if (by_room > chunk) chunk = by_room;
    }
    s_chunk = (uint32_t)min<uint64_t>(chunk, 0xFFFFFFFFull);
  }
  __syncthreads();
  const uint32_t chunk = s_chunk;
  int32_t cnt = 0;
  for (int t = beg; t < end; ++t) {
    const uint32_t l = d.tile_load[t0 + t];
    cnt += min(d.max_parts, 1 + (int32_t)(l / chunk));
  }
  // exclusive scan of per-thread counts
  int32_t inc = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_cnt[wv] = inc;
  __syncthreads();
  int32_t pre = 0;
  for (int w = 0; w < wv; ++w) pre += s_cnt[w];
  int32_t acc = pre + inc - cnt;
  for (int t = beg; t < end; ++t) {
    const uint32_t l = d.tile_load[t0 + t];
    const int parts = min(d.max_parts, 1 + (int32_t)(l / chunk));
    d.item_base[t0 + t] = acc;
    for (int j = 0; j < parts; ++j)
      d.item_tile[acc + j] = ((uint32_t)(t0 + t) << 12) | ((uint32_t)j << 6) | (uint32_t)(parts - 1);
    acc += parts;
  }
  if (tid == kPlanThreads - 1) {
    d.item_base[t0 + nt] = acc;
    d.splat_ctl[1] = acc;
  }
}

// ---------------------------------------------------------------- splat
constexpr int kChunk = kThreads;   // particles decoded into LDS per step
constexpr int kMaxRows = 32;       // bin rows a tile can need per bucket

template <class Rec>
__global__ __launch_bounds__(kThreads) void k_splat(Dev d, int t0, int nt, const Rec *__restrict__ direct,
                                                    int ndirect, float *__restrict__ raw_out,
                                                    float *__restrict__ blend_out, int64_t out_off) {
  __shared__ float acc[kTile][kPad];
  __shared__ float scratch[kThreads / 64][64];
  __shared__ float4 wx4[kBatch][kTile / 4];
  __shared__ float4 wy4[kBatch][kTile / 4];
  // decoded chunk: crest centre (tile cells), amplitude, direction
  __shared__ float dc_x[kChunk], dc_y[kChunk], dc_a[kChunk], dc_ux[kChunk], dc_uy[kChunk];
  __shared__ uint16_t it_idx[2 * kChunk];    // dense items: particle | 0x8000 for the trough
  // per bucket: bin rows reaching the tile (start, exclusive prefix of lengths)
  __shared__ int s_rlo[kMaxBuckets][kMaxRows];
  __shared__ int s_pre[kMaxBuckets][kMaxRows + 1];
  __shared__ int s_nrows[kMaxBuckets];
  __shared__ int s_bstart[kMaxBuckets];      // first index of this part in the bucket's list
  __shared__ int s_boff[kMaxBuckets + 1];    // offsets of the buckets in the item's list
  __shared__ int s_wcnt[kThreads / 64];
  __shared__ int s_tile, s_part, s_nparts, s_patch;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int nwaves = kThreads / 64;
  float *scr = scratch[wave];
  const int64_t n = d.glob->n;
  const Rec *__restrict__ S = direct ? direct : (const Rec *)((n & 1) ? d.S1 : d.S0);
  const int total = direct ? nt : d.splat_ctl[1];
  const int nb = d.nb;
  // dense-path ownership: 4x4 cells per thread, wave w owns rows 16w..16w+15
  const int dc0 = 4 * (lane & 15);
  const int dr0 = 16 * wave + 4 * (lane >> 4);

  for (int item = (int)blockIdx.x; item < total; item += (int)gridDim.x) {
    if (tid == 0) {
      int tile, part, np_;
      if (direct) {
        tile = t0 + item;
        part = 0;
        np_ = 1;
      } else {
        const uint32_t e = d.item_tile[item];
        tile = (int)(e >> 12);
        part = (int)((e >> 6) & 63);
        np_ = (int)(e & 63) + 1;
      }
      s_tile = tile;
      s_part = part;
      s_nparts = np_;
      s_patch = d.tile_patch[tile];
    }
    for (int c = tid; c < kTile * kPad; c += kThreads) (&acc[0][0])[c] = 0.f;
    __syncthreads();
    const int tile = s_tile, part = s_part, nparts = s_nparts;
    TileGeom T;
    tile_geom(d, tile, s_patch, T);
    const PatchDev &P = d.patches[T.p];
    const int32_t dxu = P.dxu;
    const int64_t ax0 = (int64_t)T.i0 * dxu + dxu / 2;
    const int64_t ay0 = (int64_t)T.j0 * dxu + dxu / 2;

    // ---- row tables of every bucket, loaded in one pass
    for (int q = tid; q < nb * kMaxRows; q += kThreads) {
      const int b = q / kMaxRows, r = q % kMaxRows;
      int nrows, lo = 0, len = 0;
      if (direct) {
        nrows = 1;
        if (r == 0) len = ndirect;
      } else {
        const int32_t m = d.margin[b];
        const int32_t binu = P.binu[b];
        const int bx_lo = (int)(ax0 / binu);
        const int bx_hi = min(P.nbx[b] - 1, (int)((ax0 + (int64_t)(T.tw - 1) * dxu + 2 * (int64_t)m) / binu));
        const int by_lo = (int)(ay0 / binu);
        const int by_hi = min(P.nby[b] - 1, (int)((ay0 + (int64_t)(T.th - 1) * dxu + 2 * (int64_t)m) / binu));
        nrows = (bx_lo <= bx_hi && by_lo <= by_hi) ? min(by_hi - by_lo + 1, kMaxRows) : 0;
        if (r < nrows) {
          const int rb = P.binbase[b] + (by_lo + r) * P.nbx[b];
          lo = min(d.off[rb + bx_lo], d.cap);
          len = max(0, min(d.off[rb + bx_hi + 1], d.cap) - lo);
        }
      }
      if (r < nrows) {
        s_rlo[b][r] = lo;
        s_pre[b][r] = len;
      }
      if (r == 0) s_nrows[b] = nrows;
    }
    __syncthreads();
    // exclusive prefix of the row lengths, one bucket per wave
    for (int b = wave; b < nb; b += nwaves) {
      const int nrows = s_nrows[b];
      const int len = lane < nrows ? s_pre[b][lane] : 0;
      int inc = len;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
      }
      if (lane < nrows) s_pre[b][lane] = inc - len;
      if (lane == 63) s_pre[b][nrows] = inc;
    }
    __syncthreads();
    if (tid == 0) {
      int accum = 0;
      for (int b = 0; b < nb; ++b) {
        const int M = s_pre[b][s_nrows[b]];
        const int p0 = (int)((int64_t)M * part / nparts), p1 = (int)((int64_t)M * (part + 1) / nparts);
        s_bstart[b] = p0;
        s_boff[b] = accum;
        accum += p1 - p0;
      }
      s_boff[nb] = accum;
    }
    __syncthreads();
    const int Mi = s_boff[nb];
    float racc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) racc[i][j] = 0.f;

    for (int c = 0; c < Mi; c += kChunk) {   // block-uniform
      const int m = min(kChunk, Mi - c);
      // ---- decode: item-list index -> bucket -> bin row -> particle (one per thread)
      if (tid < m) {
        const int g = c + tid;
        int b = 0;
        while (b + 1 < nb && s_boff[b + 1] <= g) ++b;
        const int v = s_bstart[b] + (g - s_boff[b]);
        int lo = 0, hi = s_nrows[b] - 1;   // last row with prefix <= v
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[b][mid] <= v) lo = mid; else hi = mid - 1;
        }
        const int k = s_rlo[b][lo] + (v - s_pre[b][lo]);
        float cx = 0.f, cy = 0.f, A = 0.f;
        float2 u = make_float2(0.f, 0.f);
        TileGeom Tb = T;
        Tb.Ab = P.A[b];
        const bool valid = load_item<Rec>(d, S, k, n, b, Tb, cx, cy, A, u);
        dc_x[tid] = cx;
        dc_y[tid] = cy;
        dc_a[tid] = valid ? A : 0.f;
        dc_ux[tid] = u.x;
        dc_uy[tid] = u.y;
      }
      __syncthreads();
      // ---- the chunk holds runs of consecutive buckets
      for (int b = 0; b < nb; ++b) {
        const int seg_lo = max(c, s_boff[b]) - c, seg_hi = min(c + m, s_boff[b + 1]) - c;
        if (seg_hi <= seg_lo) continue;   // block-uniform
        const float rc = d.bucket_r[b] / (float)P.dx;   // radius in cells
        const float inv_rc = 1.f / rc;
        if (rc < d.dense_rc) {
          // ---- group scatter: one crest/trough per group of G lanes
          int need = (int)floorf(2.f * rc) + 1;
          int lg = 0;
          while ((1 << lg) < need && lg < 6) ++lg;
          const int G = 1 << lg, ppw = 64 >> lg;
          const int grp = lane >> lg, gl = lane & (G - 1);
          for (int i0 = seg_lo + wave * ppw; i0 < seg_hi; i0 += nwaves * ppw) {
            const int i = i0 + grp;
            const bool valid = i < seg_hi && dc_a[i] != 0.f;
            const float cx = valid ? dc_x[i] : 0.f, cy = valid ? dc_y[i] : 0.f;
            const float A = valid ? dc_a[i] : 0.f;
            const float ux = valid ? dc_ux[i] : 0.f, uy = valid ? dc_uy[i] : 0.f;
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
              const float ccx = pass ? cx - rc * ux : cx;
              const float ccy = pass ? cy - rc * uy : cy;
              const float amp = pass ? -A : A;
              int nr = 0, nc = 0, ilo = 0, jlo = 0;
              if (valid) {
                ilo = max(0, (int)ceilf(ccx - rc));
                const int ihi = min(T.tw - 1, (int)floorf(ccx + rc));
                jlo = max(0, (int)ceilf(ccy - rc));
                const int jhi = min(T.th - 1, (int)floorf(ccy + rc));
                if (ihi >= ilo && jhi >= jlo) {
                  nc = ihi - ilo + 1;
                  nr = jhi - jlo + 1;
                }
              }
              for (int jj = gl; jj < nr; jj += G) scr[grp * G + jj] = wcos(((float)(jlo + jj) - ccy) * inv_rc);
              wave_fence();
              for (int ii = gl; ii < nc; ii += G) {
                const float wxv = amp * wcos(((float)(ilo + ii) - ccx) * inv_rc);
                float *col = &acc[jlo][ilo + ii];
                const float *sw = scr + grp * G;
                int jj = 0;
                for (; jj + 4 <= nr; jj += 4) {
                  const float w0 = sw[jj], w1 = sw[jj + 1], w2 = sw[jj + 2], w3 = sw[jj + 3];
                  atomicAdd(col + (jj + 0) * kPad, wxv * w0);
                  atomicAdd(col + (jj + 1) * kPad, wxv * w1);
                  atomicAdd(col + (jj + 2) * kPad, wxv * w2);
                  atomicAdd(col + (jj + 3) * kPad, wxv * w3);
                }
                for (; jj < nr; ++jj) atomicAdd(col + jj * kPad, wxv * sw[jj]);
              }
              wave_fence();
            }
          }
        } else {
          // ---- dense rank-K update: keep only crests/troughs that overlap the tile
          int nmine = 0;
          bool oc = false, ot = false;
          if (tid >= seg_lo && tid < seg_hi && dc_a[tid] != 0.f) {
            const float cx = dc_x[tid], cy = dc_y[tid];
            const float tx = cx - rc * dc_ux[tid], ty = cy - rc * dc_uy[tid];
            oc = cx + rc >= 0.f && cx - rc <= (float)(T.tw - 1) && cy + rc >= 0.f && cy - rc <= (float)(T.th - 1);
            ot = tx + rc >= 0.f && tx - rc <= (float)(T.tw - 1) && ty + rc >= 0.f && ty - rc <= (float)(T.th - 1);
            nmine = (oc ? 1 : 0) + (ot ? 1 : 0);
          }
          int inc = nmine;
          for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
          }
          if (lane == 63) s_wcnt[wave] = inc;
          __syncthreads();
          int base = 0, nitems = 0;
          for (int w = 0; w < nwaves; ++w) {
            if (w < wave) base += s_wcnt[w];
            nitems += s_wcnt[w];
          }
          int pos = base + inc - nmine;
          if (oc) it_idx[pos++] = (uint16_t)tid;
          if (ot) it_idx[pos] = (uint16_t)(tid | 0x8000);
          __syncthreads();
          for (int ib = 0; ib < nitems; ib += kBatch) {   // block-uniform
            const int nbatch = min(kBatch, nitems - ib);
            for (int vv = tid; vv < nbatch * 2 * kTile; vv += kThreads) {
              const int it = vv / (2 * kTile), which = (vv / kTile) & 1, q = vv % kTile;
              const int e = it_idx[ib + it], pi = e & 0x7FFF;
              const bool tr = (e & 0x8000) != 0;
              if (which == 0) {
                const float ccx = tr ? dc_x[pi] - rc * dc_ux[pi] : dc_x[pi];
                const float amp = tr ? -dc_a[pi] : dc_a[pi];
                reinterpret_cast<float *>(&wx4[it][0])[q] = (q < T.tw) ? amp * wcos(((float)q - ccx) * inv_rc) : 0.f;
              } else {
                const float ccy = tr ? dc_y[pi] - rc * dc_uy[pi] : dc_y[pi];
                reinterpret_cast<float *>(&wy4[it][0])[q] = (q < T.th) ? wcos(((float)q - ccy) * inv_rc) : 0.f;
              }
            }
            __syncthreads();
            for (int it = 0; it < nbatch; ++it) {
              const float4 yv = wy4[it][dr0 >> 2];
              if (yv.x == 0.f && yv.y == 0.f && yv.z == 0.f && yv.w == 0.f) continue;
              const float4 xv = wx4[it][dc0 >> 2];
              const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
              const float ys[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
              for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) racc[i][j] = fmaf(ys[i], xs[j], racc[i][j]);
            }
            __syncthreads();
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[dr0 + i][dc0 + j] += racc[i][j];
    __syncthreads();

    if (nparts == 1) {
      const StepPatch &W = d.sp[T.p];
      for (int c = tid; c < kTile * kTile; c += kThreads) {
        const int i = c % kTile, j = c / kTile;
        if (i < T.tw && j < T.th) blend_store(d, P, W, T, i, j, acc[j][i], raw_out, blend_out, out_off);
      }
    } else {
      float *dst = d.partials + (size_t)item * (kTile * kTile);
      for (int c = tid; c < kTile * kTile; c += kThreads) dst[c] = acc[c / kTile][c % kTile];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- reduce
// Block (tile, stripe of 4 rows): sums the partial tiles of a split tile and
// runs the blend.  Tiles with a single part were finished by k_splat.
constexpr int kStripes = kTile / 4;

__global__ __launch_bounds__(kThreads) void k_splat_reduce(Dev d, int t0, int nt) {
  const int t = (int)blockIdx.x / kStripes, q = (int)blockIdx.x % kStripes;
  if (t >= nt) return;
  const int tile = t0 + t;
  const int base = d.item_base[tile], np_ = d.item_base[tile + 1] - base;
  if (np_ <= 1) return;
  TileGeom T;
  tile_geom(d, tile, d.tile_patch[tile], T);
  const PatchDev &P = d.patches[T.p];
  const StepPatch &W = d.sp[T.p];
  const int j = 4 * q + ((int)threadIdx.x >> 6), i = threadIdx.x & 63;
  const float *src = d.partials + (size_t)base * (kTile * kTile) + j * kTile + i;
  float h0 = 0.f, h1 = 0.f, h2 = 0.f, h3 = 0.f;
  int s = 0;
  for (; s + 4 <= np_; s += 4) {
    h0 += src[(size_t)(s + 0) * (kTile * kTile)];
    h1 += src[(size_t)(s + 1) * (kTile * kTile)];
    h2 += src[(size_t)(s + 2) * (kTile * kTile)];
    h3 += src[(size_t)(s + 3) * (kTile * kTile)];
  }
  for (; s < np_; ++s) h0 += src[(size_t)s * (kTile * kTile)];
  if (i < T.tw && j < T.th) blend_store(d, P, W, T, i, j, (h0 + h1) + (h2 + h3), d.raw, d.blend, 0);
}

// ---------------------------------------------------------------- launchers
void launch_splat_plan(const Dev &d, int t0, int ntiles, int items_target, hipStream_t st) {
  if (ntiles <= 0) return;
  const int wpb = kThreads / 64;
  hipLaunchKernelGGL(k_splat_load, dim3((ntiles + wpb - 1) / wpb), dim3(kThreads), 0, st, d, t0, ntiles);
  hipLaunchKernelGGL(k_splat_plan, dim3(1), dim3(kPlanThreads), 0, st, d, t0, ntiles, items_target);
}

void launch_splat_tiles(const Dev &d, int t0, int ntiles, int grid, hipStream_t st) {
  if (ntiles <= 0) return;
  if (d.compact)
    hipLaunchKernelGGL(k_splat<RecCompact>, dim3(grid), dim3(kThreads), 0, st, d, t0, ntiles,
                       (const RecCompact *)nullptr, 0, d.raw, d.blend, (int64_t)0);
  else
    hipLaunchKernelGGL(k_splat<RecWide>, dim3(grid), dim3(kThreads), 0, st, d, t0, ntiles, (const RecWide *)nullptr,
                       0, d.raw, d.blend, (int64_t)0);
}

void launch_splat_reduce(const Dev &d, int t0, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_splat_reduce, dim3(kStripes * ntiles), dim3(kThreads), 0, st, d, t0, ntiles);
}

void launch_splat_direct(const Dev &d, int t0, int ntiles, const void *recs, int n, float *raw, int64_t out_off,
                         hipStream_t st) {
  if (ntiles <= 0) return;
  if (d.compact)
    hipLaunchKernelGGL(k_splat<RecCompact>, dim3(ntiles), dim3(kThreads), 0, st, d, t0, ntiles,
                       (const RecCompact *)recs, n, raw, (float *)nullptr, out_off);
  else
    hipLaunchKernelGGL(k_splat<RecWide>, dim3(ntiles), dim3(kThreads), 0, st, d, t0, ntiles, (const RecWide *)recs, n,
                       raw, (float *)nullptr, out_off);
}

}  // namespace hwo

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
// k_splat_load estimates each tile's cost from the particles its items will
// visit (bin offsets of this step, weighted by path); k_splat_plan corrects
// the estimates by the time each tile took in the previous frame and turns
// them into a number of parts per tile (about equal cost per part, within a
// total item budget) and a prefix of work items (k_bin_plan does the scan,
// the estimates and the plan in one block for small scenes).  k_splat is a
// grid over the
// items: an item is one part of one tile.  Each bucket's list of particles
// that can reach the tile is dealt to its parts by record line: the
// particle buffer is cut into aligned blocks of kSplit records (one 128-byte
// line of 16-byte records) and part j of `nparts` takes the entries in blocks
// whose index is j modulo nparts.  Every part samples the whole tile, so its
// four quadrants get about equal work (contiguous shares gave each part a
// band of bin rows), and every record line is fetched by one part only.  That
// list is the bins whose crests lie within 2 r_b of the tile, contiguous runs
// of the bin-sorted particle buffer.  The wavefronts of the block take
// batches of 64 list entries and work independently (the kernel's own
// comment has the schedule): each lane decodes one record into a crest and
// a trough point in tile cells, and the batch goes through one of two paths:
//   * footprints of at most kAtomicSpan cells per axis: each lane adds its
//     two points, weights in registers, A w(d_x) w(d_y) into the LDS tile
//     with LDS float atomics;
//   * larger footprints: the separable kernel makes the tile a sum of outer
//     products, H += W_y^T (A W_x).  For each 32x32 quadrant some point of
//     the batch reaches, the points are fed two at a time to a 32x32x2 FP32
//     matrix-core product into the wavefront's accumulator of that quadrant;
//     every lane computes the one row weight and the one column weight it
//     supplies.  The four accumulators of every wavefront are added to the
//     LDS tile at the end of the item.
// Two more schedules of the same items follow k_splat: k_splat_q (the block
// decodes records into LDS and each wavefront owns one quadrant) and
// k_splat_h, the default, which runs each item's small-footprint buckets as
// k_splat does and then its large-footprint buckets as k_splat_q does.
// A tile with one part is blended and written straight from LDS.  Parts of a
// split tile store their partial tile; k_splat_reduce (the next launch, so
// every store is visible on every XCD) sums them and runs the blend.
#include "hwo_dev.h"

namespace hwo {

namespace {

// Row stride of the LDS tile: 72 words puts the 8 x 8 cells of a small bin on
// distinct banks (bank = 8 row + column), where the small-footprint atomics of
// a wavefront (points sorted by bin) cluster.
constexpr int kPad = kTile + 8;

// Raised cosine w(t r) for t = d / r: cos^2(pi t / 2) on |t| < 1, else 0.
// v_cos_f32 takes its argument in revolutions: cos(pi t / 2) = cos(2 pi t / 4).
// Evaluated from q = d / (4 r), the distance in revolutions of the cosine.
__device__ __forceinline__ float wrev(float q) {
  const float c = __builtin_amdgcn_cosf(q);
  return (fabsf(q) < 0.25f) ? c * c : 0.f;
}

}  // namespace


// ---------------------------------------------------------------- load
// Relative cost of one particle visit (decode plus footprint work) by path:
// per-lane atomics with 4 or 8 cells per axis, or the matrix-core quadrants.
// Ratios fitted to measured item times (about 1 : 2 : 3.5).
constexpr uint32_t kCostSmall4 = 4, kCostSmall8 = 8, kCostMatrix = 14;
// Footprints of at most this many cells per axis go through LDS atomics;
// larger ones through the matrix cores.  An LDS float atomic costs about one
// lane per clock of the CU's LDS, so from about 20 cells per footprint on
// the outer products (one weight per lane per point and quadrant plus half
// a 32x32x2 product) are cheaper.
constexpr int kAtomicSpan = 4;

__device__ __forceinline__ uint32_t visit_cost(float rc) {
  const int span = (int)floorf(2.f * rc) + 1;
  return span <= 3 ? kCostSmall4 : (span <= kAtomicSpan ? kCostSmall8 : kCostMatrix);
}

// One wavefront per output tile: estimated splat cost of the tile, the
// particles its work items will visit (the bins within 2 r of the tile, per
// bucket, read from the bin offsets of this step) weighted by visit cost.
constexpr int kMaxRows = 32;       // bin rows a tile can need per bucket

// The loads go out in two rounds: lane b reads bucket b's bin rectangle and
// tables, then every (bucket, row) pair of the tile reads its two offsets,
// all before any is used.
__global__ __launch_bounds__(kThreads) void k_splat_load(Dev d, int t0, int nt) {
  const int t = (int)blockIdx.x * (kThreads / 64) + ((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= nt) return;
  const int tile = t0 + t;
  const PatchDev &P = d.patches[d.tile_patch[tile]];
  const int nb = d.nb;
  int rxy = 0, rzw = 0, base = 0, nbx = 0;
  uint32_t cost = 0;
  if (lane < nb) {
    const short4 rc = d.tile_rect[(size_t)tile * nb + lane];
    rxy = (int)(uint16_t)rc.x | ((int)(uint16_t)rc.y << 16);
    rzw = (int)(uint16_t)rc.z | ((int)(uint16_t)rc.w << 16);
    base = P.binbase[lane];
    nbx = P.nbx[lane];
    cost = visit_cost(d.bucket_r[lane] / (float)P.dx);
  }
  constexpr int kPer = kMaxBuckets * kMaxRows / 64;   // (bucket, row) pairs per lane
  int lo[kPer], hi[kPer];
  uint32_t cw[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int q = lane + 64 * k;
    const int b = q / kMaxRows, r = q % kMaxRows;
    const int xy = __shfl(rxy, b & 63), zw = __shfl(rzw, b & 63);
    const int bb = __shfl(base, b & 63), bn = __shfl(nbx, b & 63);
    cw[k] = (uint32_t)__shfl((int)cost, b & 63);
    lo[k] = 0;
    hi[k] = 0;
    if (b < nb && r < (int)((uint32_t)zw >> 16)) {
      const int rb = bb + ((zw & 0xFFFF) + r) * bn;
      lo[k] = d.off[rb + (xy & 0xFFFF)];
      hi[k] = d.off[rb + (int)((uint32_t)xy >> 16) + 1];
    }
  }
  uint64_t load = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    load += (uint64_t)(uint32_t)max(0, min(hi[k], d.cap) - min(lo[k], d.cap)) * cw[k];
  for (int o = 32; o > 0; o >>= 1) load += __shfl_xor(load, o);
  if (lane == 0) d.tile_load[tile] = (uint32_t)min<uint64_t>(load, 0xFFFFFFFFull);
}

// ---------------------------------------------------------------- plan
// One block: parts per tile from the loads, prefix of work items.
constexpr int kPlanThreads = 1024;
constexpr int kPlanLdsTiles = 8192;   // tiles whose item prefix fits in LDS for the parallel fill
constexpr int kFusedMaxTiles = 1024;  // tiles of a scene that k_bin_plan handles (one per thread)
constexpr int kFusedMaxBins = 16384;  // bins of a scene that k_bin_plan handles (offsets held in LDS)

// Body of the plan, run by one block of kPlanThreads threads; load[t] is the
// model cost estimate of tile t0 + t (global memory or LDS).  It is first
// corrected by the splat time measured for the tile in the previous frame:
// each tile keeps a running average of (measured / estimated) relative to the
// whole scene, and load[t] is scaled by it in place.  meas, model and ratio
// are that state for tiles t0.. as read at the start (global memory or an LDS
// copy); the updated state is written to global memory.
__device__ void plan_items(const Dev &d, int t0, int nt, int items_target, uint32_t *load, const uint32_t *meas,
                           const uint32_t *model, const float *ratio) {
  __shared__ uint64_t s_red[kPlanThreads / 64];
  __shared__ uint64_t s_red2[kPlanThreads / 64];
  __shared__ float s_gm;
  __shared__ int32_t s_cnt[kPlanThreads / 64];
  __shared__ int32_t s_nsp[kPlanThreads / 64];
  __shared__ uint32_t s_chunk;
  __shared__ int32_t s_base[kPlanLdsTiles];
  __shared__ int32_t s_total;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (nt + kPlanThreads - 1) / kPlanThreads;
  const int beg = tid * per, end = min(nt, beg + per);
  // ---- feedback from the previous frame
  {
    uint64_t ms = 0, es = 0;
    for (int t = beg; t < end; ++t) {
      const uint32_t m = meas[t], e = model[t];
      if (m && e) {
        ms += m;
        es += e;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      ms += __shfl_xor(ms, o);
      es += __shfl_xor(es, o);
    }
    if (lane == 0) {
      s_red[wv] = ms;
      s_red2[wv] = es;
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t am = 0, ae = 0;
      for (int w = 0; w < kPlanThreads / 64; ++w) {
        am += s_red[w];
        ae += s_red2[w];
      }
      s_gm = (am && ae) ? (float)((double)am / (double)ae) : 0.f;
    }
    __syncthreads();
    const float gm = s_gm;
    for (int t = beg; t < end; ++t) {
      const uint32_t m = meas[t], e = model[t];
      float r = ratio[t];
      if (gm > 0.f && m && e) r = fminf(4.f, fmaxf(0.25f, 0.5f * r + 0.5f * ((float)m / (float)e) / gm));
      d.tile_ratio[t0 + t] = r;
      d.tile_meas[t0 + t] = 0;
      d.tile_model[t0 + t] = load[t];
      load[t] = (uint32_t)fminf(4.0e9f, (float)load[t] * r);
    }
    __syncthreads();
  }
  uint64_t mine = 0;
  for (int t = beg; t < end; ++t) mine += load[t];
  uint64_t tot = mine;
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
  if (lane == 0) s_red[wv] = tot;
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
  int32_t cnt = 0, nsp = 0;   // items and split tiles of this thread's tiles
  for (int t = beg; t < end; ++t) {
    const uint32_t l = load[t];
    cnt += 1 + (int32_t)(l / chunk);
    nsp += l >= chunk ? 1 : 0;
  }
  // exclusive scans of the per-thread counts
  int32_t inc = cnt, inc_s = nsp;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o), ys = __shfl_up(inc_s, o);
    if (lane >= o) {
      inc += y;
      inc_s += ys;
    }
  }
  if (lane == 63) {
    s_cnt[wv] = inc;
    s_nsp[wv] = inc_s;
  }
  __syncthreads();
  int32_t pre = 0, pre_s = 0;
  for (int w = 0; w < wv; ++w) {
    pre += s_cnt[w];
    pre_s += s_nsp[w];
  }
  int32_t acc = pre + inc - cnt, sp = pre_s + inc_s - nsp;
  const bool in_lds = nt <= kPlanLdsTiles;
  for (int t = beg; t < end; ++t) {
    const uint32_t l = load[t];
    const int parts = 1 + (int32_t)(l / chunk);
    d.item_base[t0 + t] = acc;
    if (parts > 1) d.split_tiles[sp++] = t0 + t;
    if (in_lds) s_base[t] = acc;
    else
      for (int j = 0; j < parts; ++j) d.item_desc[acc + j] = make_int4(t0 + t, j, parts, d.tile_patch[t0 + t]);
    acc += parts;
  }
  if (tid == kPlanThreads - 1) {
    d.item_base[t0 + nt] = acc;
    d.splat_ctl[1] = acc;
    d.splat_ctl[2] = sp;
    s_total = acc;
  }
  if (!in_lds) return;
  __syncthreads();
  // every thread fills items: tile = last tile whose first item is <= item
  const int total = s_total;
  for (int it = tid; it < total; it += kPlanThreads) {
    int lo = 0, hi = nt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_base[mid] <= it) lo = mid; else hi = mid - 1;
    }
    const int next = lo + 1 < nt ? s_base[lo + 1] : total;
    d.item_desc[it] = make_int4(t0 + lo, it - s_base[lo], next - s_base[lo], d.tile_patch[t0 + lo]);
  }
}

__global__ __launch_bounds__(kPlanThreads) void k_splat_plan(Dev d, int t0, int nt, int items_target) {
  plan_items(d, t0, nt, items_target, d.tile_load + t0, d.tile_meas + t0, d.tile_model + t0, d.tile_ratio + t0);
}

// Small scenes, one block: exclusive scan of the bin histogram (offsets,
// cursors, cleared histogram, totals), then the cost estimate of every tile
// from the new offsets, then the plan.  Replaces the two scan launches, the
// load launch and the plan launch when all bins and tiles fit one block.
// The histogram is staged in LDS with coalesced loads (several in flight per
// thread) and scanned there, so the estimates read the offsets from LDS
// rather than back from memory.
__global__ __launch_bounds__(kPlanThreads) void k_bin_plan(Dev d, int nbins, int nt, int items_target) {
  __shared__ uint32_t s_load[kFusedMaxTiles];
  __shared__ uint32_t s_meas[kFusedMaxTiles], s_model[kFusedMaxTiles];
  __shared__ float s_ratio[kFusedMaxTiles];
  __shared__ int32_t s_off[kFusedMaxBins + 1];
  __shared__ int32_t s_w[kPlanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // Every load the block needs is issued here, in one round: the histogram,
  // the previous frame's state of the tiles (one tile per thread) and the
  // geometry of the (tile, bucket) pair whose estimate this thread makes.
  const int nb = d.nb;
  const bool est = tid < nt * nb;   // nt * nb <= kPlanThreads (bin_plan_fits)
  int e_t = 0, e_base = 0, e_nbx = 0;
  short4 e_rc = make_short4(0, 0, 0, 0);
  uint32_t e_cost = 0;
  if (est) {
    const int b = tid % nb;
    e_t = tid / nb;
    const PatchDev &P = d.patches[d.tile_patch[e_t]];
    e_rc = d.tile_rect[(size_t)e_t * nb + b];
    e_base = P.binbase[b];
    e_nbx = P.nbx[b];
    e_cost = visit_cost(d.bucket_r[b] / (float)P.dx);
  }
  if (tid < nt) {
    s_meas[tid] = d.tile_meas[tid];
    s_model[tid] = d.tile_model[tid];
    s_ratio[tid] = d.tile_ratio[tid];
    s_load[tid] = 0;
  }
#pragma unroll 8
  for (int i = tid; i < nbins; i += kPlanThreads) s_off[i] = d.hist[i];
  __syncthreads();
  // ---- scan: each thread a run of consecutive bins, in place; an odd run
  //      length keeps the threads of a wavefront on distinct LDS banks
  const int per = ((nbins + kPlanThreads - 1) / kPlanThreads) | 1;
  const int beg = min(nbins, tid * per), end = min(nbins, beg + per);
  int32_t sum = 0;
  for (int i = beg; i < end; ++i) sum += s_off[i];
  int32_t inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  int32_t acc = inc - sum;
  for (int w = 0; w < wv; ++w) acc += s_w[w];
  for (int i = beg; i < end; ++i) {
    const int32_t v = s_off[i];
    s_off[i] = acc;
    acc += v;
  }
  if (tid == kPlanThreads - 1) {
    s_off[nbins] = acc;
    d.glob->total = acc;
    d.glob->n_live = min(acc, d.cap);
  }
  __syncthreads();
  for (int i = tid; i <= nbins; i += kPlanThreads) {
    const int32_t v = s_off[i];
    d.off[i] = v;
    if (i < nbins) {
      d.cur[i] = v;
      d.hist[i] = 0;
    }
  }
  // ---- tile cost estimates: one (tile, bucket) pair per thread, from LDS
  if (est) {
    uint32_t seen = 0;
    for (int r = 0; r < e_rc.w; ++r) {
      const int rb = e_base + (e_rc.z + r) * e_nbx;
      seen += (uint32_t)max(0, min(s_off[rb + e_rc.y + 1], d.cap) - min(s_off[rb + e_rc.x], d.cap));
    }
    if (seen) atomicAdd(&s_load[e_t], seen * e_cost);
  }
  __syncthreads();
  plan_items(d, 0, nt, items_target, s_load, s_meas, s_model, s_ratio);
}

// ---------------------------------------------------------------- splat
constexpr int kSplit = 8;          // records per aligned block when a tile's lists are dealt to its parts

// Entries of part j of np among the record indices [0, x): those in the
// aligned kSplit-blocks whose block index is j modulo np.
__device__ __forceinline__ int part_count(int x, int j, int np) {
  const int span = kSplit * np;
  return x / span * kSplit + min(kSplit, max(0, x % span - kSplit * j));
}
// Record index of the k-th entry (from 0) of part j of np; inverse of part_count.
__device__ __forceinline__ int part_entry(int k, int j, int np) {
  return k / kSplit * (kSplit * np) + kSplit * j + k % kSplit;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Largest of v (clamped to 0..F) over the wavefront's lanes: a wave-uniform
// loop bound held in a scalar register.
template <int F>
__device__ __forceinline__ int wave_max_upto(int v) {
  int m = 0;
#pragma unroll
  for (int u = 1; u <= F; ++u) m += __ballot(v >= u) != 0ull;
  return m;
}

// Small footprints (at most F cells per axis): one crest or trough per lane,
// weights in registers, LDS float atomics into the tile.  The loops run to
// the wavefront's largest column and row counts, found once per point.
template <int F>
__device__ __forceinline__ void splat_points(float (*acc)[kPad], const float4 pv, bool valid, float rc, float qs,
                                             int tw, int th) {
  int ilo = 0, jlo = 0, nc = 0, nr = 0;
  if (valid && pv.z != 0.f) {
    ilo = max(0, (int)ceilf(pv.x - rc));
    jlo = max(0, (int)ceilf(pv.y - rc));
    nc = min(F, min(tw - 1, (int)floorf(pv.x + rc)) - ilo + 1);
    nr = min(F, min(th - 1, (int)floorf(pv.y + rc)) - jlo + 1);
  }
  const int ncw = wave_max_upto<F>(nc), nrw = wave_max_upto<F>(nr);
  // offsets of the first column and row from the centre (cells), then
  // q = offset / (4 r) per cell
  const float dx0 = (float)ilo - pv.x, dy0 = (float)jlo - pv.y;
  float wx[F];
#pragma unroll
  for (int u = 0; u < F; ++u) {
    wx[u] = 0.f;
    if (u < ncw) wx[u] = pv.z * wrev((dx0 + (float)u) * qs);
  }
#pragma unroll
  for (int jj = 0; jj < F; ++jj) {
    if (jj >= nrw) break;
    const float wy = wrev((dy0 + (float)jj) * qs);
    float *row = &acc[min(jlo + jj, kTile - 1)][ilo];
    const bool rok = jj < nr;
#pragma unroll
    for (int ii = 0; ii < F; ++ii) {
      if (ii >= ncw) break;
      if (rok && ii < nc) atomicAdd(row + ii, wy * wx[ii]);
    }
  }
}

// Radial kernel W(|d|), small footprints: as splat_points, one point per lane,
// the weight of each cell from its distance to the point.
template <int F>
__device__ __forceinline__ void splat_points_radial(float (*acc)[kPad], const float4 pv, bool valid, float rc,
                                                    float qs, int tw, int th) {
  int ilo = 0, jlo = 0, nc = 0, nr = 0;
  if (valid && pv.z != 0.f) {
    ilo = max(0, (int)ceilf(pv.x - rc));
    jlo = max(0, (int)ceilf(pv.y - rc));
    nc = min(F, min(tw - 1, (int)floorf(pv.x + rc)) - ilo + 1);
    nr = min(F, min(th - 1, (int)floorf(pv.y + rc)) - jlo + 1);
  }
  const int ncw = wave_max_upto<F>(nc), nrw = wave_max_upto<F>(nr);
  const float dx0 = (float)ilo - pv.x, dy0 = (float)jlo - pv.y;
#pragma unroll
  for (int jj = 0; jj < F; ++jj) {
    if (jj >= nrw) break;
    const float dy = dy0 + (float)jj;
    float *row = &acc[min(jlo + jj, kTile - 1)][ilo];
    const bool rok = jj < nr;
#pragma unroll
    for (int ii = 0; ii < F; ++ii) {
      if (ii >= ncw) break;
      const float dx = dx0 + (float)ii;
      const float w = wrev(__builtin_amdgcn_sqrtf(dx * dx + dy * dy) * qs);
      if (rok && ii < nc && w != 0.f) atomicAdd(row + ii, pv.z * w);
    }
  }
}

// Footprint of radius rc (cells) centred at (x, y) reaches the 32 x 32
// quadrant with first cell (xq, yq): some cell centre lies within rc on both axes.
__device__ __forceinline__ bool reaches(float x, float y, float rc, int xq, int yq) {
  return x - rc < (float)(xq + 31) && x + rc > (float)xq && y - rc < (float)(yq + 31) && y + rc > (float)yq;
}

// Add a quadrant accumulator (the matrix-core output layout: lane l holds
// column xq + l % 32 of rows yq + 8 (r / 4) + 4 (l / 32) + r % 4) to the tile.
__device__ __forceinline__ void flush_quadrant(float (*acc)[kPad], const f32x16 &cq, int xq, int yq, int lane) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = yq + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    atomicAdd(&acc[row][xq + (lane & 31)], cq[r]);
  }
}

constexpr int kBatch = 64;   // list entries a wavefront takes at a time, one per lane

// A record's decode in two halves, so that its table loads can be in flight
// while the wavefront splats the previous batch: dec_load unpacks the record
// and issues the loads (velocity and unit direction of its code, amplitude
// factor), dec_point does the arithmetic once they have arrived.
struct DecIn {
  int32_t ox, oy, age;
  int2 v;          // velocity per step of the code (2^-32 m)
  int32_t code;    // direction code (its unit vector is computed, not loaded)
  float f;         // amplitude (wide form), ring amplitude B m, or the stratified direction factor
  uint32_t flags;  // bit 0 valid, bit 1 ring particle, bits 2-4 level
};

template <class Rec>
__device__ __forceinline__ DecIn dec_load(const Dev &d, const Rec &r, int64_t n, int b, int patch, bool valid) {
  DecIn o;
  o.ox = 0; o.oy = 0; o.age = 0;
  o.v = make_int2(0, 0);
  o.code = 0;
  o.f = 1.f;
  o.flags = 0u;
  if (!valid) return o;
  const Part q = RecIO<Rec>::unpack(r, n);
  if ((int)m_bucket(q.meta) != b || (int)m_patch(q.meta) != patch) return o;
  const bool ring = m_kind(q.meta) != 0;
  const bool heave = m_heave(q.meta);
  o.flags = 1u | (ring ? 2u : 0u) | (m_level(q.meta) << 2) | (heave ? 32u : 0u) | (m_src(q.meta) << 8);
  o.ox = q.ox;
  o.oy = q.oy;
  o.age = q.age;
  o.v = velocity(d, b, q.code, !ring);
  o.code = q.code;
  if (RecIO<Rec>::kHasAmp) o.f = q.amp;
  else if (heave) o.f = 0.f;   // computed from the source's motion in dec_point
  else if (ring) o.f = d.ring_amp[m_src(q.meta) * kMaxRing + m_slot(q.meta)];
  else if (d.afac) o.f = d.afac[b * kNCode + q.code];
  return o;
}

// Crest (cx, cy) in tile cells and signed amplitude A (0: nothing to splat);
// the trough lies rc u behind the crest.  The offset of a particle of the
// sorted buffer from the tile's first cell centre is less than 2^31 position
// units (the library rejects windows plus survival margins of 2^31 units or
// more), so it is formed modulo 2^32 from the low words, which is exact and
// needs one conversion instruction; caller-supplied records (`wide`) can lie
// anywhere and take the 64-bit path.
template <class Rec>
__device__ __forceinline__ void dec_point(const Dev &d, int64_t n, const DecIn &i, const TileGeom &T, float Ab,
                                          float &cx, float &cy, float &A, bool wide) {
  if (wide) {
    const int64_t px = (int64_t)i.ox + (((int64_t)i.age * i.v.x) >> 12);
    const int64_t py = (int64_t)i.oy + (((int64_t)i.age * i.v.y) >> 12);
    cx = (float)(px - T.X0) * T.inv_dxu;
    cy = (float)(py - T.Y0) * T.inv_dxu;
  } else {
    const uint32_t mx = (uint32_t)(((int64_t)i.age * i.v.x) >> 12);
    const uint32_t my = (uint32_t)(((int64_t)i.age * i.v.y) >> 12);
    cx = (float)(int32_t)((uint32_t)i.ox + mx - (uint32_t)T.X0) * T.inv_dxu;
    cy = (float)(int32_t)((uint32_t)i.oy + my - (uint32_t)T.Y0) * T.inv_dxu;
  }
  const uint32_t lv = (i.flags >> 2) & 7u;
  const float inv3 = lv == 0 ? 1.f : lv == 1 ? 1.f / 3.f : lv == 2 ? 1.f / 9.f : lv == 3 ? 1.f / 27.f : 1.f / 81.f;
  if (!(i.flags & 1u)) A = 0.f;
  else if (RecIO<Rec>::kHasAmp) A = i.f;
  else if (i.flags & 32u) A = heave_amp(d.sources[(i.flags >> 8) & 127u], n - i.age, lv);
  else if (i.flags & 2u) A = i.f * inv3;
  else A = Ab * i.f;
}

// Next point of a batch from the wave-uniform masks of crests (0..63) and
// troughs (64..127) still to do; -1 when both are empty.
__device__ __forceinline__ int pop_point(uint64_t &m0, uint64_t &m1) {
  const bool c = m0 != 0ull;
  const uint64_t m = c ? m0 : m1;
  const int kk = m ? __builtin_ctzll(m) + (c ? 0 : kBatch) : -1;
  const uint64_t rest = m & (m - 1ull);
  m0 = c ? rest : m0;
  m1 = c ? m1 : rest;
  return kk;
}

// kRadial selects the radial kernel W(|d|) and kProf the per-bucket profile;
// both are template parameters so that the default instance carries neither.
// Each work item (one part of one output tile) is processed as follows.  The
// block loads the bin rows of every bucket that reach the tile and cuts each
// bucket's list (this part's share) into batches of 64 entries, ordered from
// the largest radii down.  Wavefront w takes batches w, w + 4, w + 8, ...
// and works independently: every lane loads and decodes one record into a
// crest and a trough point (three batches are in flight: the records of
// batch k + 2 load while the table loads of batch k + 1 and the splat of
// batch k run), and the batch goes through one of two paths into the LDS
// tile:
//   * footprints of at most kAtomicSpan cells per axis: each lane adds its
//     two points cell by cell with LDS float atomics, weights in registers;
//   * larger footprints: for each 32 x 32 quadrant of the tile that some of
//     the batch's points reach, the points (read from their lanes'
//     registers) are fed two at a time to a 32x32x2 FP32 matrix-core product
//     (rank-2 update W_y^T (A W_x), each lane computing the one row and one
//     column weight it supplies) into the wavefront's accumulator of that
//     quadrant, which stays in registers until the item is done.
// There is no barrier between batches, so no wavefront waits for another
// until the item's list is exhausted.
template <class Rec, bool kRadial, bool kProf>
// At most 168 registers per lane (the four quadrant accumulators take 64):
// three wavefronts per SIMD (three blocks per CU).
__global__ __launch_bounds__(kThreads, 3) void k_splat(Dev d, int t0, int nt, const Rec *__restrict__ direct,
                                                    int ndirect, float *__restrict__ raw_out,
                                                    float *__restrict__ blend_out, int64_t out_off) {
  __shared__ __align__(16) float acc[kTile][kPad];
  // per bucket: bin rows reaching the tile (this part's entries before the
  // row's first record, exclusive prefix of this part's entries in the rows)
  __shared__ int s_rlo[kMaxBuckets][kMaxRows];
  __shared__ int s_pre[kMaxBuckets][kMaxRows + 1];
  __shared__ int s_nrows[kMaxBuckets];
  __shared__ int s_cnt[kMaxBuckets];          // entries of this part in each bucket's list
  __shared__ int s_bat[kMaxBuckets + 1];      // first batch of the j-th bucket taken (bucket nb - 1 - j)
  __shared__ int s_tile, s_part, s_nparts, s_patch;
  __shared__ unsigned long long s_prof[kProf ? PROF_N : 1];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t n = d.glob->n;
  const Rec *__restrict__ S = direct ? direct : (const Rec *)((n & 1) ? d.S1 : d.S0);
  const int total = direct ? nt : d.splat_ctl[1];
  const int nb = d.nb;
  // profile: each wavefront charges the clock ticks since its last mark to a
  // category (the wait for the clock read also drains its LDS operations, so
  // a batch's atomics are charged to its bucket)
  uint64_t t_mark = 0;
  auto mark = [&](int cat) {
    if constexpr (kProf) {
      const uint64_t now = __builtin_amdgcn_s_memtime();
      if (lane == 0) atomicAdd(&s_prof[cat], (unsigned long long)(now - t_mark));
      t_mark = now;
    }
  };
  if constexpr (kProf)
    for (int i = tid; i < PROF_N; i += kThreads) s_prof[i] = 0ull;

  for (int item = (int)blockIdx.x; item < total; item += (int)gridDim.x) {
    if constexpr (kProf) t_mark = __builtin_amdgcn_s_memtime();
    if (tid == 0) {
      const int4 e = direct ? make_int4(t0 + item, 0, 1, d.tile_patch[t0 + item]) : d.item_desc[item];
      s_tile = e.x;
      s_part = e.y;
      s_nparts = e.z;
      s_patch = e.w;
    }
    for (int c = tid; c < kTile * kPad / 4; c += kThreads)
      reinterpret_cast<float4 *>(&acc[0][0])[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int tile = s_tile, part = s_part, nparts = s_nparts;
    TileGeom T;
    tile_geom(d, tile, s_patch, T);
    const PatchDev &P = d.patches[T.p];
    // ---- row tables of every bucket, loaded in one pass
    for (int q = tid; q < nb * kMaxRows; q += kThreads) {
      const int b = q / kMaxRows, r = q % kMaxRows;
      int nrows, lo = 0, len = 0;
      if (direct) {
        nrows = 1;
        if (r == 0) len = ndirect;
      } else {
        const short4 rc4 = d.tile_rect[(size_t)tile * nb + b];
        nrows = rc4.w;
        if (r < nrows) {
          const int rb = P.binbase[b] + (rc4.z + r) * P.nbx[b];
          const int a = min(d.off[rb + rc4.x], d.cap);
          const int e = max(a, min(d.off[rb + rc4.y + 1], d.cap));
          lo = part_count(a, part, nparts);
          len = part_count(e, part, nparts) - lo;
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
    for (int b = wave; b < nb; b += kThreads / 64) {
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
    if (wave == 0) {
      // lane j: the j-th bucket in processing order (largest radii first)
      int cnt = 0;
      if (lane < nb) {
        const int b = nb - 1 - lane;
        cnt = s_pre[b][s_nrows[b]];   // this part's entries in the bucket's list
        s_cnt[b] = cnt;
      }
      const int nbj = (cnt + kBatch - 1) / kBatch;
      int inc = nbj;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
      }
      if (lane < nb) s_bat[lane] = inc - nbj;
      if (lane == nb - 1) s_bat[nb] = inc;
    }
    __syncthreads();
    mark(PROF_SETUP);
    // the batch table in registers (lane j: the j-th bucket taken), so that
    // finding a batch's bucket costs no LDS access
    const int bat_lo = lane < nb ? s_bat[lane] : 0x7FFFFFFF;
    const int bat_cnt = lane < nb ? s_cnt[nb - 1 - lane] : 0;
    const int nbat = s_bat[nb];
    const uint64_t t_work = __builtin_amdgcn_s_memrealtime();   // 100 MHz

    // batch k -> bucket and first entry (wavefront w takes batches w, w + 4, ...)
    auto locate = [&](int k, int &b, int &cnt) {
      // j-th bucket taken: the last one whose first batch is at or before k
      // (a bucket without batches starts where the next one does)
      const int j = __popcll(__ballot(bat_lo <= k)) - 1;
      b = nb - 1 - j;
      const int e0 = (k - __builtin_amdgcn_readlane(bat_lo, j)) * kBatch;
      cnt = min(kBatch, __builtin_amdgcn_readlane(bat_cnt, j) - e0);
      return e0;
    };
    // the lane's record of a batch: list entry -> this part's block -> bin row -> particle
    auto fetch = [&](int b, int e0, int cnt, Rec &rec) {
      if (lane < cnt) {
        const int v = e0 + lane;   // this part's v-th entry of the bucket's list
        int lo = 0, hi = s_nrows[b] - 1;   // last row with prefix <= v
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[b][mid] <= v) lo = mid; else hi = mid - 1;
        }
        rec = S[part_entry(s_rlo[b][lo] + (v - s_pre[b][lo]), part, nparts)];
      }
    };

    // the wavefront's matrix-core accumulators of the four quadrants, added to
    // the tile once the item's lists are done
    f32x16 cq0, cq1, cq2, cq3;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      cq0[r] = 0.f;
      cq1[r] = 0.f;
      cq2[r] = 0.f;
      cq3[r] = 0.f;
    }
    uint32_t touched = 0;   // quadrants this wavefront's accumulators hold
    // Three batches are in flight per wavefront: the records of batch k + 2
    // load while the table loads of batch k + 1 and the splat of batch k run.
    constexpr int kWaves = kThreads / 64;
    int k0 = wave, b0 = 0, c0 = 0;
    Rec r0, r1;
    if (k0 < nbat) {
      const int e0 = locate(k0, b0, c0);
      fetch(b0, e0, c0, r0);
    }
    int k1 = wave + kWaves, b1 = 0, c1 = 0;
    if (k1 < nbat) {
      const int e0 = locate(k1, b1, c1);
      fetch(b1, e0, c1, r1);
    }
    DecIn in0 = dec_load<Rec>(d, r0, n, b0, T.p, k0 < nbat && lane < c0);
    while (k0 < nbat) {   // wave-uniform
      const int k2 = k1 + kWaves;
      int b2 = 0, c2 = 0;
      Rec r2;
      if (k2 < nbat) {
        const int e0 = locate(k2, b2, c2);
        fetch(b2, e0, c2, r2);
      }
      // ---- this batch's points: a crest and a trough per lane
      const int b = b0;
      float cx, cy, A;
      dec_point<Rec>(d, n, in0, T, P.A[b], cx, cy, A, direct != nullptr);
      const float rc = d.bucket_r[b] / (float)P.dx;   // radius in cells
      const float qs = 0.25f / rc;                    // revolutions of the cosine per cell
      const int span = (int)floorf(2.f * rc) + 1;    // cells per axis a footprint reaches
      // unit direction of the code: v_cos / v_sin take revolutions
      const float rev = (float)in0.code * (1.0f / (float)kNCode);
      const float tx = cx - rc * __builtin_amdgcn_cosf(rev), ty = cy - rc * __builtin_amdgcn_sinf(rev);
      // the next batch's table loads go out before this batch is splatted
      const DecIn in1 = dec_load<Rec>(d, r1, n, b1, T.p, k1 < nbat && lane < c1);
      if constexpr (kProf)
        if (lane == 0) atomicAdd(&s_prof[PROF_POINTS + b], (unsigned long long)(2 * c0));
      mark(PROF_DECODE);
      const float4 pc = make_float4(cx, cy, A, 0.f), ptr = make_float4(tx, ty, -A, 0.f);
      const bool live = A != 0.f;
      if (span <= kAtomicSpan) {
        // ---- small footprints: the lane's two points, LDS atomics
        if constexpr (kRadial) {
          splat_points_radial<kAtomicSpan>(acc, pc, live, rc, qs, T.tw, T.th);
          splat_points_radial<kAtomicSpan>(acc, ptr, live, rc, qs, T.tw, T.th);
        } else {
          splat_points<kAtomicSpan>(acc, pc, live, rc, qs, T.tw, T.th);
          splat_points<kAtomicSpan>(acc, ptr, live, rc, qs, T.tw, T.th);
        }
      } else {
        // ---- large footprints: quadrant by quadrant; the points a product
        //      needs are read from their lanes' registers (no LDS traffic)
        auto point = [&](const int k, float &x, float &y, float &a) {   // k wave-uniform
          const int l = k & (kBatch - 1);
          const bool crest = k < kBatch;
          x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(crest ? cx : tx), l));
          y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(crest ? cy : ty), l));
          const float av = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(A), l));
          a = crest ? av : -av;
        };
        auto quadrant = [&](f32x16 &cq, const int xq, const int yq, const uint32_t bit) {
          if (xq >= T.tw || yq >= T.th) return;   // quadrant outside a narrow tile
          uint64_t m0 = __ballot(live && reaches(cx, cy, rc, xq, yq));
          uint64_t m1 = __ballot(live && reaches(tx, ty, rc, xq, yq));
          if (!(m0 | m1)) return;   // wave-uniform
          touched |= bit;
          if constexpr (kRadial) {
            // no outer-product form: each lane accumulates its 16 cells of the
            // quadrant (the matrix-core output layout) point by point
            const float dxl = (float)(xq + (lane & 31)), ybase = (float)(yq + 4 * (lane >> 5));
            for (int kk = pop_point(m0, m1); kk >= 0; kk = pop_point(m0, m1)) {
              float px, py, pa;
              point(kk, px, py, pa);
              const float dx = dxl - px, dx2 = dx * dx;
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                const float dy = ybase + (float)(8 * (r >> 2) + (r & 3)) - py;
                cq[r] += pa * wrev(__builtin_amdgcn_sqrtf(dx2 + dy * dy) * qs);
              }
            }
          } else {
            // rank-2 update D += W_y(:, k1 k2) [A_k1 W_x(k1, :); A_k2 W_x(k2, :)]
            // per pair of points (lanes 0-31 supply the first, 32-63 the
            // second, which is a zero-amplitude copy of the first when the
            // count is odd)
            const float yrow = (float)(yq + (lane & 31)), xcol = (float)(xq + (lane & 31));
            const bool lo = lane < 32;
            for (int j1 = pop_point(m0, m1); j1 >= 0; j1 = pop_point(m0, m1)) {   // wave-uniform
              const int j2 = pop_point(m0, m1);
              float x1, y1, a1, x2, y2, a2;
              point(j1, x1, y1, a1);
              if (j2 >= 0) point(j2, x2, y2, a2);
              else { x2 = x1; y2 = y1; a2 = 0.f; }
              const float px = lo ? x1 : x2, py = lo ? y1 : y2, pa = lo ? a1 : a2;
              const float a = wrev((yrow - py) * qs);
              const float bw = pa * wrev((xcol - px) * qs);
              cq = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bw, cq, 0, 0, 0);
            }
          }
        };
        bool whole = false;
        if constexpr (!kRadial) whole = 2.f * rc >= 32.f;   // footprints at least a quadrant wide
        if (whole) {
          // every pair goes to all quadrants of the tile: the row weights of
          // the two quadrant rows and the column weights of the two quadrant
          // columns serve four products (a quadrant a point misses gets zero
          // weights)
          uint64_t m0 = __ballot(live && (reaches(cx, cy, rc, 0, 0) || reaches(cx, cy, rc, 32, 32) ||
                                          reaches(cx, cy, rc, 32, 0) || reaches(cx, cy, rc, 0, 32)));
          uint64_t m1 = __ballot(live && (reaches(tx, ty, rc, 0, 0) || reaches(tx, ty, rc, 32, 32) ||
                                          reaches(tx, ty, rc, 32, 0) || reaches(tx, ty, rc, 0, 32)));
          const bool x1 = T.tw > 32, y1 = T.th > 32;   // right and lower quadrants exist
          if (m0 | m1) touched |= 1u | (x1 ? 2u : 0u) | (y1 ? 4u : 0u) | (x1 && y1 ? 8u : 0u);
          const float l32 = (float)(lane & 31);
          const bool lo = lane < 32;
          for (int j1 = pop_point(m0, m1); j1 >= 0; j1 = pop_point(m0, m1)) {   // wave-uniform
            const int j2 = pop_point(m0, m1);
            float xa, ya, aa, xb, yb, ab;
            point(j1, xa, ya, aa);
            if (j2 >= 0) point(j2, xb, yb, ab);
            else { xb = xa; yb = ya; ab = 0.f; }
            const float px = lo ? xa : xb, py = lo ? ya : yb, pa = lo ? aa : ab;
            const float a0 = wrev((l32 - py) * qs), a1 = wrev((l32 + 32.f - py) * qs);
            const float w0 = pa * wrev((l32 - px) * qs), w1 = pa * wrev((l32 + 32.f - px) * qs);
            cq0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, w0, cq0, 0, 0, 0);
            if (x1) cq1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, w1, cq1, 0, 0, 0);
            if (y1) cq2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, w0, cq2, 0, 0, 0);
            if (x1 && y1) cq3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, w1, cq3, 0, 0, 0);
          }
        } else {
          quadrant(cq0, 0, 0, 1u);
          quadrant(cq1, 32, 0, 2u);
          quadrant(cq2, 0, 32, 4u);
          quadrant(cq3, 32, 32, 8u);
        }
      }
      mark(PROF_BUCKET + b);
      k0 = k1; b0 = b1; c0 = c1;
      k1 = k2; b1 = b2; c1 = c2;
      r1 = r2;
      in0 = in1;
    }
    __syncthreads();
    mark(PROF_WAIT);
    // the quadrant accumulators into the tile: in round i wavefront w adds
    // its accumulator of quadrant (w + i) mod 4, so the four wavefronts of a
    // round touch disjoint cells and plain read-modify-writes suffice
    if (__syncthreads_or(touched != 0u)) {   // block-uniform
      auto add_quadrant = [&](const f32x16 &cq, const int xq, const int yq) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = yq + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          acc[row][xq + (lane & 31)] += cq[r];
        }
      };
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = (wave + i) & 3;   // wave-uniform
        if ((touched >> q) & 1u) {
          if (q == 0) add_quadrant(cq0, 0, 0);
          else if (q == 1) add_quadrant(cq1, 32, 0);
          else if (q == 2) add_quadrant(cq2, 0, 32);
          else add_quadrant(cq3, 32, 32);
        }
        __syncthreads();
      }
    }
    // time spent on this item's particles, for the next frame's plan
    if (tid == 0 && !direct)
      atomicAdd(&d.tile_meas[tile], (uint32_t)min<uint64_t>(__builtin_amdgcn_s_memrealtime() - t_work, 0x3FFFFFFFull));

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
    mark(PROF_EPILOGUE);
  }
  if constexpr (kProf) {
    __syncthreads();
    for (int i = tid; i < PROF_N; i += kThreads)
      if (s_prof[i]) atomicAdd(&d.splat_prof[i], s_prof[i]);
  }
}

// ---------------------------------------------------------------- splat, quadrant-owner schedule
// The second schedule of the same splat, for scenes whose footprints are
// mostly large (long waves on fine patches): the block decodes its list 256
// records at a time into LDS (a crest and a trough point per record, with
// the quadrants each reaches), then splats that chunk bucket by bucket:
//   * small footprints (kQuadAtomicSpan cells per axis): the chunk's points
//     are spread over all four wavefronts, one per lane, LDS float atomics;
//   * larger footprints: wavefront w owns quadrant w of the tile and feeds
//     the chunk's points that reach it, two at a time, to the 32x32x2 FP32
//     matrix-core product into its one accumulator (the radial kernel
//     accumulates the quadrant's cells point by point instead).
// One accumulator per wavefront keeps the kernel at five wavefronts per
// SIMD, which hides the latency of the per-pair weight and product chain;
// the batch schedule above holds four accumulators per wavefront (three
// wavefronts per SIMD) and wins where small footprints dominate.  Both give
// the same heights up to FP32 summation order.
constexpr int kChunk = kThreads;   // records decoded into LDS per round
// Footprints of at most this many cells per axis go through LDS atomics
// (measured: 4 for the separable kernel, whose matrix-core products are
// cheap; 7 for the radial one, whose quadrant path evaluates every cell).
constexpr int kQuadAtomicSpan = 4, kQuadAtomicSpanRadial = 7;

template <class Rec, bool kRadial, bool kProf>
__global__ __launch_bounds__(kThreads, 5) void k_splat_q(Dev d, int t0, int nt, const Rec *__restrict__ direct,
                                                      int ndirect, float *__restrict__ raw_out,
                                                      float *__restrict__ blend_out, int64_t out_off) {
  __shared__ __align__(16) float acc[kTile][kPad];
  // decoded chunk: for record i of the chunk, pt[2i] is its crest and
  // pt[2i + 1] its trough: centre (tile cells), signed amplitude (0: skip),
  // quadrants reached (bit w: quadrant of wavefront w)
  __shared__ float4 pt[2 * kChunk];
  __shared__ int s_rlo[kMaxBuckets][kMaxRows];
  __shared__ int s_pre[kMaxBuckets][kMaxRows + 1];
  __shared__ int s_nrows[kMaxBuckets];
  __shared__ int s_boff[kMaxBuckets + 1];    // offsets of the buckets in this part's list
  __shared__ int s_tile, s_part, s_nparts, s_patch;
  __shared__ unsigned long long s_prof[kProf ? PROF_N : 1];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int nwaves = kThreads / 64;
  const int64_t n = d.glob->n;
  const Rec *__restrict__ S = direct ? direct : (const Rec *)((n & 1) ? d.S1 : d.S0);
  const int total = direct ? nt : d.splat_ctl[1];
  const int nb = d.nb;
  // matrix-core path: wavefront w owns the 32 x 32 quadrant (xq, yq) of the tile
  const int xq = 32 * (wave & 1), yq = 32 * (wave >> 1);
  uint64_t t_mark = 0;
  auto mark = [&](int cat) {
    if constexpr (kProf) {
      const uint64_t now = __builtin_amdgcn_s_memtime();
      if (lane == 0) atomicAdd(&s_prof[cat], (unsigned long long)(now - t_mark));
      t_mark = now;
    }
  };
  if constexpr (kProf)
    for (int i = tid; i < PROF_N; i += kThreads) s_prof[i] = 0ull;

  for (int item = (int)blockIdx.x; item < total; item += (int)gridDim.x) {
    if constexpr (kProf) t_mark = __builtin_amdgcn_s_memtime();
    if (tid == 0) {
      const int4 e = direct ? make_int4(t0 + item, 0, 1, d.tile_patch[t0 + item]) : d.item_desc[item];
      s_tile = e.x;
      s_part = e.y;
      s_nparts = e.z;
      s_patch = e.w;
    }
    for (int c = tid; c < kTile * kPad / 4; c += kThreads)
      reinterpret_cast<float4 *>(&acc[0][0])[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int tile = s_tile, part = s_part, nparts = s_nparts;
    TileGeom T;
    tile_geom(d, tile, s_patch, T);
    const PatchDev &P = d.patches[T.p];
    // ---- row tables of every bucket (this part's entries), as in k_splat
    for (int q = tid; q < nb * kMaxRows; q += kThreads) {
      const int b = q / kMaxRows, r = q % kMaxRows;
      int nrows, lo = 0, len = 0;
      if (direct) {
        nrows = 1;
        if (r == 0) len = ndirect;
      } else {
        const short4 rc4 = d.tile_rect[(size_t)tile * nb + b];
        nrows = rc4.w;
        if (r < nrows) {
          const int rb = P.binbase[b] + (rc4.z + r) * P.nbx[b];
          const int a = min(d.off[rb + rc4.x], d.cap);
          const int e = max(a, min(d.off[rb + rc4.y + 1], d.cap));
          lo = part_count(a, part, nparts);
          len = part_count(e, part, nparts) - lo;
        }
      }
      if (r < nrows) {
        s_rlo[b][r] = lo;
        s_pre[b][r] = len;
      }
      if (r == 0) s_nrows[b] = nrows;
    }
    __syncthreads();
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
    if (wave == 0) {
      // bucket offsets in the item's list (buckets in index order)
      const int cnt = lane < nb ? s_pre[lane][s_nrows[lane]] : 0;
      int inc = cnt;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
      }
      if (lane < nb) s_boff[lane] = inc - cnt;
      if (lane == nb - 1) s_boff[nb] = inc;
    }
    __syncthreads();
    mark(PROF_SETUP);
    const int Mi = s_boff[nb];
    const bool quad_live = xq < T.tw && yq < T.th;
    f32x16 cq;
#pragma unroll
    for (int r = 0; r < 16; ++r) cq[r] = 0.f;
    const uint64_t t_work = __builtin_amdgcn_s_memrealtime();   // 100 MHz

    // the records of chunk c + 1 are loaded while chunk c is splatted
    Rec rec;
    int rec_b = -1;   // bucket of the prefetched record, -1: none
    auto fetch = [&](int c) {
      rec_b = -1;
      if (tid < min(kChunk, Mi - c)) {
        // item-list index -> bucket -> bin row -> particle
        const int g = c + tid;
        int b = 0;
        while (b + 1 < nb && s_boff[b + 1] <= g) ++b;
        const int v = g - s_boff[b];
        int lo = 0, hi = s_nrows[b] - 1;   // last row with prefix <= v
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[b][mid] <= v) lo = mid; else hi = mid - 1;
        }
        rec = S[part_entry(s_rlo[b][lo] + (v - s_pre[b][lo]), part, nparts)];
        rec_b = b;
      }
    };
    fetch(0);
    for (int c = 0; c < Mi; c += kChunk) {   // block-uniform
      const int m = min(kChunk, Mi - c);
      // ---- decode the prefetched records into crest and trough points
      if (rec_b >= 0) {
        const int b = rec_b;
        const DecIn in = dec_load<Rec>(d, rec, n, b, T.p, true);
        float cx, cy, A;
        dec_point<Rec>(d, n, in, T, P.A[b], cx, cy, A, direct != nullptr);
        const float rc = d.bucket_r[b] / (float)P.dx;
        const float rev = (float)in.code * (1.0f / (float)kNCode);
        const float tx = cx - rc * __builtin_amdgcn_cosf(rev), ty = cy - rc * __builtin_amdgcn_sinf(rev);
        auto quads = [&](float x, float y) {
          if (A == 0.f) return 0u;
          return (uint32_t)reaches(x, y, rc, 0, 0) | (uint32_t)reaches(x, y, rc, 32, 0) << 1 |
                 (uint32_t)reaches(x, y, rc, 0, 32) << 2 | (uint32_t)reaches(x, y, rc, 32, 32) << 3;
        };
        pt[2 * tid] = make_float4(cx, cy, A, __uint_as_float(quads(cx, cy)));
        pt[2 * tid + 1] = make_float4(tx, ty, -A, __uint_as_float(quads(tx, ty)));
      }
      __syncthreads();
      if (c + kChunk < Mi) fetch(c + kChunk);
      mark(PROF_DECODE);
      // ---- the chunk holds runs of consecutive buckets
      for (int b = 0; b < nb; ++b) {
        const int seg_lo = max(c, s_boff[b]) - c, seg_hi = min(c + m, s_boff[b + 1]) - c;
        if (seg_hi <= seg_lo) continue;   // block-uniform
        if constexpr (kProf)
          if (tid == 0) atomicAdd(&s_prof[PROF_POINTS + b], (unsigned long long)(2 * (seg_hi - seg_lo)));
        const float rc = d.bucket_r[b] / (float)P.dx;   // radius in cells
        const float qs = 0.25f / rc;                    // revolutions of the cosine per cell
        const int span = (int)floorf(2.f * rc) + 1;    // cells per axis a footprint reaches
        const int q_lo = 2 * seg_lo, q_hi = 2 * seg_hi;
        if (span <= (kRadial ? kQuadAtomicSpanRadial : kQuadAtomicSpan)) {
          // ---- small footprints: points spread over all wavefronts
          for (int q0 = q_lo + 64 * wave; q0 < q_hi; q0 += 64 * nwaves) {
            const int q = q0 + lane;
            const bool valid = q < q_hi;
            const float4 pv = pt[valid ? q : q_lo];
            if constexpr (kRadial) {
              if (span <= 3) splat_points_radial<4>(acc, pv, valid, rc, qs, T.tw, T.th);
              else splat_points_radial<8>(acc, pv, valid, rc, qs, T.tw, T.th);
            } else {
              if (span <= 3) splat_points<4>(acc, pv, valid, rc, qs, T.tw, T.th);
              else splat_points<8>(acc, pv, valid, rc, qs, T.tw, T.th);
            }
          }
        } else if (quad_live) {
          if constexpr (kRadial) {
            // no outer-product form: each lane accumulates the 16 cells it
            // holds in the matrix-core layout (column xq + lane % 32, rows
            // yq + 8 (r / 4) + 4 (lane / 32) + r % 4), point by point
            const float dxl = (float)(xq + (lane & 31)), ybase = (float)(yq + 4 * (lane >> 5));
            for (int q0 = q_lo; q0 < q_hi; q0 += 64) {   // wave-uniform
              const int q = q0 + lane;
              const bool hit = q < q_hi && ((__float_as_uint(pt[q].w) >> wave) & 1u);
              uint64_t mask = __ballot(hit);
              while (mask) {   // wave-uniform
                const float4 pv = pt[q0 + __builtin_ctzll(mask)];
                mask &= mask - 1;
                const float dx = dxl - pv.x, dx2 = dx * dx;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                  const float dy = ybase + (float)(8 * (r >> 2) + (r & 3)) - pv.y;
                  cq[r] += pv.z * wrev(__builtin_amdgcn_sqrtf(dx2 + dy * dy) * qs);
                }
              }
            }
          } else {
            // rank-2 update D += W_y(:, k1 k2) [A_k1 W_x(k1, :); A_k2 W_x(k2, :)]
            // for each pair of the chunk's points that reach the quadrant
            // (lanes 0-31 supply the first point, 32-63 the second)
            const float yrow = (float)(yq + (lane & 31)), xcol = (float)(xq + (lane & 31));
            for (int q0 = q_lo; q0 < q_hi; q0 += 64) {   // wave-uniform
              const int q = q0 + lane;
              const bool hit = q < q_hi && ((__float_as_uint(pt[q].w) >> wave) & 1u);
              uint64_t mask = __ballot(hit);
              if (!mask) continue;   // wave-uniform
              // the next pair's point is read from LDS before the current
              // pair's product is issued
              auto pop = [&](int &k1, int &k2, float &keep) {
                k1 = __builtin_ctzll(mask);
                mask &= mask - 1;
                k2 = k1;
                keep = lane < 32 ? 1.f : 0.f;   // odd count: the second copy gets no weight
                if (mask) {
                  k2 = __builtin_ctzll(mask);
                  mask &= mask - 1;
                  keep = 1.f;
                }
              };
              int k1, k2;
              float keep;
              pop(k1, k2, keep);
              float4 pv = pt[q0 + (lane < 32 ? k1 : k2)];
              while (true) {
                const bool more = mask != 0;   // wave-uniform
                float4 pn = pv;
                float keep_n = 0.f;
                if (more) {
                  pop(k1, k2, keep_n);
                  pn = pt[q0 + (lane < 32 ? k1 : k2)];
                }
                const float a = wrev((yrow - pv.y) * qs);
                const float bw = keep * pv.z * wrev((xcol - pv.x) * qs);
                cq = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bw, cq, 0, 0, 0);
                if (!more) break;
                pv = pn;
                keep = keep_n;
              }
            }
          }
        }
        mark(PROF_BUCKET + b);
      }
      __syncthreads();
      mark(PROF_WAIT);
    }
    // ---- the matrix-core quadrants into the tile (disjoint per wavefront)
    if (quad_live) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = yq + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        acc[row][xq + (lane & 31)] += cq[r];
      }
    }
    __syncthreads();
    // time spent on this item's particles, for the next frame's plan
    if (tid == 0 && !direct)
      atomicAdd(&d.tile_meas[tile], (uint32_t)min<uint64_t>(__builtin_amdgcn_s_memrealtime() - t_work, 0x3FFFFFFFull));
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
    mark(PROF_EPILOGUE);
  }
  if constexpr (kProf) {
    __syncthreads();
    for (int i = tid; i < PROF_N; i += kThreads)
      if (s_prof[i]) atomicAdd(&d.splat_prof[i], s_prof[i]);
  }
}

// ---------------------------------------------------------------- splat, hybrid schedule
// The third schedule: each item runs the two schedules above one after the
// other, each on the buckets it handles best.
//   1. Buckets with footprints of at most kAtomicSpan cells per axis (7 with
//      the radial kernel), as in k_splat: wavefronts take batches of 64
//      entries independently (three batches in flight, no barrier), LDS
//      float atomics.
//   2. The other buckets, as in k_splat_q: the block decodes 256 records at
//      a time into LDS and wavefront w feeds the points that reach quadrant w
//      to the matrix cores, into its one accumulator.
// Without the four accumulators of the batch schedule the kernel fits five
// wavefronts per SIMD (at 96 registers a few of phase 1's values spill to
// scratch, which measured faster than four wavefronts without spills: c5
// 1.04 vs 1.08 ms, p0 0.16 vs 0.26 ms).  It is the default schedule.
template <class Rec, bool kRadial, bool kProf>
__global__ __launch_bounds__(kThreads, 5) void k_splat_h(Dev d, int t0, int nt, const Rec *__restrict__ direct,
                                                      int ndirect, float *__restrict__ raw_out,
                                                      float *__restrict__ blend_out, int64_t out_off) {
  __shared__ __align__(16) float acc[kTile][kPad];
  __shared__ float4 pt[2 * kChunk];           // phase 2: decoded chunk, as in k_splat_q
  __shared__ int s_rlo[kMaxBuckets][kMaxRows];
  __shared__ int s_pre[kMaxBuckets][kMaxRows + 1];
  __shared__ int s_nrows[kMaxBuckets];
  __shared__ int s_cnt[kMaxBuckets];          // entries of this part in each bucket's list
  __shared__ int s_bat[kMaxBuckets + 1];      // phase 1: first batch of the j-th bucket taken (bucket nb - 1 - j)
  __shared__ int s_boff[kMaxBuckets + 1];     // phase 2: offsets of the large buckets in the item's list
  __shared__ float2 s_rq[kMaxBuckets];         // radius in cells, revolutions of the cosine per cell
  __shared__ int s_tile, s_part, s_nparts, s_patch;
  __shared__ unsigned long long s_prof[kProf ? PROF_N : 1];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int nwaves = kThreads / 64;
  const int64_t n = d.glob->n;
  const Rec *__restrict__ S = direct ? direct : (const Rec *)((n & 1) ? d.S1 : d.S0);
  const int total = direct ? nt : d.splat_ctl[1];
  const int nb = d.nb;
  const int xq = 32 * (wave & 1), yq = 32 * (wave >> 1);   // phase 2: the wavefront's quadrant
  // footprints of at most this many cells per axis go through phase 1
  constexpr int kSmall = kRadial ? kQuadAtomicSpanRadial : kAtomicSpan;
  uint64_t t_mark = 0;
  auto mark = [&](int cat) {
    if constexpr (kProf) {
      const uint64_t now = __builtin_amdgcn_s_memtime();
      if (lane == 0) atomicAdd(&s_prof[cat], (unsigned long long)(now - t_mark));
      t_mark = now;
    }
  };
  if constexpr (kProf)
    for (int i = tid; i < PROF_N; i += kThreads) s_prof[i] = 0ull;

  for (int item = (int)blockIdx.x; item < total; item += (int)gridDim.x) {
    if constexpr (kProf) t_mark = __builtin_amdgcn_s_memtime();
    if (tid == 0) {
      const int4 e = direct ? make_int4(t0 + item, 0, 1, d.tile_patch[t0 + item]) : d.item_desc[item];
      s_tile = e.x;
      s_part = e.y;
      s_nparts = e.z;
      s_patch = e.w;
    }
    for (int c = tid; c < kTile * kPad / 4; c += kThreads)
      reinterpret_cast<float4 *>(&acc[0][0])[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int tile = s_tile, part = s_part, nparts = s_nparts;
    TileGeom T;
    tile_geom(d, tile, s_patch, T);
    const PatchDev &P = d.patches[T.p];
    // ---- row tables of every bucket (this part's entries), as in k_splat
    for (int q = tid; q < nb * kMaxRows; q += kThreads) {
      const int b = q / kMaxRows, r = q % kMaxRows;
      int nrows, lo = 0, len = 0;
      if (direct) {
        nrows = 1;
        if (r == 0) len = ndirect;
      } else {
        const short4 rc4 = d.tile_rect[(size_t)tile * nb + b];
        nrows = rc4.w;
        if (r < nrows) {
          const int rb = P.binbase[b] + (rc4.z + r) * P.nbx[b];
          const int a = min(d.off[rb + rc4.x], d.cap);
          const int e = max(a, min(d.off[rb + rc4.y + 1], d.cap));
          lo = part_count(a, part, nparts);
          len = part_count(e, part, nparts) - lo;
        }
      }
      if (r < nrows) {
        s_rlo[b][r] = lo;
        s_pre[b][r] = len;
      }
      if (r == 0) s_nrows[b] = nrows;
    }
    __syncthreads();
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
    if (wave == 0) {
      // lane j: the j-th bucket in phase-1 order (largest radii first) and
      // bucket j for the phase-2 offsets
      int cnt1 = 0, cnt2 = 0;
      if (lane < nb) {
        const float rcl = d.bucket_r[lane] / (float)P.dx;
        s_rq[lane] = make_float2(rcl, 0.25f / rcl);
        const int b = nb - 1 - lane;
        const int span = (int)floorf(2.f * d.bucket_r[b] / (float)P.dx) + 1;
        const int cnt = s_pre[b][s_nrows[b]];
        cnt1 = span <= kSmall ? cnt : 0;
        s_cnt[b] = cnt;
        const int span2 = (int)floorf(2.f * d.bucket_r[lane] / (float)P.dx) + 1;
        cnt2 = span2 <= kSmall ? 0 : s_pre[lane][s_nrows[lane]];
      }
      const int nbj = (cnt1 + kBatch - 1) / kBatch;
      int inc = nbj, inc2 = cnt2;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o), y2 = __shfl_up(inc2, o);
        if (lane >= o) {
          inc += y;
          inc2 += y2;
        }
      }
      if (lane < nb) {
        s_bat[lane] = inc - nbj;
        s_boff[lane] = inc2 - cnt2;
      }
      if (lane == nb - 1) {
        s_bat[nb] = inc;
        s_boff[nb] = inc2;
      }
    }
    __syncthreads();
    mark(PROF_SETUP);
    const uint64_t t_work = __builtin_amdgcn_s_memrealtime();   // 100 MHz

    // ======== phase 1: small footprints, batches per wavefront
    {
      const int bat_lo = lane < nb ? s_bat[lane] : 0x7FFFFFFF;
      const int bat_cnt = lane < nb ? s_cnt[nb - 1 - lane] : 0;
      const int nbat = s_bat[nb];
      auto locate = [&](int k, int &b, int &cnt) {
        const int j = __popcll(__ballot(bat_lo <= k)) - 1;
        b = nb - 1 - j;
        const int e0 = (k - __builtin_amdgcn_readlane(bat_lo, j)) * kBatch;
        cnt = min(kBatch, __builtin_amdgcn_readlane(bat_cnt, j) - e0);
        return e0;
      };
      auto fetch = [&](int b, int e0, int cnt, Rec &rec) {
        if (lane < cnt) {
          const int v = e0 + lane;
          int lo = 0, hi = s_nrows[b] - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[b][mid] <= v) lo = mid; else hi = mid - 1;
          }
          rec = S[part_entry(s_rlo[b][lo] + (v - s_pre[b][lo]), part, nparts)];
        }
      };
      constexpr int kWaves = kThreads / 64;
      int k0 = wave, b0 = 0, c0 = 0;
      Rec r0, r1;
      if (k0 < nbat) {
        const int e0 = locate(k0, b0, c0);
        fetch(b0, e0, c0, r0);
      }
      int k1 = wave + kWaves, b1 = 0, c1 = 0;
      if (k1 < nbat) {
        const int e0 = locate(k1, b1, c1);
        fetch(b1, e0, c1, r1);
      }
      DecIn in0 = dec_load<Rec>(d, r0, n, b0, T.p, k0 < nbat && lane < c0);
      while (k0 < nbat) {   // wave-uniform
        const int k2 = k1 + kWaves;
        int b2 = 0, c2 = 0;
        Rec r2;
        if (k2 < nbat) {
          const int e0 = locate(k2, b2, c2);
          fetch(b2, e0, c2, r2);
        }
        const int b = b0;
        float cx, cy, A;
        dec_point<Rec>(d, n, in0, T, P.A[b], cx, cy, A, direct != nullptr);
        const float2 rq = s_rq[b];
        const float rc = rq.x, qs = rq.y;
        const int span = (int)floorf(2.f * rc) + 1;
        const float rev = (float)in0.code * (1.0f / (float)kNCode);
        const float tx = cx - rc * __builtin_amdgcn_cosf(rev), ty = cy - rc * __builtin_amdgcn_sinf(rev);
        const DecIn in1 = dec_load<Rec>(d, r1, n, b1, T.p, k1 < nbat && lane < c1);
        if constexpr (kProf)
          if (lane == 0) atomicAdd(&s_prof[PROF_POINTS + b], (unsigned long long)(2 * c0));
        mark(PROF_DECODE);
        const float4 pc = make_float4(cx, cy, A, 0.f), ptr = make_float4(tx, ty, -A, 0.f);
        const bool live = A != 0.f;
        // loops sized to the bucket's span (wave-uniform)
        if constexpr (kRadial) {
          if (span <= 4) {
            splat_points_radial<4>(acc, pc, live, rc, qs, T.tw, T.th);
            splat_points_radial<4>(acc, ptr, live, rc, qs, T.tw, T.th);
          } else {
            splat_points_radial<8>(acc, pc, live, rc, qs, T.tw, T.th);
            splat_points_radial<8>(acc, ptr, live, rc, qs, T.tw, T.th);
          }
        } else if (span <= 2) {
          splat_points<2>(acc, pc, live, rc, qs, T.tw, T.th);
          splat_points<2>(acc, ptr, live, rc, qs, T.tw, T.th);
        } else {
          splat_points<kAtomicSpan>(acc, pc, live, rc, qs, T.tw, T.th);
          splat_points<kAtomicSpan>(acc, ptr, live, rc, qs, T.tw, T.th);
        }
        mark(PROF_BUCKET + b);
        k0 = k1; b0 = b1; c0 = c1;
        k1 = k2; b1 = b2; c1 = c2;
        r1 = r2;
        in0 = in1;
      }
    }

    // ======== phase 2: large footprints, one quadrant per wavefront
    const int Mi = s_boff[nb];   // block-uniform
    const bool quad_live = xq < T.tw && yq < T.th;
    f32x16 cq;
#pragma unroll
    for (int r = 0; r < 16; ++r) cq[r] = 0.f;
    if (Mi > 0) {
      Rec rec;
      int rec_b = -1;
      auto fetch2 = [&](int c) {
        rec_b = -1;
        if (tid < min(kChunk, Mi - c)) {
          const int g = c + tid;
          int b = 0;
          while (b + 1 < nb && s_boff[b + 1] <= g) ++b;
          const int v = g - s_boff[b];
          int lo = 0, hi = s_nrows[b] - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[b][mid] <= v) lo = mid; else hi = mid - 1;
          }
          rec = S[part_entry(s_rlo[b][lo] + (v - s_pre[b][lo]), part, nparts)];
          rec_b = b;
        }
      };
      fetch2(0);
      __syncthreads();   // phase 1 done everywhere before pt is written
      mark(PROF_WAIT);
      for (int c = 0; c < Mi; c += kChunk) {   // block-uniform
        const int m = min(kChunk, Mi - c);
        if (rec_b >= 0) {
          const int b = rec_b;
          const DecIn in = dec_load<Rec>(d, rec, n, b, T.p, true);
          float cx, cy, A;
          dec_point<Rec>(d, n, in, T, P.A[b], cx, cy, A, direct != nullptr);
          const float rc = s_rq[b].x;
          const float rev = (float)in.code * (1.0f / (float)kNCode);
          const float tx = cx - rc * __builtin_amdgcn_cosf(rev), ty = cy - rc * __builtin_amdgcn_sinf(rev);
          auto quads = [&](float x, float y) {
            if (A == 0.f) return 0u;
            return (uint32_t)reaches(x, y, rc, 0, 0) | (uint32_t)reaches(x, y, rc, 32, 0) << 1 |
                   (uint32_t)reaches(x, y, rc, 0, 32) << 2 | (uint32_t)reaches(x, y, rc, 32, 32) << 3;
          };
          pt[2 * tid] = make_float4(cx, cy, A, __uint_as_float(quads(cx, cy)));
          pt[2 * tid + 1] = make_float4(tx, ty, -A, __uint_as_float(quads(tx, ty)));
        }
        __syncthreads();
        if (c + kChunk < Mi) fetch2(c + kChunk);
        mark(PROF_DECODE);
        for (int b = 0; b < nb; ++b) {
          const int seg_lo = max(c, s_boff[b]) - c, seg_hi = min(c + m, s_boff[b + 1]) - c;
          if (seg_hi <= seg_lo) continue;   // block-uniform
          if constexpr (kProf)
            if (tid == 0) atomicAdd(&s_prof[PROF_POINTS + b], (unsigned long long)(2 * (seg_hi - seg_lo)));
          const float2 rq = s_rq[b];
          const float rc = rq.x, qs = rq.y;
          const int q_lo = 2 * seg_lo, q_hi = 2 * seg_hi;
          if (quad_live) {
            if constexpr (kRadial) {
              const float dxl = (float)(xq + (lane & 31)), ybase = (float)(yq + 4 * (lane >> 5));
              for (int q0 = q_lo; q0 < q_hi; q0 += 64) {   // wave-uniform
                const int q = q0 + lane;
                const bool hit = q < q_hi && ((__float_as_uint(pt[q].w) >> wave) & 1u);
                uint64_t mask = __ballot(hit);
                while (mask) {   // wave-uniform
                  const float4 pv = pt[q0 + __builtin_ctzll(mask)];
                  mask &= mask - 1;
                  const float dx = dxl - pv.x, dx2 = dx * dx;
#pragma unroll
                  for (int r = 0; r < 16; ++r) {
                    const float dy = ybase + (float)(8 * (r >> 2) + (r & 3)) - pv.y;
                    cq[r] += pv.z * wrev(__builtin_amdgcn_sqrtf(dx2 + dy * dy) * qs);
                  }
                }
              }
            } else {
              const float yrow = (float)(yq + (lane & 31)), xcol = (float)(xq + (lane & 31));
              for (int q0 = q_lo; q0 < q_hi; q0 += 64) {   // wave-uniform
                const int q = q0 + lane;
                const bool hit = q < q_hi && ((__float_as_uint(pt[q].w) >> wave) & 1u);
                uint64_t mask = __ballot(hit);
                if (!mask) continue;   // wave-uniform
                auto pop = [&](int &k1, int &k2, float &keep) {
                  k1 = __builtin_ctzll(mask);
                  mask &= mask - 1;
                  k2 = k1;
                  keep = lane < 32 ? 1.f : 0.f;
                  if (mask) {
                    k2 = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    keep = 1.f;
                  }
                };
                int k1, k2;
                float keep;
                pop(k1, k2, keep);
                float4 pv = pt[q0 + (lane < 32 ? k1 : k2)];
                while (true) {
                  const bool more = mask != 0;   // wave-uniform
                  float4 pn = pv;
                  float keep_n = 0.f;
                  if (more) {
                    pop(k1, k2, keep_n);
                    pn = pt[q0 + (lane < 32 ? k1 : k2)];
                  }
                  const float a = wrev((yrow - pv.y) * qs);
                  const float bw = keep * pv.z * wrev((xcol - pv.x) * qs);
                  cq = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bw, cq, 0, 0, 0);
                  if (!more) break;
                  pv = pn;
                  keep = keep_n;
                }
              }
            }
          }
          mark(PROF_BUCKET + b);
        }
        __syncthreads();
        mark(PROF_WAIT);
      }
    }
    __syncthreads();   // phase 1 atomics (when phase 2 had nothing) before the quadrants are added
    if (Mi > 0 && quad_live) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = yq + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        acc[row][xq + (lane & 31)] += cq[r];
      }
    }
    __syncthreads();
    if (tid == 0 && !direct)
      atomicAdd(&d.tile_meas[tile], (uint32_t)min<uint64_t>(__builtin_amdgcn_s_memrealtime() - t_work, 0x3FFFFFFFull));
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
    mark(PROF_EPILOGUE);
  }
  if constexpr (kProf) {
    __syncthreads();
    for (int i = tid; i < PROF_N; i += kThreads)
      if (s_prof[i]) atomicAdd(&d.splat_prof[i], s_prof[i]);
  }
}

// ---------------------------------------------------------------- reduce
// Persistent grid over the units (split tile, stripe of 4 rows) listed by the
// plan: sums the partial tiles of the split tile and runs the blend.  Tiles
// with a single part were finished by k_splat.  Each of the 4 wavefronts sums
// every 4th part, 4 cells per lane (16-byte loads); the wavefronts are then
// combined in LDS.
constexpr int kStripes = kTile / 4;
constexpr int kRedGroups = kThreads / 64;

__global__ __launch_bounds__(kThreads) void k_splat_reduce(Dev d) {
  __shared__ float4 red[kRedGroups][64];
  const int g = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
  const int nunits = d.splat_ctl[2] * kStripes;
  constexpr size_t kPart4 = kTile * kTile / 4;   // float4 per partial tile
  for (int u = (int)blockIdx.x; u < nunits; u += (int)gridDim.x) {
    const int tile = d.split_tiles[u / kStripes], q = u % kStripes;
    const int base = d.item_base[tile], np_ = d.item_base[tile + 1] - base;
    const float4 *src =
        reinterpret_cast<const float4 *>(d.partials + (size_t)base * (kTile * kTile) + q * 4 * kTile) + l;
    // the wavefront sums parts g, g + 4, ...; eight loads in flight per lane
    float4 h = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int s0 = g; s0 < np_; s0 += 8 * kRedGroups) {
      float4 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int s = s0 + k * kRedGroups;
        v[k] = s < np_ ? src[(size_t)s * kPart4] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        h.x += v[k].x; h.y += v[k].y; h.z += v[k].z; h.w += v[k].w;
      }
    }
    red[g][l] = h;
    __syncthreads();
    if (g == 0) {
      float4 h = red[0][l];
      for (int k = 1; k < kRedGroups; ++k) {
        const float4 v = red[k][l];
        h.x += v.x; h.y += v.y; h.z += v.z; h.w += v.w;
      }
      TileGeom T;
      tile_geom(d, tile, d.tile_patch[tile], T);
      const PatchDev &P = d.patches[T.p];
      const StepPatch &W = d.sp[T.p];
      const int c = q * 4 * kTile + 4 * l;   // first of the lane's 4 cells
      const int j = c / kTile, i = c % kTile;
      const float hv[4] = {h.x, h.y, h.z, h.w};
      if (j < T.th)
        for (int e = 0; e < 4; ++e)
          if (i + e < T.tw) blend_store(d, P, W, T, i + e, j, hv[e], d.raw, d.blend, 0);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers
void launch_splat_plan(const Dev &d, int t0, int ntiles, int items_target, hipStream_t st) {
  if (ntiles <= 0) return;
  const int wpb = kThreads / 64;
  hipLaunchKernelGGL(k_splat_load, dim3((ntiles + wpb - 1) / wpb), dim3(kThreads), 0, st, d, t0, ntiles);
  hipLaunchKernelGGL(k_splat_plan, dim3(1), dim3(kPlanThreads), 0, st, d, t0, ntiles, items_target);
}

bool bin_plan_fits(int nbins, int ntiles, int nb) {
  return nbins <= kFusedMaxBins && ntiles <= kFusedMaxTiles && (int64_t)ntiles * nb <= kPlanThreads;
}

void launch_bin_plan(const Dev &d, int nbins, int ntiles, int items_target, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_plan, dim3(1), dim3(kPlanThreads), 0, st, d, nbins, ntiles, items_target);
}

// The splat kernel for the record form and kernel shape of d.
template <bool kRadial, bool kProf>
void splat_launch(const Dev &d, dim3 grid, int t0, int ntiles, const void *recs, int n, float *raw, float *blend,
                  int64_t out_off, hipStream_t st) {
  if (d.splat_kernel == 2) {
    if (d.compact)
      hipLaunchKernelGGL((k_splat_h<RecCompact, kRadial, kProf>), grid, dim3(kThreads), 0, st, d, t0, ntiles,
                         (const RecCompact *)recs, n, raw, blend, out_off);
    else
      hipLaunchKernelGGL((k_splat_h<RecWide, kRadial, kProf>), grid, dim3(kThreads), 0, st, d, t0, ntiles,
                         (const RecWide *)recs, n, raw, blend, out_off);
  } else if (d.splat_kernel == 1) {
    if (d.compact)
      hipLaunchKernelGGL((k_splat_q<RecCompact, kRadial, kProf>), grid, dim3(kThreads), 0, st, d, t0, ntiles,
                         (const RecCompact *)recs, n, raw, blend, out_off);
    else
      hipLaunchKernelGGL((k_splat_q<RecWide, kRadial, kProf>), grid, dim3(kThreads), 0, st, d, t0, ntiles,
                         (const RecWide *)recs, n, raw, blend, out_off);
  } else if (d.compact) {
    hipLaunchKernelGGL((k_splat<RecCompact, kRadial, kProf>), grid, dim3(kThreads), 0, st, d, t0, ntiles,
                       (const RecCompact *)recs, n, raw, blend, out_off);
  } else {
    hipLaunchKernelGGL((k_splat<RecWide, kRadial, kProf>), grid, dim3(kThreads), 0, st, d, t0, ntiles,
                       (const RecWide *)recs, n, raw, blend, out_off);
  }
}

void splat_launch_any(const Dev &d, dim3 grid, int t0, int ntiles, const void *recs, int n, float *raw, float *blend,
                      int64_t out_off, hipStream_t st) {
  const bool prof = d.splat_profile && d.splat_prof && !recs;
  if (d.radial) {
    if (prof) splat_launch<true, true>(d, grid, t0, ntiles, recs, n, raw, blend, out_off, st);
    else splat_launch<true, false>(d, grid, t0, ntiles, recs, n, raw, blend, out_off, st);
  } else {
    if (prof) splat_launch<false, true>(d, grid, t0, ntiles, recs, n, raw, blend, out_off, st);
    else splat_launch<false, false>(d, grid, t0, ntiles, recs, n, raw, blend, out_off, st);
  }
}

void launch_splat_tiles(const Dev &d, int t0, int ntiles, int grid, hipStream_t st) {
  if (ntiles <= 0) return;
  splat_launch_any(d, dim3(grid), t0, ntiles, nullptr, 0, d.raw, d.blend, (int64_t)0, st);
}

void launch_splat_reduce(const Dev &d, int t0, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_splat_reduce, dim3(std::min(kStripes * ntiles, 8192)), dim3(kThreads), 0, st, d);
}

void launch_splat_direct(const Dev &d, int t0, int ntiles, const void *recs, int n, float *raw, int64_t out_off,
                         hipStream_t st) {
  if (ntiles <= 0) return;
  splat_launch_any(d, dim3(ntiles), t0, ntiles, recs, n, raw, (float *)nullptr, out_off, st);
}

}  // namespace hwo

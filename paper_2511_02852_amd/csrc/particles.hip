// particles.hip -- per-step wave-particle bookkeeping on gfx950.
//
// One step n (heights then describe t_n = n dt):
//   k_params   one block: advance the step counter, recentre the windows of
//              patches that follow a source (FP64 source position), compute
//              the FP64 background offsets of every patch, the boundary
//              injection count of every (patch, bucket, side pair) from the
//              32.32 rate of Eq 18, the ring emissions of every
//              source (Sec 4.3), and their prefix sums.
//   k_update   persistent grid over all work items of the step: previous
//   <count>    particles (subdivide, then survive), new boundary particles
//              (Philox draw -> integer inverse CDF of Dir -> entry side ->
//              position on the side) and new ring particles.  Every output
//              particle that survives gets a bin key (patch, bucket, by, bx);
//              runs of equal keys inside a wavefront are merged before the
//              histogram atomic (input is sorted by key, so runs are long).
//   k_scan     exclusive scan of the histogram -> bin offsets (and cursors);
//              clears the histogram for the next step.
//   k_update   same computation again; each run reserves its slots with one
//   <scatter>  atomic on the bin cursor and writes the records, so the
//              output buffer is sorted by bin.
// Every integer decision (counts, codes, positions, survival, bins) is made
// in exact integer arithmetic from fixed-point tables built in FP64, so the
// result matches the CPU oracle bit for bit.
#include "hwo_dev.h"

namespace hwo {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive scan of a[0..len) in place by one block; returns the total.
// Each thread scans a run of consecutive entries; the run sums are scanned
// with wavefront shuffles and one LDS slot per wavefront.
__device__ int32_t block_scan_excl(int32_t *a, int len, int32_t *s_w /* kThreads / 64 */) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int chunk = (len + kThreads - 1) / kThreads;
  const int beg = min(len, tid * chunk), end = min(len, beg + chunk);
  int32_t sum = 0;
  for (int i = beg; i < end; ++i) sum += a[i];
  int32_t inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  int32_t acc = inc - sum, total = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wv) acc += s_w[w];
    total += s_w[w];
  }
  for (int i = beg; i < end; ++i) {
    const int32_t v = a[i];
    a[i] = acc;
    acc += v;
  }
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------- windows
// Window of patch p at step n (a patch that follows a source recentres in
// whole cells on the source's FP64 position), its background offsets and the
// range of its previous particles in the input buffer.  The injection and
// emission ranges are left to the caller.
// Window origin (cells) of patch p at step n.
__device__ __forceinline__ void window_origin(const Dev &d, int p, int64_t n, int64_t &wx, int64_t &wy) {
  const PatchDev &P = d.patches[p];
  wx = 0;
  wy = 0;
  if (P.follow >= 0) {
    const double tn = (double)n * d.dt;
    const SourceDev &S = d.sources[P.follow];
    const double xs = S.x0 + S.vx * tn;
    const double ys = S.y0 + S.vy * tn;
    wx = round_away((xs - P.ax) / P.dx) - P.nx / 2;
    wy = round_away((ys - P.ay) / P.dx) - P.ny / 2;
  }
}

__device__ void patch_window(const Dev &d, int p, int64_t n, StepPatch &W) {
  const PatchDev &P = d.patches[p];
  int64_t wx, wy;
  window_origin(d, p, n, wx, wy);
  W.wx = (int32_t)wx;
  W.wy = (int32_t)wy;
  // keep every window (with a 64 m margin) inside the int32 position range
  const int64_t lim = (int64_t)1 << 31;
  const int64_t reach = (int64_t)64 << 20;
  if (wx * P.dxu - reach < -lim || (wx + P.nx) * P.dxu + reach >= lim ||
      wy * P.dxu - reach < -lim || (wy + P.ny) * P.dxu + reach >= lim)
    atomicOr(&d.glob->err, 1);
  const double X = P.ax + (double)(wx * P.dxu + P.dxu / 2) * (1.0 / 1048576.0);
  const double Y = P.ay + (double)(wy * P.dxu + P.dxu / 2) * (1.0 / 1048576.0);
  const double u = X / d.dxf, v = Y / d.dxf;
  const double fu = floor(u), fv = floor(v);
  const int64_t N = d.N;
  W.gx0 = (int32_t)((((int64_t)fu % N) + N) % N);
  W.gy0 = (int32_t)((((int64_t)fv % N) + N) % N);
  W.fx0 = (float)(u - fu);
  W.fy0 = (float)(v - fv);
  W.ex_lo = min(d.off[P.bin_lo], d.cap);
  W.ex_hi = min(d.off[P.bin_hi], d.cap);
}

// Windows of every patch at the current step without advancing it (after a
// restore, so that reads before the next step see the restored step).
__global__ __launch_bounds__(kThreads) void k_windows(Dev d) {
  const int64_t n = d.glob->n;
  for (int p = threadIdx.x; p < d.np; p += kThreads) {
    StepPatch W = d.sp[p];
    patch_window(d, p, n, W);
    d.sp[p] = W;
    StepPatch Wn = W;
    patch_window(d, p, n + 1, Wn);
    d.sp_next[p] = Wn;
  }
}

// ---------------------------------------------------------------- k_params
// The injection and emission counts and their scans stay in LDS; global
// memory gets the scanned offsets once, and the counters are bumped with
// atomics, so no step waits on a global read of what the block just wrote.
constexpr int kParamsPer = 4;   // injection slots per thread whose rate loads are in flight together

__global__ __launch_bounds__(kThreads) void k_params(Dev d) {
  __shared__ int64_t s_n;
  __shared__ int32_t s_tmp[kThreads / 64];
  __shared__ int32_t s_inj[kMaxInjSlots + 1];
  __shared__ int32_t s_em[kMaxSources + 1];
  const int tid = threadIdx.x;
  if (tid == 0) {
    const int64_t n = d.glob->n + 1;
    d.glob->n = n;
    s_n = n;
  }
  __syncthreads();
  const int64_t n = s_n;
  const double tn = (double)n * d.dt;

  // windows, background offsets, previous-particle ranges; the windows of
  // the next step for the scatter's histogram of it
  for (int p = tid; p < d.np; p += kThreads) {
    StepPatch W;
    patch_window(d, p, n, W);
    d.sp[p] = W;
    int64_t wx, wy;
    window_origin(d, p, n + 1, wx, wy);   // only the origin is used for the next step's bins
    StepPatch Wn = W;
    Wn.wx = (int32_t)wx;
    Wn.wy = (int32_t)wy;
    d.sp_next[p] = Wn;
  }

  // injection counts per (patch, bucket, pair), in that order
  const int ns_inj = d.n_inj_slots;
  for (int q0 = 0; q0 < ns_inj; q0 += kThreads * kParamsPer) {
    uint64_t R[kParamsPer];
#pragma unroll
    for (int k = 0; k < kParamsPer; ++k) {
      const int q = q0 + tid + k * kThreads;
      R[k] = 0;
      if (q < ns_inj) {
        const int pp = q / (2 * d.nb), i = (q / 2) % d.nb;
        const PatchDev &P = d.patches[pp];
        R[k] = (q & 1) ? P.Ry[i] : P.Rx[i];
      }
    }
#pragma unroll
    for (int k = 0; k < kParamsPer; ++k) {
      const int q = q0 + tid + k * kThreads;
      if (q < ns_inj) s_inj[q] = (int32_t)(cum_count(R[k], n) - cum_count(R[k], n - 1));
    }
  }
  // ring emissions in patch-sorted source order
  for (int k = tid; k < d.ns; k += kThreads) {
    const int s = d.src_order[k];
    const SourceDev &S = d.sources[s];
    // the horizontal-motion ring, then the vertical-motion ring, each on its cadence
    const bool emit_h = S.E > 0 && ((n - 1) % S.E) == 0;
    const bool emit_v = S.Eh > 0 && ((n - 1) % S.Eh) == 0;
    const int ne = (emit_h ? S.ne : 0) + (emit_v ? S.ne : 0);
    s_em[k] = ne;
    if (ne) {
      const PatchDev &P = d.patches[S.patch];
      const double xs = S.x0 + S.vx * tn;
      const double ys = S.y0 + S.vy * tn;
      d.src_pos[s] = make_int2((int32_t)round_away((xs - P.ax) * 1048576.0),
                               (int32_t)round_away((ys - P.ay) * 1048576.0));
      atomicAdd(&d.ctr[((size_t)S.patch * d.nb + S.bucket) * CNT_NUM + CNT_EMIT], (unsigned long long)ne);
    }
  }
  __syncthreads();
  // counters of created particles (before the scan overwrites the counts)
  for (int q = tid; q < d.np * d.nb; q += kThreads) {
    const int c = s_inj[2 * q] + s_inj[2 * q + 1];
    if (c) atomicAdd(&d.ctr[(size_t)q * CNT_NUM + CNT_INJ], (unsigned long long)c);
  }
  __syncthreads();
  const int32_t tot_inj = block_scan_excl(s_inj, ns_inj, s_tmp);
  if (tid == 0) s_inj[ns_inj] = tot_inj;
  const int32_t tot_em = block_scan_excl(s_em, d.ns, s_tmp);
  if (tid == 0) s_em[d.ns] = tot_em;
  __syncthreads();
  for (int q = tid; q <= ns_inj; q += kThreads) d.inj_off[q] = s_inj[q];
  for (int k = tid; k <= d.ns; k += kThreads) d.em_off[k] = s_em[k];
  for (int p = tid; p < d.np; p += kThreads) {
    const PatchDev &P = d.patches[p];
    StepPatch &W = d.sp[p];
    W.inj_lo = s_inj[p * 2 * d.nb];
    W.inj_hi = s_inj[(p + 1) * 2 * d.nb];
    W.em_lo = s_em[P.src_lo];
    W.em_hi = s_em[P.src_hi];
  }
}

// ---------------------------------------------------------------- update
// Survival and bin key of a particle at age `age` (>= 0).  -1 if it dies.
__device__ __forceinline__ int32_t survive_key(const Dev &d, const PatchDev &P, const StepPatch &W,
                                               int bucket, int code, bool boundary, int32_t ox, int32_t oy,
                                               int32_t age, int64_t &px, int64_t &py) {
  if (age > kAgeMax) return -1;
  const int2 v = velocity(d, bucket, code, boundary);
  px = (int64_t)ox + (((int64_t)age * v.x) >> 12);
  py = (int64_t)oy + (((int64_t)age * v.y) >> 12);
  const int64_t m = d.margin[bucket];
  const int64_t lox = (int64_t)W.wx * P.dxu - m, hix = (int64_t)(W.wx + P.nx) * P.dxu + m;
  const int64_t loy = (int64_t)W.wy * P.dxu - m, hiy = (int64_t)(W.wy + P.ny) * P.dxu + m;
  if (px < lox || px > hix || py < loy || py > hiy) return -1;
  const uint64_t binm = P.binm[bucket];   // 1 / bin edge, 64.64 fixed point rounded up
  const uint32_t bx = (uint32_t)__umul64hi(binm, (uint64_t)(uint32_t)(px - lox));
  const uint32_t by = (uint32_t)__umul64hi(binm, (uint64_t)(uint32_t)(py - loy));
  return P.binbase[bucket] + (int32_t)(by * (uint32_t)P.nbx[bucket] + bx);
}

// Wave-level run merge: lanes with equal consecutive keys form a run.
// Returns for each valid lane its head lane and rank in the run; heads also
// get the run length.
struct Run {
  int head, rank, len;
  bool is_head;
};
__device__ __forceinline__ Run wave_runs(int32_t key) {
  const int lane = (int)__lane_id();
  const int32_t prev = __shfl_up(key, 1);
  const bool valid = key >= 0;
  const bool h = valid && (lane == 0 || prev != key);
  const uint64_t hm = __ballot(h);
  const uint64_t bm = __ballot(h || !valid);
  Run r;
  const uint64_t below = hm & ((2ull << lane) - 1ull);
  r.head = below ? 63 - __clzll((long long)below) : 0;
  r.rank = lane - r.head;
  const uint64_t above = bm & ~((2ull << lane) - 1ull);
  const int next = above ? (__ffsll((long long)above) - 1) : 64;
  r.len = next - lane;
  r.is_head = h;
  return r;
}

// Add inc to counter ctr[key] for every lane with key >= 0: one atomic per
// distinct key in the wavefront (lanes of a wavefront nearly always share
// their patch and bucket, so this is usually a single atomic).
__device__ __forceinline__ void wave_add(unsigned long long *ctr, int key, uint32_t inc) {
  uint64_t act = __ballot(key >= 0);
  while (act) {
    const int leader = __builtin_ctzll(act);
    const int lk = __shfl(key, leader);
    const bool mine = key == lk;
    const uint64_t same = __ballot(mine);
    uint32_t v = mine ? inc : 0u;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((int)__lane_id() == leader) atomicAdd(&ctr[lk], (unsigned long long)v);
    act &= ~same;
  }
}

// Subdivision (at most one level per step): a ring particle whose age has
// reached its source's split age for its level becomes three, at codes
// c - a0/3^(L+1), c, c + a0/3^(L+1), each a third of the amplitude.  o[0] is
// the particle itself (or the middle child).  Returns the number of outputs.
__device__ __forceinline__ int subdivide(const Dev &d, const Part &q, Part o[3]) {
  o[0] = q;
  const uint32_t lev = m_level(q.meta);
  if (m_kind(q.meta) != 1 || (int)lev >= d.lmax) return 1;
  const SourceDev &S = d.sources[m_src(q.meta)];
  if (q.age < S.T[lev]) return 1;
  int off = S.a0;
  for (uint32_t l = 0; l <= lev; ++l) off /= 3;
  o[0].meta = (q.meta & ~7u) | (lev + 1);
  o[0].amp = q.amp * (1.0f / 3.0f);
  o[1] = o[0];
  o[2] = o[0];
  o[1].code = (q.code - off + kNCode) % kNCode;
  o[2].code = (q.code + off) % kNCode;
  return 3;
}

// The next step's bin histogram and subdivided/died counters of a particle
// as it stands after step n (its outputs at step n + 1: subdivision at age
// + 1, survival against the window of step n + 1).  Adding them while the
// particle is written saves the next step a pass over every record.  All
// lanes of the wavefront call this (ballots inside).
__device__ __forceinline__ void predict_next(const Dev &d, const Part &q, bool valid) {
  Part c[3];
  int32_t key[3] = {-1, -1, -1};
  int pid = 0, bkt = 0;
  bool sub = false;
  uint32_t ndead = 0;
  if (valid) {
    Part q1 = q;
    q1.age = q.age + 1;
    const int nc = subdivide(d, q1, c);
    sub = nc == 3;
    pid = (int)m_patch(q.meta);
    bkt = (int)m_bucket(q.meta);
    const PatchDev &P = d.patches[pid];
    const StepPatch W = d.sp_next[pid];
    const bool boundary = m_kind(q.meta) == 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (r < nc) {
        int64_t px, py;
        key[r] = survive_key(d, P, W, bkt, c[r].code, boundary, c[r].ox, c[r].oy, c[r].age, px, py);
        if (key[r] < 0) ++ndead;
      }
    }
  }
  const int cbase = (pid * d.nb + bkt) * CNT_NUM;
  wave_add(d.ctr_next, sub ? cbase + CNT_SUB : -1, 1u);
  wave_add(d.ctr_next, ndead ? cbase + CNT_DIED : -1, ndead);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    if (r > 0 && __ballot(key[r] >= 0) == 0ull) continue;
    const Run run = wave_runs(key[r]);
    if (run.is_head) atomicAdd(&d.hist[key[r]], run.len);
  }
}

// Modes of the update pass.
//   kCountNew   the bin histogram of the particles created this step
//               (injected and emitted); the previous step's scatter already
//               counted the particles that carry over
//   kScatter    all particles of the step in bin order into the output
//               buffer, and the next step's histogram of what was written
enum { kCountNew = 0, kScatter = 1 };

template <class Rec, int kMode>
__global__ __launch_bounds__(kThreads) void k_update(Dev d, int p0, int p1) {
  const int64_t n = d.glob->n;
  const Rec *__restrict__ Sin = (const Rec *)(((n - 1) & 1) ? d.S1 : d.S0);
  Rec *__restrict__ Sout = (Rec *)((n & 1) ? d.S1 : d.S0);
  const StepPatch A = d.sp[p0], B = d.sp[p1 - 1];
  const int ex0 = A.ex_lo, nex = max(0, B.ex_hi - A.ex_lo);
  const int in0 = A.inj_lo, ninj = B.inj_hi - A.inj_lo;
  const int em0 = A.em_lo, nem = B.em_hi - A.em_lo;
  const int total = nex + ninj + nem;
  const int kbeg = kMode == kCountNew ? nex : 0;   // counting skips the carried-over particles
  const int lane = (int)__lane_id();
  // injection slot offsets and direction CDFs, copied to LDS by the blocks
  // that hold new boundary particles (their searches then stay in LDS)
  __shared__ int32_t s_inj[kMaxInjSlots + 1];
  __shared__ uint32_t s_cdf[kMaxBuckets * 2 * kDirBins];
  bool tables = false;
  // the record of the thread's next previous particle is loaded one
  // iteration ahead
  const int stride = (int)gridDim.x * kThreads;
  Rec rec_next;
  {
    const int k0 = kbeg + (int)blockIdx.x * kThreads + (int)threadIdx.x;
    if (k0 < nex) rec_next = Sin[ex0 + k0];
  }
  if (kMode == kCountNew && p0 == 0) {
    // this step's subdivided and died counts of the carried-over particles,
    // found by the previous step's scatter (before this step's scatter
    // starts on the next step's)
    for (int q = (int)blockIdx.x * kThreads + (int)threadIdx.x; q < d.np * d.nb * CNT_NUM;
         q += (int)gridDim.x * kThreads) {
      const unsigned long long v = d.ctr_next[q];
      if (v) {
        atomicAdd(&d.ctr[q], v);
        d.ctr_next[q] = 0ull;
      }
    }
  }

  for (int base = kbeg + (int)blockIdx.x * kThreads; base < total; base += stride) {
    const int k = base + (int)threadIdx.x;
    const Rec rec = rec_next;
    if (k + stride < nex) rec_next = Sin[ex0 + k + stride];
    if (!tables && base < nex + ninj && base + kThreads > nex) {   // block-uniform
      for (int i = threadIdx.x; i <= d.n_inj_slots; i += kThreads) s_inj[i] = d.inj_off[i];
      for (int i = threadIdx.x; i < d.nb * 2 * kDirBins; i += kThreads) s_cdf[i] = d.cdf[i];
      __syncthreads();
      tables = true;
    }
    Part o[3];
    int32_t key[3] = {-1, -1, -1};
    int nout = 0;
    int pid = 0, bkt = 0;
    bool subdivided = false;
    uint32_t ndead = 0;
    if (k < nex) {
      // ---- a previous particle: subdivide, then survive
      Part q = RecIO<Rec>::unpack(rec, n);
      if (!RecIO<Rec>::kHasAmp && q.age == 0) q.age = 65536;   // 16-bit birth wrapped: expired
      pid = (int)m_patch(q.meta);
      bkt = (int)m_bucket(q.meta);
      nout = subdivide(d, q, o);
      subdivided = nout == 3;
    } else if (k < nex + ninj) {
      // ---- a new boundary particle
      const int gi = in0 + (k - nex);
      int lo = 0, hi = d.n_inj_slots;   // last slot with inj_off[slot] <= gi
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_inj[mid] <= gi) lo = mid; else hi = mid;
      }
      const int slot = lo, j = gi - s_inj[slot];
      pid = slot / (2 * d.nb);
      bkt = (slot / 2) % d.nb;
      const int pair = slot & 1;
      uint64_t c[4] = {(uint64_t)pid, (uint64_t)(bkt * 2 + pair), (uint64_t)n, (uint64_t)j};
      philox4x64(c, d.seed, kStreamInject);
      const PatchDev &P0 = d.patches[pid];
      int code;
      if (!d.afac) {
        // inverse CDF of Dir (times the obliquity of this side pair, when
        // weighted) over the 64 direction bins
        const uint32_t Q = d.cdfQ[bkt * 2 + pair];
        const uint32_t t = (uint32_t)__umul64hi(c[0], (uint64_t)Q);
        const uint32_t *cdf = s_cdf + (bkt * 2 + pair) * kDirBins;
        int b = 0;   // smallest bin with t < cdf[b]
        for (int step = 32; step > 0; step >>= 1)
          if (cdf[b + step - 1] <= t) b += step;
        code = d.codes[b];
      } else {
        // stratified group: the m-th particle of this side pair's stream
        // takes sector m mod N_theta around the wind, uniformly inside it
        const int64_t nth = P0.ntheta;
        const int64_t m = cum_count(pair ? P0.Ry[bkt] : P0.Rx[bkt], n - 1) + j;
        const int64_t sct = m % nth;
        const int64_t lo = sct * kNCode / nth, hi = (sct + 1) * kNCode / nth;
        code = (int)((d.wind_code + kNCode / 2 + lo + (int64_t)__umul64hi(c[0], (uint64_t)(hi - lo))) % kNCode);
      }
      const PatchDev &P = d.patches[pid];
      const StepPatch W = d.sp[pid];
      const int2 v = d.V[bkt * kNCode + code];
      Part q;
      if (pair == 0) {
        q.ox = (v.x > 0) ? W.wx * P.dxu : (W.wx + P.nx) * P.dxu;
        q.oy = W.wy * P.dxu + (int32_t)__umul64hi(c[1], (uint64_t)P.ny * (uint64_t)P.dxu);
      } else {
        q.oy = (v.y > 0) ? W.wy * P.dxu : (W.wy + P.ny) * P.dxu;
        q.ox = W.wx * P.dxu + (int32_t)__umul64hi(c[1], (uint64_t)P.nx * (uint64_t)P.dxu);
      }
      q.age = 0;
      q.code = code;
      q.meta = pack_meta(0, 0, bkt, pid, kNoSource, 0);
      q.amp = P.A[bkt] * (d.afac ? d.afac[bkt * kNCode + code] : 1.f);
      o[0] = q;
      nout = 1;
    } else if (k < total) {
      // ---- a new ring particle
      const int gi = em0 + (k - nex - ninj);
      int lo = 0, hi = d.ns;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (d.em_off[mid] <= gi) lo = mid; else hi = mid;
      }
      const int s = d.src_order[lo];
      const SourceDev &S = d.sources[s];
      // the source's block: its horizontal-motion ring (when emitted this
      // step) first, then its vertical-motion ring
      const bool emit_h = S.E > 0 && ((n - 1) % S.E) == 0;
      int j = gi - d.em_off[lo];
      const bool heave = !emit_h || j >= S.ne;
      if (heave && emit_h) j -= S.ne;
      const int2 sp = d.src_pos[s];
      const int2 O = d.ring_O[S.ring0 + j];
      pid = S.patch;
      bkt = S.bucket;
      Part q;
      q.ox = sp.x + O.x;
      q.oy = sp.y + O.y;
      q.age = 0;
      q.code = j * S.a0;
      q.meta = pack_meta(0, 1, bkt, pid, s, j) | (heave ? kHeaveBit : 0u);
      q.amp = heave ? heave_amp(S, n, 0u) : S.B * d.ring_m[S.ring0 + j];
      o[0] = q;
      nout = 1;
    }
    if (nout) {
      const PatchDev &P = d.patches[pid];
      const StepPatch W = d.sp[pid];
#pragma unroll
      for (int r = 0; r < 3; ++r) {   // constant bound: o[] and key[] stay in registers
        if (r < nout) {
          int64_t px, py;
          key[r] = survive_key(d, P, W, (int)m_bucket(o[r].meta), o[r].code, m_kind(o[r].meta) == 0, o[r].ox,
                               o[r].oy, o[r].age, px, py);
          if (key[r] < 0) ++ndead;
        }
      }
    }
    if (kMode == kCountNew) {
      // only new particles here: none subdivides, some die at once
      const int cbase = (pid * d.nb + bkt) * CNT_NUM;
      wave_add(d.ctr, ndead ? cbase + CNT_DIED : -1, ndead);
    }
    // merge runs of equal keys, one atomic per run
    bool written[3] = {false, false, false};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (r > 0 && __ballot(key[r] >= 0) == 0ull) continue;
      const Run run = wave_runs(key[r]);
      if (kMode == kCountNew) {
        if (run.is_head) atomicAdd(&d.hist[key[r]], run.len);
      } else {
        int32_t basepos = 0;
        if (run.is_head) basepos = atomicAdd(&d.cur[key[r]], run.len);
        basepos = __shfl(basepos, run.head);
        if (key[r] >= 0) {
          const int32_t slotpos = basepos + run.rank;
          if (slotpos < d.cap) {
            RecIO<Rec>::store(Sout, slotpos, o[r], n);
            written[r] = true;
          } else {
            atomicAdd(&d.glob->dropped, 1ull);
          }
        }
      }
    }
    if (kMode == kScatter) {
      // this step's subdivided / died counts of carried-over particles were
      // added by the previous step's scatter; the next step's are added here
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (r > 0 && __ballot(written[r]) == 0ull) continue;
        predict_next(d, o[r], written[r]);
      }
    }
    (void)lane;
  }
}

// The next step's histogram and counters of the particles in the current
// buffer (after a restore, when no scatter has predicted them).
template <class Rec>
__global__ __launch_bounds__(kThreads) void k_predict(Dev d, int p0, int p1) {
  const int64_t n = d.glob->n;
  const Rec *__restrict__ S = (const Rec *)((n & 1) ? d.S1 : d.S0);
  const int lo = min(d.off[d.patches[p0].bin_lo], d.cap), hi = min(d.off[d.patches[p1 - 1].bin_hi], d.cap);
  for (int base = lo + (int)blockIdx.x * kThreads; base < hi; base += (int)gridDim.x * kThreads) {   // block-uniform
    const int k = base + (int)threadIdx.x;
    Part q;
    const bool valid = k < hi;
    if (valid) q = RecIO<Rec>::unpack(S[k], n);   // age 0: born this step
    predict_next(d, q, valid);
  }
}

// ---------------------------------------------------------------- scan
constexpr int kScanPer = 8;
constexpr int kScanChunk = kThreads * kScanPer;

int scan_blocks(int nbins) { return (nbins + kScanChunk - 1) / kScanChunk; }

__global__ __launch_bounds__(kThreads) void k_scan_a(Dev d, int lo, int hi) {
  __shared__ int32_t s[kThreads];
  const int beg = lo + blockIdx.x * kScanChunk;
  const int end = min(hi, beg + kScanChunk);
  int32_t v[kScanPer];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {   // all loads before the sum
    const int i = beg + (int)threadIdx.x + k * kThreads;
    v[k] = i < end ? d.hist[i] : 0;
  }
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) sum += v[k];
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.bsum[blockIdx.x] = s[0];
}

// Block b: prefix of the block sums before it, then an exclusive scan of
// its chunk (each thread 8 consecutive bins, wave scans via shuffles).
__global__ __launch_bounds__(kThreads) void k_scan_b(Dev d, int lo, int hi, int first, int last) {
  __shared__ int32_t s_w[kThreads / 64 + 1];
  __shared__ int32_t s_pre;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // prefix of earlier blocks
  int32_t pre = 0;
  for (int i = tid; i < (int)blockIdx.x; i += kThreads) pre += d.bsum[i];
  for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o);
  if (lane == 0) s_w[wv] = pre;
  __syncthreads();
  if (tid == 0) {
    int32_t base = first ? 0 : d.off[lo];
    for (int w = 0; w < kThreads / 64; ++w) base += s_w[w];
    s_pre = base;
  }
  __syncthreads();
  const int32_t start = s_pre;
  const int beg = lo + blockIdx.x * kScanChunk + tid * kScanPer;
  int32_t v[kScanPer];
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int i = beg + k;
    v[k] = (i < hi) ? d.hist[i] : 0;
    sum += v[k];
  }
  // inclusive scan of per-thread sums across the wave
  int32_t inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  int32_t wpre = 0;
  for (int w = 0; w < wv; ++w) wpre += s_w[w];
  int32_t acc = start + wpre + inc - sum;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int i = beg + k;
    if (i < hi) {
      d.off[i] = acc;
      d.cur[i] = acc;
      d.hist[i] = 0;
    }
    acc += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == kThreads - 1) {
    // acc now holds the running total after the last bin of this block
    d.off[hi] = acc;
    if (last) {
      d.glob->total = acc;
      d.glob->n_live = min(acc, d.cap);
    }
  }
}

// ---------------------------------------------------------------- CDF
// One wavefront per (bucket, side pair): inclusive scan of the 64 integer
// direction weights (exact), giving the inverse-CDF table for injection.
__global__ void k_cdf(const uint32_t *q, uint32_t *cdf, uint32_t *cdfQ) {
  const int b = blockIdx.x, lane = threadIdx.x;
  uint32_t v = q[b * kDirBins + lane];
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  cdf[b * kDirBins + lane] = v;
  if (lane == 63) cdfQ[b] = v;
}

void launch_cdf(const Dev &d, const uint32_t *q, uint32_t *cdf, uint32_t *cdfQ, hipStream_t st) {
  hipLaunchKernelGGL(k_cdf, dim3(d.nb * 2), dim3(64), 0, st, q, cdf, cdfQ);
}

// ---------------------------------------------------------------- launchers
void launch_params(const Dev &d, hipStream_t st) {
  hipLaunchKernelGGL(k_params, dim3(1), dim3(kThreads), 0, st, d);
}

void launch_windows(const Dev &d, hipStream_t st) {
  hipLaunchKernelGGL(k_windows, dim3(1), dim3(kThreads), 0, st, d);
}

void launch_update(const Dev &d, int p0, int p1, bool scatter, int grid, hipStream_t st) {
  if (d.compact) {
    if (scatter) hipLaunchKernelGGL((k_update<RecCompact, kScatter>), dim3(grid), dim3(kThreads), 0, st, d, p0, p1);
    else hipLaunchKernelGGL((k_update<RecCompact, kCountNew>), dim3(grid), dim3(kThreads), 0, st, d, p0, p1);
  } else {
    if (scatter) hipLaunchKernelGGL((k_update<RecWide, kScatter>), dim3(grid), dim3(kThreads), 0, st, d, p0, p1);
    else hipLaunchKernelGGL((k_update<RecWide, kCountNew>), dim3(grid), dim3(kThreads), 0, st, d, p0, p1);
  }
}

// Blocks of the update pass resident per compute unit (the persistent grid
// must fit in one round, or its last blocks would run after the others).
int update_blocks_per_cu(bool compact, bool scatter) {
  int nb = 0;
  hipError_t e;
  if (compact)
    e = scatter ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update<RecCompact, kScatter>, kThreads, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update<RecCompact, kCountNew>, kThreads, 0);
  else
    e = scatter ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update<RecWide, kScatter>, kThreads, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update<RecWide, kCountNew>, kThreads, 0);
  return (e == hipSuccess && nb > 0) ? nb : 4;
}

void launch_predict(const Dev &d, int p0, int p1, int grid, hipStream_t st) {
  if (d.compact) hipLaunchKernelGGL((k_predict<RecCompact>), dim3(grid), dim3(kThreads), 0, st, d, p0, p1);
  else hipLaunchKernelGGL((k_predict<RecWide>), dim3(grid), dim3(kThreads), 0, st, d, p0, p1);
}

void launch_scan(const Dev &d, int lo, int hi, bool first, bool last, hipStream_t st) {
  const int nblk = scan_blocks(hi - lo);
  if (nblk > 1) hipLaunchKernelGGL(k_scan_a, dim3(nblk), dim3(kThreads), 0, st, d, lo, hi);
  hipLaunchKernelGGL(k_scan_b, dim3(nblk > 0 ? nblk : 1), dim3(kThreads), 0, st, d, lo, hi, first ? 1 : 0,
                     last ? 1 : 0);
}

}  // namespace hwo

// hwo_dev.h -- internal definitions of the gfx950 hybrid-ocean library.
//
// Fixed-point conventions (shared as a *format* with the oracle, each side
// writes its own code):
//   positions   int32, 2^-20 m units, relative to the patch anchor
//   velocity    int32 per step, 2^-32 m units; position(age) =
//               origin + floor(age * V / 4096)
//   directions  integer codes, 2 pi / 10368 per unit (2 * 64 * 3^4)
//   rates       32.32 fixed point groups*eta per step; count(n) =
//               floor(n R / 2^32) - floor((n - 1) R / 2^32)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hwo {

constexpr int kMaxBuckets = 16;
constexpr int kDirBins = 64;
constexpr int kMaxLevel = 4;
constexpr int kNCode = 10368;
constexpr int kAgeMax = 65535;
constexpr int kMaxPatches = 127;
constexpr int kMaxSources = 127;
constexpr int kMaxInjSlots = 2 * kMaxBuckets * kMaxPatches;   // (patch, bucket, side pair) injection slots
constexpr int kMaxRing = 128;
constexpr uint32_t kNoSource = 127;
constexpr int kTile = 64;          // splat output tile edge (cells)
constexpr int kThreads = 256;
constexpr uint64_t kStreamInject = 1;
constexpr uint64_t kStreamH0 = 2;

// ---------------------------------------------------------------- records
// meta word: level 0-2 | kind 3 | bucket 4-7 | patch 8-14 | src 15-21 | slot 22-28 | heave 29
// (kind 1 is a ring particle; the heave bit marks the rings of vertical motion)
__host__ __device__ inline uint32_t pack_meta(uint32_t level, uint32_t kind, uint32_t bucket,
                                              uint32_t patch, uint32_t src, uint32_t slot) {
  return level | (kind << 3) | (bucket << 4) | (patch << 8) | (src << 15) | (slot << 22);
}
__host__ __device__ inline uint32_t m_level(uint32_t m) { return m & 7u; }
__host__ __device__ inline uint32_t m_kind(uint32_t m) { return (m >> 3) & 1u; }
__host__ __device__ inline uint32_t m_bucket(uint32_t m) { return (m >> 4) & 15u; }
__host__ __device__ inline uint32_t m_patch(uint32_t m) { return (m >> 8) & 127u; }
__host__ __device__ inline uint32_t m_src(uint32_t m) { return (m >> 15) & 127u; }
__host__ __device__ inline uint32_t m_slot(uint32_t m) { return (m >> 22) & 127u; }
constexpr uint32_t kHeaveBit = 1u << 29;
__host__ __device__ inline bool m_heave(uint32_t m) { return (m & kHeaveBit) != 0u; }

// Plain form: 32 bytes, every attribute a full 32-bit word, amplitude FP32.
struct RecWide {
  int32_t ox, oy;
  int32_t birth;
  int32_t code;
  uint32_t meta;
  float amp;
  int32_t pad0, pad1;
};
// Compact form: 16 bytes; birth modulo 2^16 (ages never exceed 65535) and
// code share a word; the amplitude is rebuilt from per-patch / per-ring
// tables, so no attribute is rounded.
struct RecCompact {
  int32_t ox, oy;
  uint32_t bc;   // birth & 0xffff | code << 16
  uint32_t meta;
};
static_assert(sizeof(RecWide) == 32, "wide record");
static_assert(sizeof(RecCompact) == 16, "compact record");

// Decoded particle.
struct Part {
  int32_t ox, oy;
  int32_t age;     // n - birth (>= 0); 65536 means expired
  int32_t code;
  uint32_t meta;
  float amp;       // wide form only
};

// ---------------------------------------------------------------- tables
struct PatchDev {
  double ax, ay, dx;
  int32_t nx, ny, dxu, follow;
  float band, ratio;           // blend band (m); dx / background cell
  float inv_band;
  int32_t bin_lo, bin_hi;      // bins of this patch in the global histogram
  int32_t tile0, ntx, nty;     // splat output tiles
  int32_t ntheta;              // directions per group (stratified mode)
  int32_t src_lo, src_hi;      // range in the patch-sorted source list
  int64_t cell0;               // offset of this patch in the height buffers
  float A[kMaxBuckets];        // boundary amplitude per bucket
  uint64_t Rx[kMaxBuckets], Ry[kMaxBuckets];
  int32_t binu[kMaxBuckets];   // bin edge (position units)
  uint64_t binm[kMaxBuckets];  // ceil(2^64 / binu): x / binu = high word of binm * x for any 32-bit x
  int32_t nbx[kMaxBuckets], nby[kMaxBuckets], binbase[kMaxBuckets];
  // texel-layer synthesis: per bucket, the x-filtered layer (rows of the
  // patch plus lay_R cells on every side, patch columns, row-major)
  int64_t lt_off[kMaxBuckets];
  int32_t lay_R[kMaxBuckets], tap_off[kMaxBuckets];
};

struct SourceDev {
  double x0, y0, vx, vy;
  float B;
  int32_t patch, bucket, ne, a0, E, ring0;
  int32_t T[kMaxLevel];
  // vertical motion: a ring every Eh steps (0: none), amplitude
  // Bh (z(birth - Eh) - z(birth)) with z = sin(2 pi n hf), hf = dt / heave period
  int32_t Eh;
  double Bh, hf;
};

// Amplitude of a vertical-motion ring particle born at step nb, level lv:
// the volume displaced between the ring before it and its birth.  The phase
// n dt / heave_T is reduced to [0, 1) in FP64 and its sine taken by the
// hardware sine, which works in revolutions (absolute error ~1e-7).
__device__ inline float heave_amp(const SourceDev &S, int64_t nb, uint32_t lv) {
  double p0 = (double)(nb - S.Eh) * S.hf, p1 = (double)nb * S.hf;
  p0 -= floor(p0);
  p1 -= floor(p1);
  const float dz = __builtin_amdgcn_sinf((float)p0) - __builtin_amdgcn_sinf((float)p1);
  const float inv3 = lv == 0 ? 1.f : lv == 1 ? 1.f / 3.f : lv == 2 ? 1.f / 9.f : lv == 3 ? 1.f / 27.f : 1.f / 81.f;
  return (float)S.Bh * dz * inv3;
}

struct StepPatch {             // per patch, rewritten every step
  int32_t wx, wy;              // window origin (cells)
  int32_t gx0, gy0;            // background cell of the first patch cell
  float fx0, fy0;              // fractional offset, FP64-derived
  int32_t ex_lo, ex_hi;        // previous particles of this patch in the input buffer
  int32_t inj_lo, inj_hi;      // new boundary particles
  int32_t em_lo, em_hi;        // new ring particles
};

struct Globals {
  int64_t n;                   // current step
  int32_t n_live;              // particles in the current buffer (<= capacity)
  int32_t total;               // live particles counted this step (may exceed capacity)
  unsigned long long dropped;  // particles lost to capacity, cumulative
  int32_t err;                 // bit 0: position range exceeded
  int32_t pad;
};

// Per-bucket splat profile (wavefront clock ticks of s_memtime, summed over
// wavefronts; points visited): categories of a work item's time.
enum {
  PROF_SETUP = 0,    // item set-up: row tables, prefix of the lists, part shares
  PROF_DECODE = 1,   // records decoded into crest/trough points (and the barrier after)
  PROF_WAIT = 2,     // end-of-chunk barrier: waiting for the other wavefronts
  PROF_EPILOGUE = 3, // quadrants into the tile, blend or partial tile store
  PROF_BUCKET = 4,   // + b: footprints of bucket b
  PROF_POINTS = PROF_BUCKET + kMaxBuckets,   // + b: crest and trough points of bucket b visited
  PROF_N = PROF_POINTS + kMaxBuckets
};

enum { CNT_INJ = 0, CNT_EMIT, CNT_SUB, CNT_DIED, CNT_NUM };

// Everything a kernel needs, passed by value.
struct Dev {
  int32_t np, ns, nb, N, cap, nbins, ntiles, compact, lmax;
  int32_t n_inj_slots;         // np * nb * 2
  int32_t wind_code;           // wind direction in direction-code units
  double g, dt, L, dxf;
  uint64_t seed;
  const PatchDev *patches;
  const SourceDev *sources;
  const int32_t *src_order;    // sources sorted by patch
  const int2 *V;               // [nb][kNCode] velocity per step
  const int2 *Vbin;            // [nb][kDirBins] velocity of each direction bin's code (boundary particles)
  const float2 *UC;            // [kNCode] unit direction
  const float *afac;           // [nb][kNCode] stratified-direction amplitude factor sqrt(2 pi Dir); null: inverse-CDF mode
  const uint32_t *cdf;         // [nb][side pair][64] inclusive integer CDF
  const uint32_t *cdfQ;        // [nb][side pair] totals
  const int32_t *codes;        // [64] direction code of each bin
  const float *bucket_r;       // [nb] radius (m)
  const int32_t *margin;       // [nb] ceil(2 r 2^20)
  const float *ring_m;         // [sum ne] ring multipliers
  const float *ring_amp;       // [ns][kMaxRing] ring amplitude B m of each slot before subdivision
  const int2 *ring_O;          // [sum ne] ring offsets (units)
  Globals *glob;
  StepPatch *sp;
  StepPatch *sp_next;          // windows of the next step (the scatter counts the next step's bins)
  int32_t *inj_off;            // [n_inj_slots + 1]
  int32_t *em_off;             // [ns + 1]
  int2 *src_pos;               // [ns] source position (units, patch frame)
  unsigned long long *ctr;     // [np][nb][CNT_NUM]
  unsigned long long *ctr_next;   // [np][nb][CNT_NUM] the next step's subdivided / died counts so far
  int32_t *hist, *off, *cur, *bsum;
  void *S0, *S1;               // particle buffers; step n reads S[(n-1)&1], writes S[n&1]
  const float2 *h0T;           // [N][N] h0 transposed: row = kx index
  const float2 *tw;            // [N] e^{2 pi i k / N}
  int32_t nfields;             // background fields: 1 height, or 5 (+ dH/dx, dH/dy, choppy Dx, Dy)
  int32_t fft_mfma16;          // 1: first FFT stage as a radix-16 DFT on the matrix cores (split bf16)
  int32_t splat_kernel;        // splat schedule: 0 batches per wavefront, 1 quadrant per wavefront, 2 both in turn
  float2 *FT;                  // [nfields][N/2+1][N]
  float *H;                    // [nfields][N][N], field 0 the height
  float *raw, *blend;          // heights, all patches
  // splat work plan
  uint32_t *tile_load;         // [ntiles] estimated splat cost per output tile (model units)
  int32_t *item_base;          // [ntiles + 1] first work item of each tile (plan)
  int4 *item_desc;             // [max_items] tile, part, parts of the tile, patch (plan)
  const int32_t *tile_patch;   // [ntiles] patch of each output tile
  const short4 *tile_rect;     // [ntiles][nb] bins reaching the tile: bx_lo, bx_hi, by_lo, nrows
  uint32_t *tile_meas;         // [ntiles] splat time of the tile this frame (100 MHz ticks)
  uint32_t *tile_model;        // [ntiles] model estimate the current plan was made from
  float *tile_ratio;           // [ntiles] running average of measured / estimated (scene mean 1)
  int32_t *splat_ctl;          // [1] total items, [2] split tiles (plan)
  int32_t *split_tiles;        // [ntiles] tiles with more than one part (plan)
  float *partials;             // [max_items][kTile * kTile] partial tiles of split tiles
  int32_t max_items;           // capacity of partials (items)
  uint32_t chunk_load;         // least estimated cost of a work item
  int32_t radial;              // 1: radial kernel W(|d|) instead of w(dx) w(dy) (exact splat only)
  // texel-layer synthesis (synth == 1)
  int32_t synth;
  int32_t n_xtiles;            // 64 x 64 tiles of all x-filtered layers
  int64_t ncells;              // cells of all patches
  float *lt;                   // x-filtered layers
  float *yplanes;              // [nb][ncells] per-bucket maps after the y pass
  const float *taps;           // raised cosine at whole-cell offsets, 2R+1 per (patch, bucket)
  const int32_t *xt_base;      // [np * nb + 1] first x tile of each (patch, bucket)
  int32_t xparts;              // most parts per x tile (1: no cutting)
  int32_t *xt_nparts;          // [n_xtiles] parts of each x tile this frame
  float *xpartial;             // [n_xtiles][xparts][64 * 64] partial x-filtered tiles
  const int2 *toff;            // [nb][kNCode] trough offset round(r (cos, sin) 2^20)
  int32_t lsmem;               // dynamic LDS bytes of the layer passes
  float *nrm;                  // [3][ncells] unit normals (x, y, z planes); null unless enabled
  unsigned long long *splat_prof;   // [PROF_N] per-bucket splat profile
  int32_t splat_profile;            // 1: launch the profiling instance of the splat
};

// ---------------------------------------------------------------- helpers
__host__ __device__ inline int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}

// Round half away from zero, exact for |x| < 2^52 (x - trunc(x) is exact).
__device__ inline int64_t round_away(double x) {
  double t = trunc(x);
  double f = x - t;
  if (f >= 0.5) t += 1.0;
  else if (f <= -0.5) t -= 1.0;
  return (int64_t)t;
}

// Philox4x64-10 (Salmon et al., SC'11).
__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    uint64_t n0 = hi1 ^ c[1] ^ k0;
    uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__device__ inline int64_t cum_count(uint64_t R, int64_t n) {
  uint64_t hi = R >> 32, lo = R & 0xFFFFFFFFull;
  return (int64_t)((uint64_t)n * hi + (((uint64_t)n * lo) >> 32));
}

template <class Rec> struct RecIO;

template <> struct RecIO<RecWide> {
  __device__ static Part load(const RecWide *S, int64_t i, int64_t n) { return unpack(S[i], n); }
  __device__ static Part unpack(const RecWide &r, int64_t n) {
    Part p;
    p.ox = r.ox; p.oy = r.oy; p.code = r.code; p.meta = r.meta; p.amp = r.amp;
    p.age = (int32_t)(n - (int64_t)r.birth);
    return p;
  }
  __device__ static void store(RecWide *S, int64_t i, const Part &p, int64_t n) {
    RecWide r;
    r.ox = p.ox; r.oy = p.oy; r.birth = (int32_t)(n - p.age); r.code = p.code; r.meta = p.meta;
    r.amp = p.amp; r.pad0 = 0; r.pad1 = 0;
    S[i] = r;
  }
  static constexpr bool kHasAmp = true;
};

template <> struct RecIO<RecCompact> {
  __device__ static Part load(const RecCompact *S, int64_t i, int64_t n) { return unpack(S[i], n); }
  __device__ static Part unpack(const RecCompact &r, int64_t n) {
    Part p;
    p.ox = r.ox; p.oy = r.oy; p.code = (int32_t)(r.bc >> 16); p.meta = r.meta; p.amp = 0.f;
    uint32_t a = ((uint32_t)n - (r.bc & 0xFFFFu)) & 0xFFFFu;
    p.age = (int32_t)a;   // 0 for a stored particle means 65536 (expired); callers fix up
    return p;
  }
  __device__ static void store(RecCompact *S, int64_t i, const Part &p, int64_t n) {
    RecCompact r;
    r.ox = p.ox; r.oy = p.oy;
    r.bc = ((uint32_t)(n - p.age) & 0xFFFFu) | ((uint32_t)p.code << 16);
    r.meta = p.meta;
    S[i] = r;
  }
  static constexpr bool kHasAmp = false;
};

// Amplitude of a particle: boundary particles carry the patch/bucket
// amplitude (times the direction factor in stratified mode); ring particles
// B * m_slot / 3^level.
template <class Rec>
__device__ inline float particle_amp(const Dev &d, const Part &p, int64_t n) {
  if (RecIO<Rec>::kHasAmp) return p.amp;
  uint32_t m = p.meta;
  if (m_kind(m) == 0)
    return d.patches[m_patch(m)].A[m_bucket(m)] * (d.afac ? d.afac[m_bucket(m) * kNCode + p.code] : 1.f);
  const SourceDev &s = d.sources[m_src(m)];
  if (m_heave(m)) return heave_amp(s, n - p.age, m_level(m));
  // 3^-level, each constant correctly rounded (a select chain, not a local array)
  const uint32_t lv = m_level(m);
  const float inv3 = lv == 0 ? 1.f : lv == 1 ? 1.f / 3.f : lv == 2 ? 1.f / 9.f : lv == 3 ? 1.f / 27.f : 1.f / 81.f;
  return s.B * d.ring_m[s.ring0 + m_slot(m)] * inv3;
}

// Velocity per step of a particle.  Boundary particles drawn from the 64
// direction bins (inverse-CDF mode, d.afac null) carry a bin's code, so their
// velocities come from the small per-bin table, which stays in the L1 cache;
// other codes (ring particles, stratified directions) read the full table.
__device__ __forceinline__ int2 velocity(const Dev &d, int bucket, int code, bool boundary) {
  if (boundary && !d.afac) {
    const int t = ((code - d.wind_code - kNCode / 2 - kNCode / (2 * kDirBins)) % kNCode + kNCode) % kNCode;
    if (t % (kNCode / kDirBins) == 0) return d.Vbin[bucket * kDirBins + t / (kNCode / kDirBins)];
  }
  return d.V[bucket * kNCode + code];   // any other code (caller-placed records included)
}

// ---------------------------------------------------------------- output tiles
// Patch maps are cut into kTile x kTile output tiles, numbered patch by patch.
struct TileGeom {
  int p, i0, j0, tw, th;
  float Ab;            // boundary amplitude of the bucket being splatted
  int64_t X0, Y0;      // first cell centre (position units)
  float inv_dxu;
};

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
  const float t = fminf(dd * P.inv_band, 1.f);
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


// ---------------------------------------------------------------- launchers
void launch_h0(const Dev &d, float2 *h0T, float2 *tw, double alpha, double wp, double gamma,
               double s_const, double wind_dir, int h0_mode, hipStream_t st);
void launch_fft_a(const Dev &d, hipStream_t st);
void launch_fft_b(const Dev &d, hipStream_t st);
void launch_params(const Dev &d, hipStream_t st);
// Windows of every patch at the current step (no advance).
void launch_windows(const Dev &d, hipStream_t st);
void launch_update(const Dev &d, int p0, int p1, bool scatter, int grid, hipStream_t st);
int update_blocks_per_cu(bool compact, bool scatter);
// The next step's histogram and counters of the current buffer (after a restore).
void launch_predict(const Dev &d, int p0, int p1, int grid, hipStream_t st);
void launch_scan(const Dev &d, int bin_lo, int bin_hi, bool first, bool last, hipStream_t st);
void launch_splat_plan(const Dev &d, int t0, int ntiles, int items_target, hipStream_t st);
void launch_splat_tiles(const Dev &d, int t0, int ntiles, int grid, hipStream_t st);
// Fused scan + tile estimates + plan for a whole small scene (one block).
bool bin_plan_fits(int nbins, int ntiles, int nb);
void launch_bin_plan(const Dev &d, int nbins, int ntiles, int items_target, hipStream_t st);
void launch_splat_reduce(const Dev &d, int t0, int ntiles, hipStream_t st);
void launch_splat_direct(const Dev &d, int t0, int ntiles, const void *recs, int n, float *raw,
                         int64_t out_off, hipStream_t st);
void launch_cdf(const Dev &d, const uint32_t *q, uint32_t *cdf, uint32_t *cdfQ, hipStream_t st);
// Texel-layer synthesis.
hipError_t prepare_layers(const Dev &d);
void launch_deposit_x(const Dev &d, const void *recs, int n, hipStream_t st);
void launch_filter_y(const Dev &d, int t0, int ntiles, hipStream_t st);
void launch_layer_sum(const Dev &d, int p0, int p1, int64_t cells, float *raw, float *blend, int64_t out_off,
                      hipStream_t st);
// Finite-difference normals of the blended maps.
void launch_normals(const Dev &d, hipStream_t st);
// Height and unit normal at n world points (double2 in, float4 out, device).
void launch_probes(const Dev &d, const void *xy, int n, void *out, hipStream_t st);
int scan_blocks(int nbins);

}  // namespace hwo

/* hwo.h -- C ABI of the MI355X hybrid-ocean hot path.
 *
 * Per frame the library computes, on one gfx950 GPU (Xue et al., "Real-Time
 * Interactive Hybrid Ocean: Spectrum-Consistent Wave Particle-FFT Coupling",
 * arXiv 2511.02852):
 *   (a) the FFT background: directional JONSWAP spectrum (Sec 3.1, Eq 1-6),
 *       evolved under deep-water dispersion and inverse-transformed (Sec 4.1);
 *   (b) boundary injection of wave particles into every patch, per frequency
 *       bucket, with counts from Eq 18 and directions drawn from the
 *       same directional spectrum (Sec 3.3, Sec 4.2);
 *   (c) propagation at each bucket's phase speed c_i = g / w_i (Sec 3.2),
 *       ring emission from moving sources into the closest-radius bucket
 *       (Sec 4.3) and 3-way subdivision of ring particles;
 *   (d) the per-bucket splat of the raised-cosine crest/trough particle pair
 *       (Fig 1, Sec 4.2) into patch height maps, layers summed;
 *   (e) the blend of each patch map with the background (Sec 3.1, Sec 4.2).
 *
 * Conventions
 *   - Every function returns an int status: HWO_OK (0) or a negative code;
 *     hwo_last_error() gives a message.  No exception crosses the ABI.
 *   - The library owns all device state (allocated through the caller's
 *     allocator if given).  The caller owns every destination buffer.
 *   - Scene calls (set_spectrum, add_patch, add_source, set_bins) must come
 *     before the first step; afterwards they fail with HWO_ESTATE.
 *   - hwo_step is asynchronous on the library stream; read_* calls
 *     synchronise that stream.  One handle must not be used from two threads
 *     at once.
 *   - Patch and source ids are dense, in call order; they select the RNG
 *     streams, so the same scene and seed always give the same particles.
 */
#ifndef HWO_H
#define HWO_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HWO_OK = 0,
    HWO_EINVAL = -1,    /* bad argument */
    HWO_ESTATE = -2,    /* call out of order */
    HWO_ENOMEM = -3,    /* allocation failed */
    HWO_EDEVICE = -4,   /* HIP runtime error */
    HWO_ERANGE = -5,    /* buffer too small / index out of range */
    HWO_EOVERFLOW = -6  /* particle capacity exceeded (counts still valid) */
};

typedef struct hwo_ocean hwo_ocean;

/* Device allocator hooks: alloc(bytes, ctx) returns a device pointer or NULL;
 * free(ptr, ctx) releases it.  NULL hooks select hipMalloc / hipFree. */
typedef void *(*hwo_alloc_fn)(size_t bytes, void *ctx);
typedef void (*hwo_free_fn)(void *ptr, void *ctx);

typedef struct {
    int32_t fft_n;          /* background grid N (power of two, 16..4096) */
    double fft_L;           /* background period (m) */
    double g;               /* gravity (m/s^2) */
    double dt;              /* step (s); heights after step n describe t = n dt */
    uint64_t seed;          /* Philox key for h0 and injection draws */
    int32_t compact;        /* 0: 32-byte particle records, 1: 16-byte records */
    int32_t batched;        /* 0: launches per patch; 1: one launch per stage for
                               all patches, whole frame replayed as a hipGraph */
    void *stream;           /* hipStream_t to run on; NULL: the library creates one */
    hwo_alloc_fn dev_alloc; /* optional device allocator */
    hwo_free_fn dev_free;
    void *alloc_ctx;
    int64_t max_particles;  /* particle capacity; 0 selects an estimate */
    int32_t synth;          /* height synthesis: 0 the separable kernel at each
                               particle's exact position (default); 1 the paper's
                               texel layers (Sec 4.2) -- bilinear deposit per bucket,
                               passes along x and y with the raised cosine at
                               whole-cell offsets, layers summed.  The passes
                               stage (2R + 81) x 64 floats in LDS, R = ceil(r/dx) - 1,
                               so a radius beyond 279 cells is HWO_EINVAL at the
                               first step */
    int32_t normals;        /* 1: also derive unit normals of the blended maps by
                               finite differences every frame (Sec 4.2), read as
                               layers 2-4 of hwo_read_heightmaps; 0: none */
    int32_t bg_fields;      /* 1: the FFT also makes the background slopes dH/dx,
                               dH/dy and the choppy displacement (x, y), read as
                               layers 1-4 of the background; 0: height only */
    int32_t kernel;         /* shape of the crest and trough kernel (Fig 1):
                               0 separable w(dx) w(dy), w(d) = (1 + cos(pi d / r)) / 2
                               for |d| < r; 1 radial W(|d|) with the same profile.
                               The radial kernel needs synth 0 (the texel passes
                               are separable); synth 1 with kernel 1 is HWO_EINVAL. */
    int32_t fft_mfma16;     /* 1: the first stage of every background FFT row
                               (N >= 1024) is a radix-16 DFT on the matrix cores
                               with split bf16 (hi + lo) operands and FP32
                               accumulation; 0 (default): the FP32 radix-8/4/2
                               stages only.  An option for measurement: it is
                               no faster (the passes are bound by HBM) and its
                               error is about ten times larger. */
} hwo_config;

/* Spectrum and bucket parameters (Sec 3.1, Sec 3.3). */
typedef struct {
    double U10, fetch;      /* wind speed at 10 m (m/s), fetch (m) -- Eq 4 */
    double gamma;           /* peak enhancement; <= 0: Eq 4 */
    double spread_s;        /* cos-2s exponent; < 0: Mitsuyasu s(w), Eq 6 */
    double wind_dir;        /* radians from +x */
    int32_t n_buckets;      /* 1..16 log-spaced wavelength buckets */
    double lambda_min, lambda_max; /* bucket wavelength range (m) */
    double eta;             /* particles per injected group (paper N_theta) */
    int32_t max_level;      /* subdivision levels of ring particles, 0..4 */
    double subdiv_frac;     /* split when ring spacing > subdiv_frac * radius */
    int32_t h0_mode;        /* 0 Gaussian h0, 1 unit modulus */
    int32_t bucket_mode;    /* 0: n_buckets log-spaced wavelength buckets over
                               [lambda_min, lambda_max]; 1: equal-energy buckets
                               over [0.5 w_p, 2.5 w_p] (Sec 3.3), lambda range unused */
    int32_t dir_mode;       /* 0: boundary directions by inverse CDF of Dir, equal
                               amplitudes; 1: stratified groups (Sec 3.3) -- the m-th
                               particle of a side-pair stream takes sector m mod N_theta
                               (N_theta = eta, a whole number), amplitude from
                               S(w_i, theta) */
    int32_t flux_mode;      /* 0: each side pair injects the group count of Eq 18;
                               1: obliquity-weighted -- a pair's count is scaled by
                               the mean |cos| of the angle between the wave and the
                               side normal under Dir, and its directions are drawn
                               from Dir |cos|.  Needs dir_mode 0. */
} hwo_spectrum;

typedef struct {
    double anchor_x, anchor_y; /* world position (m) of the patch frame origin */
    int32_t nx, ny;         /* cells; max 4096 each */
    double dx;              /* cell size (m); dx * 2^20 must be an even integer */
    double eta;             /* <= 0: spectrum eta */
    double blend_band;      /* <= 0: min(largest radius, min side / 4) */
    int32_t follow;         /* source id that recentres the window, -1 static */
} hwo_patch;

/* Work partition of the per-bucket splat (the tunable launch parameters of
 * the batched form; hwo_get_plan / hwo_set_plan / hwo_autotune). */
typedef struct {
    int32_t chunk_load;     /* least estimated cost of one splat work item (model units) */
    int32_t items_target;   /* work items per frame the plan aims for beyond one per output tile */
    int32_t splat_grid;     /* persistent splat blocks launched; 0: four per compute unit */
    int32_t splat_kernel;   /* splat schedule: 0 each wavefront splats its own batches of records
                               (four quadrant accumulators per wavefront), 1 each wavefront owns one
                               quadrant of the tile and the block decodes records into LDS, 2 the
                               first for small footprints and then the second for large ones
                               (default); the same heights up to FP32 summation order */
} hwo_plan;

typedef struct {
    double x0, y0;          /* world start (m) */
    double vx, vy;          /* velocity (m/s); zero speed emits nothing */
    double radius, draft;   /* disc radius and draft (m) */
    int32_t ring_n;         /* particles per ring; must divide 128 */
    int32_t patch;          /* patch receiving the particles */
    double heave_amp;       /* vertical motion z(t) = heave_amp sin(2 pi t / heave_period) (m); 0: none */
    double heave_period;    /* (s); > 0 when heave_amp > 0 */
} hwo_source;

/* Create a handle for one ocean.  The configuration carries the inputs the
 * paper's pipeline takes besides the spectrum (Sec 4.1, Fig 3): the FFT
 * background grid and period, gravity, the time step and the seed of the
 * random draws, plus the record form, the launch form and the synthesis and
 * kernel options.  Validates cfg; allocates nothing on the device.  *out
 * receives the handle (owned by the caller until hwo_destroy_ocean).
 * HWO_EINVAL for a NULL argument or an invalid field (grid not a power of two
 * in 16..4096, non-positive period, g or dt, unknown mode). */
int hwo_create_ocean(const hwo_config *cfg, hwo_ocean **out);
/* Release every device allocation and the handle (Sec 4.1 pipeline state);
 * NULL is ignored.  The caller must not use o afterwards. */
void hwo_destroy_ocean(hwo_ocean *o);
/* Message of the last failing call on o (the status codes above, Sec 4.1
 * pipeline); owned by the handle, valid until the next call on it. */
const char *hwo_last_error(const hwo_ocean *o);

/* Spectrum and buckets (Sec 3.1 Eq 1-6; Sec 3.2 kinematics r_i = pi g / w_i^2,
 * c_i = g / w_i; Sec 3.3 buckets, Eq 7 amplitude, Eq 18 rates): builds the
 * bucket, direction and velocity tables, h0(k) and the FFT twiddles (FP64 on
 * the GPU, stored FP32).  Once per handle, before add_patch / add_source
 * (HWO_ESTATE otherwise); HWO_EINVAL for out-of-range parameters. */
int hwo_set_spectrum(hwo_ocean *o, const hwo_spectrum *sp);
/* Add a wave-particle patch, the rectangular region around an interactive
 * object where the particle field replaces the FFT (Sec 3.1 local
 * replacement; boundary injection Sec 3.3, Eq 18).  Max 127 patches; *id
 * receives its index (dense, in call order; it selects the patch's RNG
 * streams).  HWO_EINVAL for a bad size or dx (the larger side times dx
 * at most 1.5e9 position units of 2^-20 m), and, with dir_mode 1, for an
 * effective eta that is not a whole number in 1..10368 (one direction code
 * per particle at most); HWO_ESTATE after the first step.  The first step
 * also fails with HWO_EINVAL when the larger side plus a bucket's survival
 * margin (2 r) reaches 2^31 position units. */
int hwo_add_patch(hwo_ocean *o, const hwo_patch *p, int32_t *id);
/* Add a moving object that disturbs the water (Sec 4.3, object acts on
 * water): a disc emitting rings of particles into patch src->patch, into the
 * bucket whose radius is closest to the disc's.  Horizontal motion emits a
 * ring signed by the heading each time the disc has moved half a radius;
 * vertical motion (heave_amp > 0) emits an isotropic ring each time the
 * previous one has travelled half a radius, carrying the volume the disc
 * displaced meanwhile.  Max 127; *id receives its index.  HWO_EINVAL for a
 * bad patch index, radius, ring size or heave; HWO_ESTATE after the first
 * step. */
int hwo_add_source(hwo_ocean *o, const hwo_source *s, int32_t *id);
/* Per-bucket particle bin edge in cells (n == n_buckets, each 1..4096) of
 * the counting sort that groups particles for the per-bucket splat (Sec 4.2
 * per-bucket layers).  Optional; changes only the bin histogram, never
 * heights or other counts.  HWO_ESTATE after the first step. */
int hwo_set_bins(hwo_ocean *o, const int32_t *bin_cells, int32_t n);

/* Advance nsteps frames of the pipeline (Sec 4.1, Fig 3): FFT background,
 * boundary injection, ring emission, propagation and subdivision, binning,
 * per-bucket splat and blend.  Asynchronous on the library stream.  The
 * first call allocates device memory and fixes the scene.  HWO_EINVAL for
 * nsteps < 0, HWO_ERANGE if the step index would pass 2^31 - 1,
 * HWO_EDEVICE for a HIP failure. */
int hwo_step(hwo_ocean *o, int32_t nsteps);
/* Wait for the frames issued by hwo_step (Sec 4.1 pipeline). */
int hwo_sync(hwo_ocean *o);
/* Frames issued so far: heights describe t = n dt (Sec 4.1); -1 for NULL. */
int64_t hwo_step_index(const hwo_ocean *o);

/* Copy a height map (FP32, row-major [y][x]) into dst (host or device memory
 * per dst_is_device), the outputs of the blend (Sec 3.1 stitching, Sec 4.2
 * composition of FFT and particle heights).  which = -1: background N x N
 * (Sec 4.1), layer 0 the height,
 * 1 dH/dx, 2 dH/dy, 3 and 4 the choppy displacement sum -i (k/|k|) h~
 * e^{ik.x} in x and y (HWO_ESTATE unless hwo_config.bg_fields; these fields
 * omit the Nyquist rows and columns); which = p >= 0: patch p
 * (ny x nx) with layer 0 = blended, 1 = raw wave-particle height, 2, 3, 4 =
 * x, y, z component of the unit normal of the blended map (central
 * differences, one-sided at the patch edges; HWO_ESTATE unless
 * hwo_config.normals).  HWO_ERANGE if dst_elems is too small.  Syncs. */
int hwo_read_heightmaps(hwo_ocean *o, int32_t which, int32_t layer, float *dst,
                        int64_t dst_elems, int32_t dst_is_device);

/* Particle bookkeeping of patch p (Sec 3.3 injection counts, Eq 18; Sec 4.3
 * ring emission), six int64 per bucket: live, injected, emitted,
 * subdivided, died, dropped (capacity overflow, whole ocean).
 * dst_elems >= 6 n_buckets, else HWO_ERANGE.  Returns HWO_EOVERFLOW (with
 * valid counts) if particles were dropped. */
int hwo_read_counts(hwo_ocean *o, int32_t patch, int64_t *dst, int64_t dst_elems);

/* Frequency buckets after set_spectrum (Sec 3.2-3.3): four doubles per bucket,
 * w_i (rad/s), dw_i (rad/s), particle radius r_i = pi g / w_i^2 (m) and phase
 * speed c_i = g / w_i (m/s); bucket 0 holds the shortest waves.  n >= 4
 * n_buckets, else HWO_ERANGE; HWO_ESTATE before set_spectrum. */
int hwo_read_buckets(const hwo_ocean *o, double *dst, int32_t n);
/* Bin grid of (patch, bucket) used to group particles for the per-bucket
 * splat (Sec 4.2): dims = {bin edge cells, nbx, nby}.  HWO_ERANGE for a bad
 * index, HWO_ESTATE before the first step. */
int hwo_tile_dims(hwo_ocean *o, int32_t patch, int32_t bucket, int64_t *dims);
/* Live particles per bin (Sec 4.2 per-bucket grouping), row-major [by][bx],
 * bins anchored at the window origin minus the bucket margin 2 r.
 * HWO_ERANGE if n < nbx nby. */
int hwo_read_tiles(hwo_ocean *o, int32_t patch, int32_t bucket, int64_t *dst, int64_t n);

/* Live particles (Sec 3.2 single particle: direction, frequency bucket,
 * amplitude source) as canonical records of 10 int64:
 * patch, bucket, kind (0 boundary, 1 ring of horizontal motion, 2 ring of
 * vertical motion), level, code (units of
 * 2 pi / 10368), birth step, origin x, origin y (2^-20 m from the patch
 * anchor), source (-1 boundary), ring slot.  *n_out receives the count;
 * fails with HWO_ERANGE if max_recs is too small. */
int hwo_read_particles(hwo_ocean *o, int64_t *dst, int64_t max_recs, int64_t *n_out);

/* Test hook: splat caller-placed canonical records (the crest/trough pair of
 * Fig 1, Sec 3.2) into patch p's raw map at the current step (no binning),
 * result in dst (host, ny x nx).  With synth 1 the records go through the
 * texel layers instead (which it overwrites).  HWO_EINVAL for a record of
 * another patch or an out-of-range field; HWO_ESTATE before the first step. */
int hwo_test_splat(hwo_ocean *o, int32_t patch, const int64_t *recs, int64_t n, float *dst,
                   int64_t dst_elems);

/* Object-receives-water sampling (Sec 4.3): height and unit normal of the
 * current frame at n world points.  xy holds n (x, y) pairs in metres (FP64),
 * out receives n x 4 floats: height, normal x, y, z.  Both in host memory, or
 * both in device memory when on_device != 0.  A point inside the cell-centre
 * hull of a patch (the first such patch) samples its blended map, else the
 * periodic background; bilinear height, slopes from central differences
 * (one-sided at patch edges) interpolated the same way.  HWO_ESTATE before
 * the first step; n at most 2^24.  Syncs. */
int hwo_sample_probes(hwo_ocean *o, const double *xy, int64_t n, float *out, int32_t on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the probe
 * sampling of hwo_sample_probes with host arrays xy (n x 2 doubles, world
 * metres) and out (n x 4 floats: height, unit normal), staged through a
 * static device array of 4 MiB that each GPU holds until the process ends;
 * this call allocates nothing.  n at most 131072 (HWO_ERANGE above),
 * HWO_ESTATE before the first step (it never builds the device state,
 * which allocates), HWO_EDEVICE if the array's address could not be looked
 * up when the spectrum was set.  Every handle on one GPU shares that GPU's
 * array: calls that overlap on one GPU (from several threads or streams)
 * race; consecutive calls do not, since each synchronises the stream before
 * it returns.  The caller owns xy and out. */
int hwo_sample_probes_static(hwo_ocean *o, const double *xy, int64_t n, float *out);

/* Checkpoint and resume of the pipeline state (Sec 4.1, Fig 3: the state
 * one frame hands to the next).  A snapshot is a host-memory image of the
 * state at the current step boundary (step index, counters, bin offsets, live
 * particle records, splat partition feedback) plus a fingerprint of the scene.
 * hwo_snapshot_size gives its size in bytes (HWO_ESTATE before the first
 * step); hwo_snapshot writes it into dst (HWO_ERANGE if dst_bytes is too
 * small); hwo_restore loads an image into a handle built with the same scene,
 * configuration and record form (HWO_EINVAL otherwise), after which stepping
 * continues exactly as from the saved step: integer state bit for bit,
 * heights up to FP32 summation order.  Heights, probes and test splats read
 * between a restore and the next step describe the restored step index's
 * windows; the height maps are those the handle held before restoring.  The
 * caller owns both buffers.  All three synchronise the stream. */
int hwo_snapshot_size(hwo_ocean *o, int64_t *bytes);
int hwo_snapshot(hwo_ocean *o, void *dst, int64_t dst_bytes);
int hwo_restore(hwo_ocean *o, const void *src, int64_t src_bytes);

/* Per-stage timing, benchmark support for the frame-time measurements of
 * Sec 5.2 (Table 2).  enable != 0 brackets every kernel launch with HIP
 * events (graph replay is then disabled); hwo_stage_times returns
 * accumulated milliseconds and launch counts per stage:
 *   0 params  1 fft_a  2 fft_b  3 count  4 scan  5 scatter  6 splat
 *   7 splat_plan  8 splat_reduce  9 bin_plan  10 deposit_x  11 filter_y
 *   12 layer_sum  13 normals (n >= 14).  bin_plan is the one-block scan + tile
 *   estimates + plan that replaces stages 4 and 7 in the batched form of
 *   scenes with at most 16384 bins, 1024 output tiles and 1024 (tile, bucket)
 *   pairs.  Stages 6-8 run with synth 0, stages 10-12 with synth 1. */
int hwo_set_timing(hwo_ocean *o, int32_t enable);
int hwo_stage_times(hwo_ocean *o, double *ms, int64_t *launches, int32_t n);
/* Per-bucket profile of the splat (Sec 4.2: the per-bucket layers of
 * Fig 1's crest/trough pairs), for attributing its time.  With enable = 1
 * the splat runs as a profiling instance of its kernel in which each
 * wavefront reads the shader clock (s_memtime) at the boundaries of its work
 * and adds the ticks since its previous mark to a category; enable 0 returns
 * to the plain instance (a change re-captures the frame graph); the
 * accumulators are cleared by every call.  hwo_read_splat_profile copies the 36 accumulators
 * into dst (n >= 36), as doubles: [0] item set-up, [1] record decode,
 * [2] end-of-chunk wait, [3] epilogue (blend or partial tile), [4 + b]
 * footprints of bucket b, [20 + b] crest and trough points of bucket b
 * visited (b < 16).  Ticks are summed over wavefronts, so only their
 * shares are meaningful; the marks themselves cost a little time.
 * HWO_EINVAL for a bad argument, HWO_ESTATE (read) before the device state
 * exists.  Both synchronise the stream. */
int hwo_set_splat_profile(hwo_ocean *o, int32_t enable);
int hwo_read_splat_profile(hwo_ocean *o, double *dst, int32_t n);
/* Benchmark support (Sec 5.2 frame-time measurements): after at least one
 * step, launch the kernels of one
 * stage reps times back to back between two HIP events on the library stream
 * and store the mean milliseconds per repetition (all launch groups of the
 * stage).  Only stages whose kernels are idempotent for a finished frame are
 * accepted: 1 fft_a, 2 fft_b, 6 splat, 7 splat_plan, 8 splat_reduce (synth 0),
 * 10 deposit_x, 11 filter_y, 12 layer_sum (synth 1), 13 normals (when
 * enabled); any other stage gives
 * HWO_EINVAL, a call before the first step HWO_ESTATE.  Outputs are rewritten
 * with the same values (up to FP32 summation order). */
int hwo_time_stage(hwo_ocean *o, int32_t stage, int32_t reps, double *ms_per_rep);
/* Tuning of the per-bucket splat (Sec 4.2: the per-bucket layers of Fig 1's
 * pairs, here one launch over all tiles of all patches).  hwo_get_plan
 * reports the current work partition; hwo_set_plan replaces it (chunk_load
 * 64..2^24, items_target 0..8192, splat_grid 0..65535, splat_kernel 0..2;
 * HWO_EINVAL otherwise), effective from the next step (the frame graph is
 * captured again).  hwo_autotune searches the partition on the current
 * frame: after at least one step it re-runs the plan, splat and reduce
 * stages (which rewrite the same heights, up to FP32 summation order) reps
 * times per candidate, for each splat schedule coordinate by coordinate over
 * chunk_load, items_target and splat_grid, keeps the fastest, sets it and
 * reports it with its time and that of the partition it started from
 * (milliseconds per plan + splat + reduce).  Integer state is never touched.  HWO_ESTATE before the first
 * step, HWO_EINVAL with texel layers (synth 1) or reps < 1.  Synchronise. */
int hwo_get_plan(hwo_ocean *o, hwo_plan *out);
int hwo_set_plan(hwo_ocean *o, const hwo_plan *plan);
int hwo_autotune(hwo_ocean *o, int32_t reps, hwo_plan *best, double *best_ms, double *start_ms);
/* Bytes of particle storage per record for the active form (16 or 32): the
 * particle attributes of Sec 3.2 (position, direction, bucket, amplitude
 * source, birth); -1 for NULL. */
int32_t hwo_record_bytes(const hwo_ocean *o);

#ifdef __cplusplus
}
#endif
#endif

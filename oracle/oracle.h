/* oracle.h -- FP64 single-threaded CPU oracle of the hybrid-ocean hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * Every value is computed in double precision, in plain loops, one thread.
 * Integer decisions (counts, codes, fixed-point positions, bins) are made
 * exactly as the method's fixed-point reading defines them.
 *
 * Canonical particle record (10 x int64), shared as a *format* with the GPU
 * library's test hooks:
 *   [0] patch  [1] bucket  [2] kind (0 boundary, 1 source)  [3] level
 *   [4] code   [5] birth   [6] origin_x  [7] origin_y  (2^-20 m, anchor-relative)
 *   [8] source (-1 for boundary)  [9] ring slot (0 for boundary)
 */
#ifndef HWO_ORACLE_H
#define HWO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_ocean orc_ocean;

orc_ocean *orc_create(int32_t fft_n, double fft_L, double g, double dt, uint64_t seed);
void orc_destroy(orc_ocean *o);
const char *orc_error(const orc_ocean *o);

int orc_set_spectrum(orc_ocean *o, double U10, double fetch, double gamma, double spread_s,
                     double wind_dir, int32_t n_buckets, double lambda_min, double lambda_max,
                     double eta, int32_t max_level, double subdiv_frac, int32_t h0_mode,
                     int32_t bucket_mode, int32_t dir_mode, int32_t flux_mode);
int orc_add_patch(orc_ocean *o, double ax, double ay, int32_t nx, int32_t ny, double dx,
                  double eta, double band, int32_t follow);
int orc_add_source(orc_ocean *o, double x0, double y0, double vx, double vy, double radius,
                   double draft, int32_t ring_n, int32_t patch, double heave_a, double heave_T);
int orc_set_bins(orc_ocean *o, const int32_t *bin_cells);
/* Height synthesis: 0 the exact-position splat, 1 texel layers per bucket
 * (bilinear deposit) smoothed by separable x and y passes (Sec 4.2).
 * kernel: 0 the separable product w(dx) w(dy), 1 the radial w(|d|) with the
 * same raised-cosine profile (Fig 1); the radial kernel needs mode 0. */
int orc_set_synthesis(orc_ocean *o, int32_t mode, int32_t kernel);
/* Unit normals of patch p from height map h (ny x nx) by finite differences
 * (Sec 4.2); out holds three ny x nx planes: x, y and z components. */
int orc_normals(orc_ocean *o, int32_t p, const double *h, double *out);
/* Background field at time t (N x N, row-major [y][x]): 0 height, 1 dH/dx,
 * 2 dH/dy, 3 and 4 the choppy displacement sum -i (k/|k|) h~ e^{ik.x}
 * (x and y); fields 1-4 exclude the Nyquist rows/columns. */
int orc_background_field(orc_ocean *o, int32_t field, double t, double *H);
/* Height and unit normal at n world points (xy: x, y pairs) from background H
 * (N x N) and the blended maps B of all patches back to back (Sec 4.3
 * object-receives-water sampling); out: 4 values per probe (h, nx, ny, nz). */
int orc_sample_probes(orc_ocean *o, const double *H, const double *B, const double *xy, int64_t n, double *out);
int orc_step(orc_ocean *o, int32_t nsteps);
int64_t orc_step_index(const orc_ocean *o);

/* outputs at t_n = n*dt */
int orc_background(orc_ocean *o, double *H);
int orc_background_at(orc_ocean *o, double t, double *H);
int orc_patch_maps(orc_ocean *o, int32_t patch, const double *H, double *raw, double *blended);
int orc_counts(const orc_ocean *o, int32_t patch, int64_t *dst);
int orc_tile_dims(const orc_ocean *o, int32_t patch, int32_t bucket, int64_t *dims);
int orc_tiles(const orc_ocean *o, int32_t patch, int32_t bucket, int64_t *dst, int64_t n);
int64_t orc_num_particles(const orc_ocean *o);
int64_t orc_particles(const orc_ocean *o, int64_t *dst, int64_t n);
int orc_window(const orc_ocean *o, int32_t patch, int64_t *w);

/* tables and pins */
double orc_jonswap(const orc_ocean *o, double w);
double orc_dir(const orc_ocean *o, double w, double theta);
double orc_spread(const orc_ocean *o, double w);
int orc_spectrum_consts(const orc_ocean *o, double *out);
int orc_bucket(const orc_ocean *o, int32_t i, double *out);
int orc_patch_bucket(const orc_ocean *o, int32_t p, int32_t i, double *out);
/* Integer direction weights, inclusive CDF and bin codes of bucket i for side
 * pair `pair` (0: the sides normal to x, 1: normal to y), 64 entries each. */
int orc_dir_table(const orc_ocean *o, int32_t i, int32_t pair, int64_t *q, int64_t *cdf, int64_t *codes);
int orc_velocity(const orc_ocean *o, int32_t i, int32_t code, int64_t *v);
int orc_source_info(const orc_ocean *o, int32_t s, double *out);
int64_t orc_inject_count(const orc_ocean *o, int32_t p, int32_t i, int32_t pair, int64_t n);
void orc_philox4x64(const uint64_t *ctr, const uint64_t *key, uint64_t *out);
void orc_fft_inverse(double *re, double *im, int32_t n);
void orc_fft2_inverse(double *re, double *im, int32_t n);
void orc_dft2_inverse(const double *re, const double *im, double *ore, double *oim, int32_t n);
int orc_h0(const orc_ocean *o, double *re, double *im);
int orc_set_h0(orc_ocean *o, const double *re, const double *im);
int orc_splat(orc_ocean *o, int32_t patch, const int64_t *recs, int64_t n, double *raw);
/* Step index n (and its windows) for an oracle without particles: evaluation
 * of caller-supplied particles and maps at that step. */
int orc_seek(orc_ocean *o, int64_t n);
/* particle state after step n from caller records (orc_particles layout); test infrastructure */
int orc_load(orc_ocean *o, int64_t n, const int64_t *recs, int64_t count);
/* Blend of a caller-supplied raw patch map with background H at the current step. */
int orc_blend(orc_ocean *o, int32_t patch, const double *H, const double *raw, double *blended);

#ifdef __cplusplus
}
#endif
#endif

/* oracle.c -- FP64 single-threaded CPU oracle of the hybrid-ocean hot path
 * (Xue et al., "Real-Time Interactive Hybrid Ocean: Spectrum-Consistent Wave
 * Particle-FFT Coupling", arXiv 2511.02852).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this code; the GPU library
 * never does.  It shares no source, header, table or helper with the GPU
 * library: every table here is rebuilt from the paper's formulas.
 *
 * What it computes, per step n (t_n = n*dt):
 *   - FFT background: Sec 3.1 (Eq 1-6) spectrum, evolved as a standard
 *     Tessendorf-style spectral field under deep-water dispersion w^2 = g k
 *     (Sec 4.1 "FFT updates"), inverse-transformed with a radix-2 FFT.
 *   - Wave-particle patches: frequency buckets (log-spaced, or the
 *     equal-energy partition of [0.5 w_p, 2.5 w_p] of Sec 3.3) with
 *     w_i, r_i = pi g / w_i^2, c_i = g / w_i (Sec 3.2 kinematics), amplitude
 *     A = sqrt(2 S dw dtheta) (Eq 7, importance-sampled or per stratified
 *     direction), boundary injection rate N_i = 4 L dt w_i^3 / (pi^3 g) per
 *     pair of opposite sides (Eq 18, optionally scaled by the mean obliquity),
 *     directions drawn from the directional spectrum (Sec 4.2) or stratified
 *     over N_theta sectors (Sec 3.3),
 *     fixed-point analytic propagation at c_i, ring emission from moving
 *     sources into the closest-radius bucket (Sec 4.3), 3-way subdivision,
 *     and a raised-cosine crest/trough pair splat (Fig 1, Sec 4.2), separable
 *     w(dx) w(dy) or radial w(|d|).
 *   - Blend of patch and background with a smooth distance weight (Sec 3.1,
 *     Sec 4.2).
 * Where the paper is silent the readings are the ones listed in the design
 * notes (fixed-point units, direction codes, Philox streams, blend profile).
 *
 * Parity pins (tests/test_oracle_*.py): closed-form JONSWAP integral, Dir
 * normalisation and special case, naive DFT / numpy FFT / Parseval, single
 * mode phase speed, numpy Philox4x64, energy identity of the injection rate,
 * pair-lattice cosine sum, crest volume, subdivision conservation, blend
 * limits, equal-energy bucket integrals, stratified sector balance and the
 * direction amplitude factor's normalisation, the steady-state spectral
 * density of obliquity-weighted injection, the bin histogram against a
 * histogram of the crest positions, window recentring within half a cell of
 * the source track and ring origins on the source position.  Full-scene
 * particle bookkeeping beyond these is parity unpinned
 * except through the identities tested there.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXB 16
#define NDIR 64                 /* direction bins of the injection CDF */
#define LMAX_CAP 4              /* subdivision levels */
#define NCODE 10368             /* direction codes per turn: 2 * NDIR * 3^4 */
#define AGE_MAX 65535
#define UNIT 1048576.0          /* fixed-point position units per metre (2^20) */
#define TWO32 4294967296.0
#define TWO30 1073741824.0
#define STREAM_INJECT 1u
#define STREAM_H0 2u

enum { C_LIVE = 0, C_INJ, C_EMIT, C_SUB, C_DIED, C_NUM };

typedef struct {
    int64_t ox, oy, birth;
    int32_t code, level, kind, bucket, patch, src, slot;
} prt_t;

typedef struct {
    double ax, ay, dx, eta, band;
    int32_t nx, ny, follow;
    int64_t dxu, wx, wy;
    double A[MAXB];
    uint64_t Rx[MAXB], Ry[MAXB];
    int64_t cnt[MAXB][C_NUM];
    int64_t binw[MAXB], nbx[MAXB], nby[MAXB];
    int64_t *hist[MAXB];
} patch_t;

typedef struct {
    double x0, y0, vx, vy, R, draft, speed, heading, B, sum_abs;
    int32_t ne, patch, bucket, a0;
    int64_t E, T[LMAX_CAP];
    /* vertical (heave) motion z(t) = heave_a sin(2 pi t / heave_T); rings
     * every Eh steps carry the volume the disc displaced since the last one */
    double heave_a, heave_T, Bh;
    int64_t Eh;
    double *m;
    int64_t *Ox, *Oy;
} src_t;

struct orc_ocean {
    int32_t N;
    double L, g, dt;
    uint64_t seed;
    int have_spec, stepped, bins_set;
    int32_t synth;               /* 0 exact-position splat, 1 texel layers + separable passes */
    int32_t kernel;              /* 0 separable w(dx) w(dy), 1 radial w(|d|) (synth 0 only) */
    double U10, fetch, gamma, s_const, wind_dir, alpha, wp, eta, subdiv_frac;
    int32_t nb, lmax, h0_mode, wind_code, dir_mode, flux_mode;
    double lam_min, lam_max;
    double w[MAXB], dw[MAXB], r[MAXB], c[MAXB], lam[MAXB];
    int64_t margin[MAXB];
    /* direction weights per bucket and side pair (0: sides normal to x) */
    int64_t q[MAXB][2][NDIR], cdf[MAXB][2][NDIR], Q[MAXB][2];
    double kappa[MAXB][2];   /* flux factor of each side pair; 1 when flux_mode is 0 */
    int32_t codes[NDIR];
    int64_t *V;                 /* [nb][NCODE][2] */
    double *h0re, *h0im;        /* [N][N], row = y index */
    int np, ns;
    patch_t *pt;
    src_t *sr;
    int32_t bin_cells[MAXB];
    int64_t n;
    prt_t *P;
    int64_t nP, capP;
    char err[256];
};

static int fail(orc_ocean *o, const char *msg) {
    snprintf(o->err, sizeof o->err, "%s", msg);
    return -1;
}

/* floor division for b > 0 */
static int64_t fdiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static int64_t pmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

static int64_t ipow3(int k) {
    int64_t v = 1;
    for (int i = 0; i < k; ++i) v *= 3;
    return v;
}

/* ---------------------------------------------------------------- Philox */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 64x64->128 multiplies with a Weyl-sequence key schedule. */
static uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

void orc_philox4x64(const uint64_t *ctr, const uint64_t *key, uint64_t *out) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t lo0 = M0 * c0, hi0 = mulhi64(M0, c0);
        uint64_t lo1 = M1 * c2, hi1 = mulhi64(M1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double unit_open(uint64_t u) {
    return (double)(u >> 11) * (1.0 / 9007199254740992.0) + (1.0 / 18014398509481984.0);
}

/* ---------------------------------------------------------------- spectrum */
/* Eq 2-3: JONSWAP.  sigma = 0.07 below the peak, 0.09 above (standard values;
 * the paper names sigma without a value). */
double orc_jonswap(const orc_ocean *o, double w) {
    if (w <= 0.0) return 0.0;
    double sigma = (w <= o->wp) ? 0.07 : 0.09;
    double d = w - o->wp;
    double r = exp(-(d * d) / (2.0 * sigma * sigma * o->wp * o->wp));
    double x = o->wp / w;
    double x4 = x * x * x * x;
    return o->alpha * o->g * o->g * pow(w, -5.0) * exp(-1.25 * x4) * pow(o->gamma, r);
}

/* Eq 6 (Mitsuyasu) when no constant exponent is given. */
double orc_spread(const orc_ocean *o, double w) {
    if (o->s_const >= 0.0) return o->s_const;
    double mu = (w <= o->wp) ? 5.0 : -2.5;
    return 16.0 * pow(w / o->wp, mu);
}

/* Eq 5: normalised cos-2s spreading, theta relative to the wind in [-pi, pi]. */
static double dir_s(double s, double theta) {
    double norm = tgamma(s + 1.0) / (2.0 * sqrt(M_PI) * tgamma(s + 0.5));
    double cth = cos(0.5 * theta);
    if (cth < 0.0) cth = -cth;
    return norm * pow(cth, 2.0 * s);
}

double orc_dir(const orc_ocean *o, double w, double theta) {
    return dir_s(orc_spread(o, w), theta);
}

int orc_spectrum_consts(const orc_ocean *o, double *out) {
    if (!o->have_spec) return -1;
    out[0] = o->alpha;
    out[1] = o->wp;
    out[2] = o->gamma;
    out[3] = (double)o->wind_code;
    return 0;
}

/* ---------------------------------------------------------------- create */
orc_ocean *orc_create(int32_t fft_n, double fft_L, double g, double dt, uint64_t seed) {
    if (fft_n < 2 || (fft_n & (fft_n - 1)) != 0 || !(fft_L > 0) || !(g > 0) || !(dt > 0))
        return NULL;
    orc_ocean *o = (orc_ocean *)calloc(1, sizeof *o);
    o->N = fft_n;
    o->L = fft_L;
    o->g = g;
    o->dt = dt;
    o->seed = seed;
    for (int i = 0; i < MAXB; ++i) o->bin_cells[i] = 16;
    return o;
}

static void free_patch(patch_t *p) {
    for (int i = 0; i < MAXB; ++i) free(p->hist[i]);
}

void orc_destroy(orc_ocean *o) {
    if (!o) return;
    free(o->V);
    free(o->h0re);
    free(o->h0im);
    for (int p = 0; p < o->np; ++p) free_patch(&o->pt[p]);
    for (int s = 0; s < o->ns; ++s) {
        free(o->sr[s].m);
        free(o->sr[s].Ox);
        free(o->sr[s].Oy);
    }
    free(o->pt);
    free(o->sr);
    free(o->P);
    free(o);
}

const char *orc_error(const orc_ocean *o) { return o ? o->err : "null ocean"; }

static void gen_h0(orc_ocean *o);

/* Equal-energy partition of the sampling band [0.5 w_p, 2.5 w_p] into n
 * buckets (Sec 3.3): ascending edges e[0..n] with equal integrals of S_J
 * between neighbours.  The cumulative integral is composite Simpson over
 * 65536 panels; an edge is placed by linear interpolation of the cumulative
 * integral inside the panel that contains its target. */
static void equal_energy_edges(const orc_ocean *o, int n, double *e) {
    const int K = 65536;
    const double a = 0.5 * o->wp, b = 2.5 * o->wp, h = (b - a) / (double)K;
    double *C = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    C[0] = 0.0;
    for (int k = 0; k < K; ++k) {
        const double x = a + (double)k * h;
        C[k + 1] = C[k] + h / 6.0 * (orc_jonswap(o, x) + 4.0 * orc_jonswap(o, x + 0.5 * h) + orc_jonswap(o, x + h));
    }
    e[0] = a;
    e[n] = b;
    int k = 0;
    for (int i = 1; i < n; ++i) {
        const double tau = C[K] * (double)i / (double)n;
        while (k < K - 1 && C[k + 1] <= tau) ++k;
        e[i] = a + (double)k * h + h * ((tau - C[k]) / (C[k + 1] - C[k]));
    }
    free(C);
}

int orc_set_spectrum(orc_ocean *o, double U10, double fetch, double gamma, double spread_s,
                     double wind_dir, int32_t n_buckets, double lambda_min, double lambda_max,
                     double eta, int32_t max_level, double subdiv_frac, int32_t h0_mode,
                     int32_t bucket_mode, int32_t dir_mode, int32_t flux_mode) {
    if (o->have_spec) return fail(o, "spectrum already set");
    if (!(U10 > 0) || !(fetch > 0)) return fail(o, "U10 and fetch must be positive");
    if (n_buckets < 1 || n_buckets > MAXB) return fail(o, "n_buckets out of range");
    if (bucket_mode != 0 && bucket_mode != 1) return fail(o, "bucket_mode must be 0 or 1");
    if (dir_mode != 0 && dir_mode != 1) return fail(o, "dir_mode must be 0 or 1");
    if (flux_mode != 0 && flux_mode != 1) return fail(o, "flux_mode must be 0 or 1");
    if (flux_mode == 1 && dir_mode != 0) return fail(o, "obliquity-weighted injection needs dir_mode 0");
    if (bucket_mode == 0 && (!(lambda_min > 0) || !(lambda_max > lambda_min))) return fail(o, "bad lambda range");
    if (!(eta > 0)) return fail(o, "eta must be positive");
    if (max_level < 0 || max_level > LMAX_CAP) return fail(o, "max_level out of range");
    if (!(subdiv_frac > 0)) return fail(o, "subdiv_frac must be positive");
    double g = o->g;
    o->U10 = U10;
    o->fetch = fetch;
    o->s_const = spread_s;
    o->wind_dir = wind_dir;
    o->eta = eta;
    o->lmax = max_level;
    o->subdiv_frac = subdiv_frac;
    o->h0_mode = h0_mode;
    o->dir_mode = dir_mode;
    o->flux_mode = flux_mode;
    o->nb = n_buckets;
    o->lam_min = lambda_min;
    o->lam_max = lambda_max;
    /* Eq 4 */
    o->alpha = 0.076 * pow(U10 * U10 / (fetch * g), 0.22);
    o->wp = 22.0 * pow(g * g / (U10 * fetch), 1.0 / 3.0);
    o->gamma = (gamma > 0.0) ? gamma : 7.0 * pow(g * fetch / (U10 * U10), -0.142);

    /* Buckets: edge frequencies in descending order (bucket 0 holds the
     * shortest waves), either from log-spaced wavelength edges or from the
     * equal-energy partition of [0.5 w_p, 2.5 w_p]; w_i the geometric mean of
     * the edge frequencies, dw_i the edge difference; Sec 3.2 kinematics. */
    double we[MAXB + 1];
    if (bucket_mode == 0) {
        for (int j = 0; j <= n_buckets; ++j) {
            double le = lambda_min * pow(lambda_max / lambda_min, (double)j / (double)n_buckets);
            we[j] = sqrt(2.0 * M_PI * g / le);
        }
    } else {
        double e[MAXB + 1];
        equal_energy_edges(o, n_buckets, e);
        for (int j = 0; j <= n_buckets; ++j) we[j] = e[n_buckets - j];
    }
    for (int i = 0; i < n_buckets; ++i) {
        double w = sqrt(we[i] * we[i + 1]);
        o->w[i] = w;
        o->dw[i] = we[i] - we[i + 1];
        o->r[i] = M_PI * g / (w * w);
        o->c[i] = g / w;
        o->lam[i] = 2.0 * M_PI * g / (w * w);
        o->margin[i] = (int64_t)ceil(2.0 * o->r[i] * UNIT);
        if (o->c[i] * o->dt >= 0.5) return fail(o, "bucket speed too high for the fixed-point step");
    }

    /* Direction codes: 2*pi/NCODE per unit; bin b centre is wind + theta_b. */
    o->wind_code = (int32_t)pmod(llround(wind_dir * (double)NCODE / (2.0 * M_PI)), NCODE);
    for (int b = 0; b < NDIR; ++b)
        o->codes[b] = (int32_t)pmod((int64_t)o->wind_code + NCODE / 2 +
                                    (int64_t)(2 * b + 1) * (NCODE / (2 * NDIR)), NCODE);

    /* Integer inverse-CDF weights of Dir per bucket (Sec 4.2: directions are
     * sampled from the same directional spectrum), one table per side pair.
     * With obliquity weighting a wave heading phi crosses the sides normal
     * to x at the rate c |cos phi| (|sin phi| for y), so the pair's directions
     * follow Dir |cos phi| and its group count (Eq 18) is scaled by the mean
     * of |cos phi| under Dir, kappa. */
    double dth = 2.0 * M_PI / (double)NDIR;
    for (int i = 0; i < n_buckets; ++i) {
        double s = orc_spread(o, o->w[i]);
        for (int pair = 0; pair < 2; ++pair) {
            int64_t acc = 0;
            double num = 0.0, den = 0.0;
            for (int b = 0; b < NDIR; ++b) {
                double th = -M_PI + ((double)b + 0.5) * dth;
                double d = dir_s(s, th);
                double phi = 2.0 * M_PI * (double)o->codes[b] / (double)NCODE;
                double ob = fabs(pair == 0 ? cos(phi) : sin(phi));
                num += d * ob;
                den += d;
                int64_t qb = llround((flux_mode ? d * ob : d) * dth * TWO30);
                o->q[i][pair][b] = qb;
                acc += qb;
                o->cdf[i][pair][b] = acc;
            }
            o->Q[i][pair] = acc;
            o->kappa[i][pair] = flux_mode ? num / den : 1.0;
            if (acc <= 0) return fail(o, "empty direction distribution");
        }
    }

    /* Fixed-point velocity per step, 2^-32 m units. */
    o->V = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)n_buckets * NCODE);
    for (int i = 0; i < n_buckets; ++i) {
        double cdt = o->c[i] * o->dt;
        for (int code = 0; code < NCODE; ++code) {
            double ang = 2.0 * M_PI * (double)code / (double)NCODE;
            o->V[((size_t)i * NCODE + code) * 2 + 0] = llround(cdt * cos(ang) * TWO32);
            o->V[((size_t)i * NCODE + code) * 2 + 1] = llround(cdt * sin(ang) * TWO32);
        }
    }
    o->have_spec = 1;
    gen_h0(o);
    return 0;
}

int orc_bucket(const orc_ocean *o, int32_t i, double *out) {
    if (!o->have_spec || i < 0 || i >= o->nb) return -1;
    out[0] = o->w[i];
    out[1] = o->dw[i];
    out[2] = o->r[i];
    out[3] = o->c[i];
    out[4] = o->lam[i];
    out[5] = (double)o->margin[i];
    return 0;
}

int orc_dir_table(const orc_ocean *o, int32_t i, int32_t pair, int64_t *q, int64_t *cdf, int64_t *codes) {
    if (!o->have_spec || i < 0 || i >= o->nb || pair < 0 || pair > 1) return -1;
    for (int b = 0; b < NDIR; ++b) {
        q[b] = o->q[i][pair][b];
        cdf[b] = o->cdf[i][pair][b];
        codes[b] = o->codes[b];
    }
    return 0;
}

int orc_velocity(const orc_ocean *o, int32_t i, int32_t code, int64_t *v) {
    if (!o->have_spec || i < 0 || i >= o->nb || code < 0 || code >= NCODE) return -1;
    v[0] = o->V[((size_t)i * NCODE + code) * 2 + 0];
    v[1] = o->V[((size_t)i * NCODE + code) * 2 + 1];
    return 0;
}

/* ---------------------------------------------------------------- patches */
int orc_add_patch(orc_ocean *o, double ax, double ay, int32_t nx, int32_t ny, double dx,
                  double eta, double band, int32_t follow) {
    if (!o->have_spec) return fail(o, "set_spectrum first");
    if (o->stepped) return fail(o, "scene is fixed after the first step");
    if (nx < 1 || ny < 1 || !(dx > 0)) return fail(o, "bad patch size");
    double dxu = dx * UNIT;
    if (dxu != floor(dxu) || ((int64_t)dxu) % 2 != 0) return fail(o, "dx must be an even multiple of 2^-20 m");
    o->pt = (patch_t *)realloc(o->pt, sizeof(patch_t) * (size_t)(o->np + 1));
    patch_t *p = &o->pt[o->np];
    memset(p, 0, sizeof *p);
    p->ax = ax;
    p->ay = ay;
    p->nx = nx;
    p->ny = ny;
    p->dx = dx;
    p->dxu = (int64_t)dxu;
    p->eta = (eta > 0.0) ? eta : o->eta;
    if (o->dir_mode == 1 && (p->eta != floor(p->eta) || p->eta > (double)NCODE))
        return fail(o, "stratified directions need a whole number of particles per group");
    double rmax = o->r[o->nb - 1];
    double lmin = (double)(nx < ny ? nx : ny) * dx / 4.0;
    p->band = (band > 0.0) ? band : (rmax < lmin ? rmax : lmin);
    p->follow = follow;
    double Lx = (double)nx * dx, Ly = (double)ny * dx;
    for (int i = 0; i < o->nb; ++i) {
        double w = o->w[i];
        /* Eq 7, importance-sampled: A^2 = 2 S_J(w_i) dw_i / eta */
        p->A[i] = sqrt(2.0 * orc_jonswap(o, w) * o->dw[i] / p->eta);
        /* Eq 18: groups per step for the pair of sides of length L */
        double gx = 4.0 * Ly * o->dt * w * w * w / (M_PI * M_PI * M_PI * o->g);
        double gy = 4.0 * Lx * o->dt * w * w * w / (M_PI * M_PI * M_PI * o->g);
        p->Rx[i] = (uint64_t)llround(p->eta * gx * o->kappa[i][0] * TWO32);
        p->Ry[i] = (uint64_t)llround(p->eta * gy * o->kappa[i][1] * TWO32);
    }
    o->np += 1;
    return 0;
}

int orc_patch_bucket(const orc_ocean *o, int32_t p, int32_t i, double *out) {
    if (p < 0 || p >= o->np || i < 0 || i >= o->nb) return -1;
    out[0] = o->pt[p].A[i];
    out[1] = (double)o->pt[p].Rx[i];
    out[2] = (double)o->pt[p].Ry[i];
    out[3] = o->pt[p].band;
    out[4] = o->pt[p].eta;
    return 0;
}

/* ---------------------------------------------------------------- sources */
/* Sec 4.3: a moving body emits particles into the bucket with the closest
 * radius; the crest volume of one emission equals the volume swept by the
 * disc since the previous emission (ring model of the design notes). */
int orc_add_source(orc_ocean *o, double x0, double y0, double vx, double vy, double radius,
                   double draft, int32_t ring_n, int32_t patch, double heave_a, double heave_T) {
    if (!o->have_spec) return fail(o, "set_spectrum first");
    if (o->stepped) return fail(o, "scene is fixed after the first step");
    if (patch < 0 || patch >= o->np) return fail(o, "source patch out of range");
    if (!(radius > 0) || !(draft >= 0)) return fail(o, "bad source radius/draft");
    if (!(heave_a >= 0) || (heave_a > 0 && !(heave_T > 0))) return fail(o, "bad heave amplitude/period");
    if (ring_n < 1 || ring_n > 128 || (NCODE / 81) % ring_n != 0) return fail(o, "ring_n must divide 128");
    o->sr = (src_t *)realloc(o->sr, sizeof(src_t) * (size_t)(o->ns + 1));
    src_t *s = &o->sr[o->ns];
    memset(s, 0, sizeof *s);
    s->x0 = x0;
    s->y0 = y0;
    s->vx = vx;
    s->vy = vy;
    s->R = radius;
    s->draft = draft;
    s->ne = ring_n;
    s->patch = patch;
    s->a0 = NCODE / ring_n;
    s->speed = sqrt(vx * vx + vy * vy);
    s->heading = atan2(vy, vx);
    int best = 0;
    for (int i = 1; i < o->nb; ++i)
        if (fabs(o->r[i] - radius) < fabs(o->r[best] - radius)) best = i;
    s->bucket = best;
    double rb = o->r[best], cb = o->c[best];
    s->m = (double *)malloc(sizeof(double) * (size_t)ring_n);
    s->Ox = (int64_t *)malloc(sizeof(int64_t) * (size_t)ring_n);
    s->Oy = (int64_t *)malloc(sizeof(int64_t) * (size_t)ring_n);
    s->sum_abs = 0.0;
    for (int j = 0; j < ring_n; ++j) {
        double phi = 2.0 * M_PI * (double)j / (double)ring_n;
        s->m[j] = cos(phi - s->heading);
        s->sum_abs += fabs(s->m[j]);
        s->Ox[j] = llround(radius * cos(phi) * UNIT);
        s->Oy[j] = llround(radius * sin(phi) * UNIT);
    }
    if (s->speed > 0.0) {
        double e = floor(0.5 * rb / (s->speed * o->dt));
        s->E = e < 1.0 ? 1 : (int64_t)e;
        s->B = 2.0 * radius * s->speed * (double)s->E * o->dt * draft / (rb * rb * s->sum_abs);
    } else {
        s->E = 0;
        s->B = 0.0;
    }
    for (int L = 0; L < LMAX_CAP; ++L) {
        double alpha = 2.0 * M_PI / ((double)ring_n * (double)ipow3(L));
        double x = (o->subdiv_frac * rb / alpha - radius) / (cb * o->dt);
        int64_t T = (int64_t)floor(x) + 1;
        s->T[L] = T < 0 ? 0 : T;
    }
    /* Vertical motion (Sec 4.3: vertical motions trigger ring ripples).  A
     * ring leaves every Eh steps, the time the previous one needs to travel
     * half a radius at the bucket's speed; its n_e crests share the volume
     * pi R^2 dz the disc pushed out since the previous ring (dz = drop of
     * the disc; a rising disc gives troughs first), each crest of volume
     * A r_b^2 with the separable raised cosine: A = pi R^2 dz / (n_e r_b^2). */
    s->heave_a = heave_a;
    s->heave_T = heave_T;
    if (heave_a > 0) {
        double e = floor(0.5 * rb / (cb * o->dt));
        s->Eh = e < 1.0 ? 1 : (int64_t)e;
        s->Bh = M_PI * radius * radius * heave_a / ((double)ring_n * rb * rb);
    }
    o->ns += 1;
    return 0;
}

/* Disc elevation of source s at step n over its heave amplitude:
 * sin(2 pi n dt / heave_T). */
static double heave_z(const orc_ocean *o, const src_t *s, int64_t n) {
    return sin(2.0 * M_PI * ((double)n * o->dt) / s->heave_T);
}

int orc_source_info(const orc_ocean *o, int32_t si, double *out) {
    if (si < 0 || si >= o->ns) return -1;
    const src_t *s = &o->sr[si];
    out[0] = s->bucket;
    out[1] = (double)s->E;
    out[2] = s->B;
    out[3] = s->heading;
    out[4] = s->sum_abs;
    for (int L = 0; L < LMAX_CAP; ++L) out[5 + L] = (double)s->T[L];
    out[9] = s->a0;
    out[10] = (double)s->Eh;
    out[11] = s->Bh;
    return 0;
}

int orc_set_bins(orc_ocean *o, const int32_t *bin_cells) {
    if (!o->have_spec) return fail(o, "set_spectrum first");
    if (o->stepped) return fail(o, "bins are fixed after the first step");
    for (int i = 0; i < o->nb; ++i) {
        if (bin_cells[i] < 1) return fail(o, "bin size must be positive");
        o->bin_cells[i] = bin_cells[i];
    }
    return 0;
}

/* ---------------------------------------------------------------- stepping */
static void source_pos(const orc_ocean *o, const src_t *s, int64_t n, double *xs, double *ys) {
    double t = (double)n * o->dt;
    *xs = s->x0 + s->vx * t;
    *ys = s->y0 + s->vy * t;
}

static void update_windows(orc_ocean *o, int64_t n) {
    for (int p = 0; p < o->np; ++p) {
        patch_t *pt = &o->pt[p];
        if (pt->follow < 0) {
            pt->wx = 0;
            pt->wy = 0;
        } else {
            double xs, ys;
            source_pos(o, &o->sr[pt->follow], n, &xs, &ys);
            pt->wx = llround((xs - pt->ax) / pt->dx) - pt->nx / 2;
            pt->wy = llround((ys - pt->ay) / pt->dx) - pt->ny / 2;
        }
    }
}

static void position(const orc_ocean *o, const prt_t *q, int64_t n, int64_t *px, int64_t *py) {
    int64_t age = n - q->birth;
    const int64_t *v = &o->V[((size_t)q->bucket * NCODE + q->code) * 2];
    *px = q->ox + fdiv(age * v[0], 4096);
    *py = q->oy + fdiv(age * v[1], 4096);
}

static int alive(const orc_ocean *o, const prt_t *q, int64_t n) {
    if (n - q->birth > AGE_MAX) return 0;
    int64_t px, py;
    position(o, q, n, &px, &py);
    const patch_t *pt = &o->pt[q->patch];
    int64_t m = o->margin[q->bucket];
    int64_t lox = pt->wx * pt->dxu - m, hix = (pt->wx + pt->nx) * pt->dxu + m;
    int64_t loy = pt->wy * pt->dxu - m, hiy = (pt->wy + pt->ny) * pt->dxu + m;
    return px >= lox && px <= hix && py >= loy && py <= hiy;
}

static void push(orc_ocean *o, prt_t **buf, int64_t *nb, int64_t *cap, const prt_t *q) {
    (void)o;
    if (*nb == *cap) {
        *cap = *cap ? *cap * 2 : 1024;
        *buf = (prt_t *)realloc(*buf, sizeof(prt_t) * (size_t)*cap);
    }
    (*buf)[(*nb)++] = *q;
}

/* floor(n * R / 2^32) for a 32.32 fixed-point rate, exact in 64 bits */
static int64_t cum_count(uint64_t R, int64_t n) {
    uint64_t hi = R >> 32, lo = R & 0xFFFFFFFFULL;
    return (int64_t)((uint64_t)n * hi + (((uint64_t)n * lo) >> 32));
}

int64_t orc_inject_count(const orc_ocean *o, int32_t p, int32_t i, int32_t pair, int64_t n) {
    if (p < 0 || p >= o->np || i < 0 || i >= o->nb || n < 1) return -1;
    uint64_t R = pair == 0 ? o->pt[p].Rx[i] : o->pt[p].Ry[i];
    return cum_count(R, n) - cum_count(R, n - 1);
}

static void rebuild_hist(orc_ocean *o) {
    for (int p = 0; p < o->np; ++p) {
        patch_t *pt = &o->pt[p];
        for (int i = 0; i < o->nb; ++i) {
            int64_t m = o->margin[i];
            int64_t span_x = pt->nx * pt->dxu + 2 * m, span_y = pt->ny * pt->dxu + 2 * m;
            int64_t binu = (int64_t)o->bin_cells[i] * pt->dxu;
            pt->binw[i] = o->bin_cells[i];
            pt->nbx[i] = fdiv(span_x, binu) + 1;
            pt->nby[i] = fdiv(span_y, binu) + 1;
            size_t nh = (size_t)(pt->nbx[i] * pt->nby[i]);
            if (!pt->hist[i]) pt->hist[i] = (int64_t *)malloc(sizeof(int64_t) * nh);
            memset(pt->hist[i], 0, sizeof(int64_t) * nh);
            pt->cnt[i][C_LIVE] = 0;
        }
    }
    for (int64_t k = 0; k < o->nP; ++k) {
        const prt_t *q = &o->P[k];
        patch_t *pt = &o->pt[q->patch];
        int i = q->bucket;
        int64_t px, py;
        position(o, q, o->n, &px, &py);
        int64_t m = o->margin[i];
        int64_t binu = (int64_t)o->bin_cells[i] * pt->dxu;
        int64_t bx = fdiv(px - (pt->wx * pt->dxu - m), binu);
        int64_t by = fdiv(py - (pt->wy * pt->dxu - m), binu);
        pt->hist[i][by * pt->nbx[i] + bx] += 1;
        pt->cnt[i][C_LIVE] += 1;
    }
}

static int step_once(orc_ocean *o) {
    int64_t n = o->n + 1;
    update_windows(o, n);
    prt_t *NP = NULL;
    int64_t nn = 0, cap = 0;
    prt_t out[3];

    /* existing particles: subdivide, then survive */
    for (int64_t k = 0; k < o->nP; ++k) {
        const prt_t *q = &o->P[k];
        int64_t age = n - q->birth;
        int nout = 1;
        out[0] = *q;
        if (q->kind >= 1 && q->level < o->lmax && age >= o->sr[q->src].T[q->level]) {
            int32_t off = (int32_t)(o->sr[q->src].a0 / ipow3(q->level + 1));
            out[0].level = q->level + 1;
            out[1] = out[0];
            out[2] = out[0];
            out[1].code = (int32_t)pmod(q->code - off, NCODE);
            out[2].code = (int32_t)pmod(q->code + off, NCODE);
            nout = 3;
            o->pt[q->patch].cnt[q->bucket][C_SUB] += 1;
        }
        for (int j = 0; j < nout; ++j) {
            if (alive(o, &out[j], n))
                push(o, &NP, &nn, &cap, &out[j]);
            else
                o->pt[out[j].patch].cnt[out[j].bucket][C_DIED] += 1;
        }
    }

    /* boundary injection, Eq 18 per pair of opposite sides */
    for (int p = 0; p < o->np; ++p) {
        patch_t *pt = &o->pt[p];
        for (int i = 0; i < o->nb; ++i) {
            for (int pair = 0; pair < 2; ++pair) {
                uint64_t R = pair == 0 ? pt->Rx[i] : pt->Ry[i];
                int64_t cnt = cum_count(R, n) - cum_count(R, n - 1);
                for (int64_t j = 0; j < cnt; ++j) {
                    uint64_t ctr[4] = {(uint64_t)p, (uint64_t)(i * 2 + pair), (uint64_t)n, (uint64_t)j};
                    uint64_t key[2] = {o->seed, STREAM_INJECT};
                    uint64_t u[4];
                    orc_philox4x64(ctr, key, u);
                    prt_t q;
                    memset(&q, 0, sizeof q);
                    if (o->dir_mode == 0) {
                        /* inverse CDF of Dir over the 64 direction bins */
                        uint64_t t = mulhi64(u[0], (uint64_t)o->Q[i][pair]);
                        int b = 0;
                        while (!((int64_t)t < o->cdf[i][pair][b])) ++b;
                        q.code = o->codes[b];
                    } else {
                        /* stratified group (Sec 3.3): the m-th particle of this
                         * side pair's stream takes sector m mod N_theta of
                         * [-pi, pi) around the wind, uniformly inside it */
                        int64_t nth = (int64_t)pt->eta;
                        int64_t m = cum_count(R, n - 1) + j;
                        int64_t s = m % nth;
                        int64_t lo = s * NCODE / nth, hi = (s + 1) * NCODE / nth;
                        q.code = (int32_t)pmod((int64_t)o->wind_code + NCODE / 2 + lo +
                                                   (int64_t)mulhi64(u[0], (uint64_t)(hi - lo)), NCODE);
                    }
                    const int64_t *v = &o->V[((size_t)i * NCODE + q.code) * 2];
                    if (pair == 0) {
                        q.ox = (v[0] > 0) ? pt->wx * pt->dxu : (pt->wx + pt->nx) * pt->dxu;
                        q.oy = pt->wy * pt->dxu + (int64_t)mulhi64(u[1], (uint64_t)(pt->ny * pt->dxu));
                    } else {
                        q.oy = (v[1] > 0) ? pt->wy * pt->dxu : (pt->wy + pt->ny) * pt->dxu;
                        q.ox = pt->wx * pt->dxu + (int64_t)mulhi64(u[1], (uint64_t)(pt->nx * pt->dxu));
                    }
                    q.birth = n;
                    q.level = 0;
                    q.kind = 0;
                    q.bucket = i;
                    q.patch = p;
                    q.src = -1;
                    q.slot = 0;
                    pt->cnt[i][C_INJ] += 1;
                    if (alive(o, &q, n))
                        push(o, &NP, &nn, &cap, &q);
                    else
                        pt->cnt[i][C_DIED] += 1;
                }
            }
        }
    }

    /* source ring emission: the horizontal-motion ring (kind 1) and the
     * vertical-motion ring (kind 2), each on its own cadence */
    for (int si = 0; si < o->ns; ++si) {
        const src_t *s = &o->sr[si];
        const int horizontal = s->E > 0 && ((n - 1) % s->E) == 0;
        const int vertical = s->heave_a > 0 && ((n - 1) % s->Eh) == 0;
        if (!horizontal && !vertical) continue;
        patch_t *pt = &o->pt[s->patch];
        double xs, ys;
        source_pos(o, s, n, &xs, &ys);
        int64_t sx = llround((xs - pt->ax) * UNIT);
        int64_t sy = llround((ys - pt->ay) * UNIT);
        for (int kind = 1; kind <= 2; ++kind) {
            if (kind == 1 ? !horizontal : !vertical) continue;
            for (int j = 0; j < s->ne; ++j) {
                prt_t q;
                memset(&q, 0, sizeof q);
                q.ox = sx + s->Ox[j];
                q.oy = sy + s->Oy[j];
                q.birth = n;
                q.code = j * s->a0;
                q.level = 0;
                q.kind = kind;
                q.bucket = s->bucket;
                q.patch = s->patch;
                q.src = si;
                q.slot = j;
                pt->cnt[s->bucket][C_EMIT] += 1;
                if (alive(o, &q, n))
                    push(o, &NP, &nn, &cap, &q);
                else
                    pt->cnt[s->bucket][C_DIED] += 1;
            }
        }
    }

    free(o->P);
    o->P = NP;
    o->nP = nn;
    o->capP = cap;
    o->n = n;
    return 0;
}

int orc_step(orc_ocean *o, int32_t nsteps) {
    if (!o->have_spec) return fail(o, "set_spectrum first");
    if (nsteps < 0) return fail(o, "nsteps must be >= 0");
    o->stepped = 1;
    for (int32_t k = 0; k < nsteps; ++k) step_once(o);
    update_windows(o, o->n);
    rebuild_hist(o);
    return 0;
}

int64_t orc_step_index(const orc_ocean *o) { return o->n; }

int orc_window(const orc_ocean *o, int32_t p, int64_t *w) {
    if (p < 0 || p >= o->np) return -1;
    w[0] = o->pt[p].wx;
    w[1] = o->pt[p].wy;
    return 0;
}

int orc_counts(const orc_ocean *o, int32_t p, int64_t *dst) {
    if (p < 0 || p >= o->np) return -1;
    for (int i = 0; i < o->nb; ++i)
        for (int k = 0; k < C_NUM; ++k) dst[i * C_NUM + k] = o->pt[p].cnt[i][k];
    return 0;
}

int orc_tile_dims(const orc_ocean *o, int32_t p, int32_t i, int64_t *dims) {
    if (p < 0 || p >= o->np || i < 0 || i >= o->nb || !o->pt[p].hist[i]) return -1;
    dims[0] = o->pt[p].binw[i];
    dims[1] = o->pt[p].nbx[i];
    dims[2] = o->pt[p].nby[i];
    return 0;
}

int orc_tiles(const orc_ocean *o, int32_t p, int32_t i, int64_t *dst, int64_t n) {
    if (p < 0 || p >= o->np || i < 0 || i >= o->nb || !o->pt[p].hist[i]) return -1;
    int64_t nh = o->pt[p].nbx[i] * o->pt[p].nby[i];
    if (n < nh) return -1;
    memcpy(dst, o->pt[p].hist[i], sizeof(int64_t) * (size_t)nh);
    return 0;
}

int64_t orc_num_particles(const orc_ocean *o) { return o->nP; }

int64_t orc_particles(const orc_ocean *o, int64_t *dst, int64_t n) {
    int64_t k;
    for (k = 0; k < o->nP && k < n; ++k) {
        const prt_t *q = &o->P[k];
        int64_t *d = dst + 10 * k;
        d[0] = q->patch;
        d[1] = q->bucket;
        d[2] = q->kind;
        d[3] = q->level;
        d[4] = q->code;
        d[5] = q->birth;
        d[6] = q->ox;
        d[7] = q->oy;
        d[8] = q->src;
        d[9] = q->slot;
    }
    return k;
}

/* ---------------------------------------------------------------- FFT */
/* Radix-2 decimation-in-time, e^{+i} kernel, no normalisation. */
void orc_fft_inverse(double *re, double *im, int32_t n) {
    for (int32_t i = 1, j = 0; i < n; ++i) {
        int32_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    double *tc = (double *)malloc(sizeof(double) * (size_t)(n / 2 + 1));
    double *ts = (double *)malloc(sizeof(double) * (size_t)(n / 2 + 1));
    for (int32_t k = 0; k <= n / 2; ++k) {
        tc[k] = cos(2.0 * M_PI * (double)k / (double)n);
        ts[k] = sin(2.0 * M_PI * (double)k / (double)n);
    }
    for (int32_t len = 2; len <= n; len <<= 1) {
        int32_t half = len / 2, stride = n / len;
        for (int32_t i = 0; i < n; i += len) {
            for (int32_t k = 0; k < half; ++k) {
                double wr = tc[k * stride], wi = ts[k * stride];
                double xr = re[i + k + half], xi = im[i + k + half];
                double vr = xr * wr - xi * wi, vi = xr * wi + xi * wr;
                double ur = re[i + k], ui = im[i + k];
                re[i + k] = ur + vr;
                im[i + k] = ui + vi;
                re[i + k + half] = ur - vr;
                im[i + k + half] = ui - vi;
            }
        }
    }
    free(tc);
    free(ts);
}

void orc_fft2_inverse(double *re, double *im, int32_t n) {
    for (int32_t y = 0; y < n; ++y) orc_fft_inverse(re + (size_t)y * n, im + (size_t)y * n, n);
    double *cr = (double *)malloc(sizeof(double) * (size_t)n);
    double *ci = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t x = 0; x < n; ++x) {
        for (int32_t y = 0; y < n; ++y) {
            cr[y] = re[(size_t)y * n + x];
            ci[y] = im[(size_t)y * n + x];
        }
        orc_fft_inverse(cr, ci, n);
        for (int32_t y = 0; y < n; ++y) {
            re[(size_t)y * n + x] = cr[y];
            im[(size_t)y * n + x] = ci[y];
        }
    }
    free(cr);
    free(ci);
}

/* Naive O(N^4) 2D inverse DFT, for small-grid pins. */
void orc_dft2_inverse(const double *re, const double *im, double *ore, double *oim, int32_t n) {
    for (int32_t jy = 0; jy < n; ++jy)
        for (int32_t jx = 0; jx < n; ++jx) {
            double sr = 0.0, si = 0.0;
            for (int32_t my = 0; my < n; ++my)
                for (int32_t mx = 0; mx < n; ++mx) {
                    int64_t ph = ((int64_t)mx * jx + (int64_t)my * jy) % n;
                    double a = 2.0 * M_PI * (double)ph / (double)n;
                    double c = cos(a), s = sin(a);
                    double xr = re[(size_t)my * n + mx], xi = im[(size_t)my * n + mx];
                    sr += xr * c - xi * s;
                    si += xr * s + xi * c;
                }
            ore[(size_t)jy * n + jx] = sr;
            oim[(size_t)jy * n + jx] = si;
        }
}

/* ---------------------------------------------------------------- h0 */
static int32_t signed_index(int32_t j, int32_t n) { return j < n / 2 ? j : j - n; }

/* h0(k) = 1/2 (xi_r + i xi_i) sqrt(S_k) dk with S_k = S(w, theta) g / (2 w k),
 * so that sum_k E|h(k)|^2 approximates the spectral variance. */
static void gen_h0(orc_ocean *o) {
    int32_t N = o->N;
    free(o->h0re);
    free(o->h0im);
    o->h0re = (double *)calloc((size_t)N * N, sizeof(double));
    o->h0im = (double *)calloc((size_t)N * N, sizeof(double));
    double dk = 2.0 * M_PI / o->L;
    for (int32_t jy = 0; jy < N; ++jy)
        for (int32_t jx = 0; jx < N; ++jx) {
            int32_t mx = signed_index(jx, N), my = signed_index(jy, N);
            if (mx == 0 && my == 0) continue;
            double kx = dk * (double)mx, ky = dk * (double)my;
            double k = sqrt(kx * kx + ky * ky);
            double w = sqrt(o->g * k);
            double th = atan2(ky, kx) - o->wind_dir;
            th = th - 2.0 * M_PI * floor((th + M_PI) / (2.0 * M_PI));
            double Sk = orc_jonswap(o, w) * orc_dir(o, w, th) * o->g / (2.0 * w * k);
            uint64_t ctr[4] = {(uint64_t)jy, (uint64_t)jx, 0, 0};
            uint64_t key[2] = {o->seed, STREAM_H0};
            uint64_t u[4];
            orc_philox4x64(ctr, key, u);
            double ua = unit_open(u[0]), ub = unit_open(u[1]);
            double hr, hi;
            if (o->h0_mode == 1) {
                double amp = dk * sqrt(0.5 * Sk);
                hr = amp * cos(2.0 * M_PI * ub);
                hi = amp * sin(2.0 * M_PI * ub);
            } else {
                double rho = sqrt(-2.0 * log(ua));
                double amp = 0.5 * sqrt(Sk) * dk;
                hr = amp * rho * cos(2.0 * M_PI * ub);
                hi = amp * rho * sin(2.0 * M_PI * ub);
            }
            o->h0re[(size_t)jy * N + jx] = hr;
            o->h0im[(size_t)jy * N + jx] = hi;
        }
}

int orc_h0(const orc_ocean *o, double *re, double *im) {
    if (!o->have_spec) return -1;
    size_t n2 = (size_t)o->N * o->N;
    memcpy(re, o->h0re, sizeof(double) * n2);
    memcpy(im, o->h0im, sizeof(double) * n2);
    return 0;
}

int orc_set_h0(orc_ocean *o, const double *re, const double *im) {
    if (!o->have_spec) return -1;
    size_t n2 = (size_t)o->N * o->N;
    memcpy(o->h0re, re, sizeof(double) * n2);
    memcpy(o->h0im, im, sizeof(double) * n2);
    return 0;
}

/* H(x_j, t) = Re sum_k htilde(k, t) e^{i k.x_j},
 * htilde(k, t) = h0(k) e^{-i w t} + conj(h0(-k)) e^{+i w t}, w = sqrt(g |k|). */
/* Background fields derived from the same spectrum (choppy displacement and
 * slopes, the usual companions of the height transform): field 0 height H,
 * 1 and 2 the slopes dH/dx and dH/dy (spectrum times i kx, i ky), 3 and 4
 * the horizontal displacements D = sum -i (k / |k|) h~ e^{ik.x} (x and y).
 * For fields 1-4 the Nyquist rows and columns and k = 0 carry nothing, so
 * every field stays real. */
int orc_background_field(orc_ocean *o, int32_t field, double t, double *H) {
    if (!o->have_spec) return fail(o, "set_spectrum first");
    if (field < 0 || field > 4) return fail(o, "field must be 0..4");
    int32_t N = o->N;
    size_t n2 = (size_t)N * N;
    double *re = (double *)malloc(sizeof(double) * n2);
    double *im = (double *)malloc(sizeof(double) * n2);
    double dk = 2.0 * M_PI / o->L;
    for (int32_t jy = 0; jy < N; ++jy)
        for (int32_t jx = 0; jx < N; ++jx) {
            int32_t mx = signed_index(jx, N), my = signed_index(jy, N);
            double kx = dk * (double)mx, ky = dk * (double)my;
            double w = sqrt(o->g * sqrt(kx * kx + ky * ky));
            double c = cos(w * t), s = sin(w * t);
            size_t a = (size_t)jy * N + jx;
            size_t b = (size_t)((N - jy) % N) * N + (size_t)((N - jx) % N);
            double ar = o->h0re[a], ai = o->h0im[a];
            double br = o->h0re[b], bi = -o->h0im[b]; /* conj(h0(-k)) */
            /* a e^{-iwt} + b e^{+iwt} */
            double hr = ar * c + ai * s + br * c - bi * s;
            double hi = ai * c - ar * s + bi * c + br * s;
            double m = 0.0; /* the factor is i m for fields 1-4 */
            if (field != 0 && jx != N / 2 && jy != N / 2) {
                double kk = sqrt(kx * kx + ky * ky);
                if (field == 1) m = kx;
                else if (field == 2) m = ky;
                else if (kk > 0.0) m = -(field == 3 ? kx : ky) / kk;
            }
            if (field == 0) {
                re[a] = hr;
                im[a] = hi;
            } else {
                re[a] = -m * hi;
                im[a] = m * hr;
            }
        }
    orc_fft2_inverse(re, im, N);
    for (size_t k = 0; k < n2; ++k) H[k] = re[k];
    free(re);
    free(im);
    return 0;
}

int orc_background_at(orc_ocean *o, double t, double *H) { return orc_background_field(o, 0, t, H); }

int orc_background(orc_ocean *o, double *H) { return orc_background_at(o, (double)o->n * o->dt, H); }

/* ---------------------------------------------------------------- splat */
static double amplitude(const orc_ocean *o, const prt_t *q) {
    if (q->kind == 0) {
        const patch_t *pt = &o->pt[q->patch];
        if (o->dir_mode == 0) return pt->A[q->bucket];
        /* Eq 7 with the particle's own direction and dtheta = 2 pi / N_theta:
         * A^2 = 2 S_J(w_i) Dir(theta) dw_i dtheta = A_{p,i}^2 * 2 pi Dir(theta) */
        double th = 2.0 * M_PI * (double)q->code / (double)NCODE - o->wind_dir;
        return pt->A[q->bucket] * sqrt(2.0 * M_PI * dir_s(orc_spread(o, o->w[q->bucket]), th));
    }
    const src_t *s = &o->sr[q->src];
    if (q->kind == 2)   /* heave ring: the volume displaced between its birth and the previous ring */
        return s->Bh * (heave_z(o, s, q->birth - s->Eh) - heave_z(o, s, q->birth)) / (double)ipow3(q->level);
    return s->B * s->m[q->slot] / (double)ipow3(q->level);
}

/* w(d) = 1/2 (1 + cos(pi d / r)) for |d| < r, else 0 (raised cosine) */
static double wker(double d, double r) {
    if (fabs(d) >= r) return 0.0;
    return 0.5 * (1.0 + cos(M_PI * d / r));
}

/* Add A * w(x_c - cx) w(y_c - cy) over the patch cells; cx, cy in 2^-20 m units. */
static void splat_kernel(const orc_ocean *o, const patch_t *pt, double *raw, double cxu, double cyu,
                         double A, double r, double *wxv, double *wyv) {
    double dxu = (double)pt->dxu;
    double ru = r * UNIT;
    int64_t i0 = (int64_t)floor((cxu - ru) / dxu) - pt->wx - 1;
    int64_t i1 = (int64_t)ceil((cxu + ru) / dxu) - pt->wx + 1;
    int64_t j0 = (int64_t)floor((cyu - ru) / dxu) - pt->wy - 1;
    int64_t j1 = (int64_t)ceil((cyu + ru) / dxu) - pt->wy + 1;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > pt->nx - 1) i1 = pt->nx - 1;
    if (j1 > pt->ny - 1) j1 = pt->ny - 1;
    if (i0 > i1 || j0 > j1) return;
    (void)o;
    for (int64_t i = i0; i <= i1; ++i) {
        double xc = (double)((pt->wx + i) * pt->dxu + pt->dxu / 2);
        wxv[i - i0] = wker((xc - cxu) / UNIT, r);
    }
    for (int64_t j = j0; j <= j1; ++j) {
        double yc = (double)((pt->wy + j) * pt->dxu + pt->dxu / 2);
        wyv[j - j0] = wker((yc - cyu) / UNIT, r);
    }
    for (int64_t j = j0; j <= j1; ++j) {
        double ay = A * wyv[j - j0];
        if (ay == 0.0) continue;
        double *row = raw + (size_t)j * pt->nx;
        for (int64_t i = i0; i <= i1; ++i) row[i] += ay * wxv[i - i0];
    }
}

/* Radial variant of the same profile: add A * w(|x_c - c|) over the patch
 * cells, with the distance taken in the plane rather than per axis. */
static void splat_kernel_radial(const patch_t *pt, double *raw, double cxu, double cyu, double A, double r) {
    double dxu = (double)pt->dxu;
    double ru = r * UNIT;
    int64_t i0 = (int64_t)floor((cxu - ru) / dxu) - pt->wx - 1;
    int64_t i1 = (int64_t)ceil((cxu + ru) / dxu) - pt->wx + 1;
    int64_t j0 = (int64_t)floor((cyu - ru) / dxu) - pt->wy - 1;
    int64_t j1 = (int64_t)ceil((cyu + ru) / dxu) - pt->wy + 1;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > pt->nx - 1) i1 = pt->nx - 1;
    if (j1 > pt->ny - 1) j1 = pt->ny - 1;
    for (int64_t j = j0; j <= j1; ++j) {
        double yc = (double)((pt->wy + j) * pt->dxu + pt->dxu / 2);
        for (int64_t i = i0; i <= i1; ++i) {
            double xc = (double)((pt->wx + i) * pt->dxu + pt->dxu / 2);
            double rho = hypot(xc - cxu, yc - cyu) / UNIT;
            raw[(size_t)j * pt->nx + i] += A * wker(rho, r);
        }
    }
}

/* Crest +A at the particle, trough -A one radius behind it along its
 * direction (the positive-negative pair of Fig 1). */
static void splat_particle(const orc_ocean *o, const patch_t *pt, double *raw, const prt_t *q,
                           double *wxv, double *wyv) {
    int64_t px, py;
    position(o, q, o->n, &px, &py);
    double r = o->r[q->bucket];
    double A = amplitude(o, q);
    double ang = 2.0 * M_PI * (double)q->code / (double)NCODE;
    double tx = r * cos(ang) * UNIT, ty = r * sin(ang) * UNIT;
    if (o->kernel == 1) {
        splat_kernel_radial(pt, raw, (double)px, (double)py, A, r);
        splat_kernel_radial(pt, raw, (double)px - tx, (double)py - ty, -A, r);
        return;
    }
    splat_kernel(o, pt, raw, (double)px, (double)py, A, r, wxv, wyv);
    splat_kernel(o, pt, raw, (double)px - tx, (double)py - ty, -A, r, wxv, wyv);
}

/* ---------------------------------------------------------------- texel layers
 * Sec 4.2 synthesis: every particle point (crest +A at p, trough -A at
 * p - r u) is accumulated into its bucket's layer texture on the patch's cell
 * grid, each layer is smoothed by a pass along x and then along y with the
 * raised cosine sampled at whole-cell offsets, and the layers are summed.
 * Deposit is bilinear onto the four surrounding cell centres (the paper does
 * not state the deposit; bilinear keeps the texel result within O(dx^2) of
 * the exact-position kernel).  The trough offset is rounded to position
 * units, round(r (cos, sin) 2^20), so texel choices are exact integers.
 * A layer spans the patch plus R = ceil(r / dx) - 1 cells on each side: the
 * taps w(k dx) are non-zero for |k| <= R only, so deposits farther out never
 * reach a patch cell. */
static int64_t layer_reach(const patch_t *pt, double r) {
    int64_t R = (int64_t)ceil(r / pt->dx) - 1;
    return R < 0 ? 0 : R;
}

static void deposit(const patch_t *pt, double *lay, int64_t R, int64_t xu, int64_t yu, double A) {
    const int64_t W = pt->nx + 2 * R, Hh = pt->ny + 2 * R;
    const int64_t h = pt->dxu / 2;
    int64_t X = xu - pt->wx * pt->dxu - h, Y = yu - pt->wy * pt->dxu - h;
    int64_t i0 = fdiv(X, pt->dxu), j0 = fdiv(Y, pt->dxu);
    double tx = (double)(X - i0 * pt->dxu) / (double)pt->dxu;
    double ty = (double)(Y - j0 * pt->dxu) / (double)pt->dxu;
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            int64_t i = i0 + di + R, j = j0 + dj + R;
            if (i < 0 || i >= W || j < 0 || j >= Hh) continue;
            double wgt = (di ? tx : 1.0 - tx) * (dj ? ty : 1.0 - ty);
            lay[j * W + i] += A * wgt;
        }
}

static void layer_synth(const orc_ocean *o, const patch_t *pt, double *raw, const prt_t *P, int64_t n, int32_t p) {
    for (int b = 0; b < o->nb; ++b) {
        const double r = o->r[b];
        const int64_t R = layer_reach(pt, r);
        const int64_t W = pt->nx + 2 * R, Hh = pt->ny + 2 * R;
        double *lay = (double *)calloc((size_t)(W * Hh), sizeof(double));
        double *T = (double *)calloc((size_t)(pt->nx * Hh), sizeof(double));
        double *w = (double *)malloc(sizeof(double) * (size_t)(2 * R + 1));
        for (int64_t k = -R; k <= R; ++k) w[k + R] = wker((double)k * pt->dx, r);
        for (int64_t k = 0; k < n; ++k) {
            const prt_t *q = &P[k];
            if (q->patch != p || q->bucket != b) continue;
            int64_t px, py;
            position(o, q, o->n, &px, &py);
            double A = amplitude(o, q);
            double ang = 2.0 * M_PI * (double)q->code / (double)NCODE;
            int64_t tx = llround(r * cos(ang) * UNIT), ty = llround(r * sin(ang) * UNIT);
            deposit(pt, lay, R, px, py, A);
            deposit(pt, lay, R, px - tx, py - ty, -A);
        }
        /* pass along x: T[j][i] = sum_k lay[j][i + R - k] w(k dx), i in the patch */
        for (int64_t j = 0; j < Hh; ++j)
            for (int64_t i = 0; i < pt->nx; ++i) {
                double s = 0.0;
                for (int64_t k = -R; k <= R; ++k) s += lay[j * W + i + R - k] * w[k + R];
                T[j * pt->nx + i] = s;
            }
        /* pass along y, summed into the patch map */
        for (int64_t j = 0; j < pt->ny; ++j)
            for (int64_t i = 0; i < pt->nx; ++i) {
                double s = 0.0;
                for (int64_t k = -R; k <= R; ++k) s += T[(j + R - k) * pt->nx + i] * w[k + R];
                raw[j * pt->nx + i] += s;
            }
        free(lay);
        free(T);
        free(w);
    }
}

int orc_set_synthesis(orc_ocean *o, int32_t mode, int32_t kernel) {
    if (mode != 0 && mode != 1) return fail(o, "synthesis mode must be 0 or 1");
    if (kernel != 0 && kernel != 1) return fail(o, "kernel must be 0 or 1");
    if (kernel == 1 && mode != 0) return fail(o, "the radial kernel needs the exact-position synthesis");
    o->synth = mode;
    o->kernel = kernel;
    return 0;
}

static void blend(const orc_ocean *o, const patch_t *pt, const double *H, const double *raw,
                  double *out) {
    int32_t N = o->N;
    double dxf = o->L / (double)N;
    for (int32_t j = 0; j < pt->ny; ++j)
        for (int32_t i = 0; i < pt->nx; ++i) {
            double di = fmin(fmin((double)i + 0.5, (double)pt->nx - (double)i - 0.5),
                             fmin((double)j + 0.5, (double)pt->ny - (double)j - 0.5)) * pt->dx;
            double t = di / pt->band;
            if (t > 1.0) t = 1.0;
            double wgt = t * t * (3.0 - 2.0 * t);
            double X = pt->ax + (double)((pt->wx + i) * pt->dxu + pt->dxu / 2) / UNIT;
            double Y = pt->ay + (double)((pt->wy + j) * pt->dxu + pt->dxu / 2) / UNIT;
            double fx = X / dxf, fy = Y / dxf;
            fx -= (double)N * floor(fx / (double)N);
            fy -= (double)N * floor(fy / (double)N);
            int64_t x0 = (int64_t)floor(fx), y0 = (int64_t)floor(fy);
            double a = fx - (double)x0, b = fy - (double)y0;
            int64_t x0m = pmod(x0, N), y0m = pmod(y0, N);
            int64_t x1m = (x0m + 1) % N, y1m = (y0m + 1) % N;
            double h00 = H[y0m * N + x0m], h01 = H[y0m * N + x1m];
            double h10 = H[y1m * N + x0m], h11 = H[y1m * N + x1m];
            double hb = (1.0 - b) * ((1.0 - a) * h00 + a * h01) + b * ((1.0 - a) * h10 + a * h11);
            size_t c = (size_t)j * pt->nx + i;
            out[c] = wgt * raw[c] + (1.0 - wgt) * hb;
        }
}

int orc_patch_maps(orc_ocean *o, int32_t p, const double *H, double *raw, double *blended) {
    if (p < 0 || p >= o->np) return fail(o, "patch out of range");
    const patch_t *pt = &o->pt[p];
    size_t nc = (size_t)pt->nx * pt->ny;
    memset(raw, 0, sizeof(double) * nc);
    if (o->synth == 1) {
        layer_synth(o, pt, raw, o->P, o->nP, p);
    } else {
        int64_t wmax = pt->nx > pt->ny ? pt->nx : pt->ny;
        double *wxv = (double *)malloc(sizeof(double) * (size_t)(wmax + 8));
        double *wyv = (double *)malloc(sizeof(double) * (size_t)(wmax + 8));
        for (int64_t k = 0; k < o->nP; ++k)
            if (o->P[k].patch == p) splat_particle(o, pt, raw, &o->P[k], wxv, wyv);
        free(wxv);
        free(wyv);
    }
    if (blended) {
        double *Hown = NULL;
        if (!H) {
            Hown = (double *)malloc(sizeof(double) * (size_t)o->N * o->N);
            orc_background(o, Hown);
            H = Hown;
        }
        blend(o, pt, H, raw, blended);
        free(Hown);
    }
    return 0;
}

/* Set the step index of an oracle that holds no particles, with the windows
 * of that step, so that caller-supplied particles (orc_splat) and maps
 * (orc_blend) are evaluated at step n.  The oracle's own state does not
 * advance: injection, emission and counters are not run. */
int orc_seek(orc_ocean *o, int64_t n) {
    if (!o->have_spec) return fail(o, "set_spectrum first");
    if (o->nP > 0) return fail(o, "seek needs an oracle without particles");
    if (n < 0) return fail(o, "step must be >= 0");
    o->stepped = 1;
    o->n = n;
    update_windows(o, n);
    return 0;
}

/* Blend a caller-supplied raw map of patch p with background H (N x N) at
 * the current step. */
int orc_blend(orc_ocean *o, int32_t p, const double *H, const double *raw, double *blended) {
    if (p < 0 || p >= o->np) return fail(o, "patch out of range");
    if (!H || !raw || !blended) return fail(o, "null map");
    blend(o, &o->pt[p], H, raw, blended);
    return 0;
}

/* Sec 4.2: normals of a patch map by finite differences.  The slope along x
 * at cell (i, j) is the central difference (h[i+1] - h[i-1]) / (2 dx), one-
 * sided at the first and last column (zero for a single column); likewise
 * along y.  The unit normal is (-sx, -sy, 1) / sqrt(1 + sx^2 + sy^2), stored
 * as three ny x nx planes (x, y, z components). */
int orc_normals(orc_ocean *o, int32_t p, const double *h, double *out) {
    if (p < 0 || p >= o->np) return fail(o, "patch out of range");
    if (!h || !out) return fail(o, "null map");
    const patch_t *pt = &o->pt[p];
    const int64_t nx = pt->nx, ny = pt->ny, nc = nx * ny;
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            double sx = 0.0, sy = 0.0;
            if (nx > 1) {
                int64_t a = i > 0 ? i - 1 : i, b = i < nx - 1 ? i + 1 : i;
                sx = (h[j * nx + b] - h[j * nx + a]) / ((double)(b - a) * pt->dx);
            }
            if (ny > 1) {
                int64_t a = j > 0 ? j - 1 : j, b = j < ny - 1 ? j + 1 : j;
                sy = (h[b * nx + i] - h[a * nx + i]) / ((double)(b - a) * pt->dx);
            }
            double inv = 1.0 / sqrt(1.0 + sx * sx + sy * sy);
            out[j * nx + i] = -sx * inv;
            out[nc + j * nx + i] = -sy * inv;
            out[2 * nc + j * nx + i] = inv;
        }
    return 0;
}

/* Sec 4.3 object-receives-water: the surface seen by a floating object at
 * probe points.  A probe inside the cell-centre hull of a patch (the first
 * such patch in index order) samples that patch's blended map, else the
 * background (periodic).  Height is the bilinear interpolant of the map;
 * the slopes are central differences at the four surrounding grid points
 * (one-sided at a patch's first and last row or column), interpolated the
 * same way; the normal is (-sx, -sy, 1) normalised.  H is the N x N
 * background, B the blended maps of all patches back to back; out receives
 * four values per probe: height and the normal's x, y, z. */
static void fd_slopes(const double *h, int64_t nx, int64_t ny, int periodic, int64_t i, int64_t j,
                      double dx, double *sx, double *sy) {
    int64_t a, b;
    if (periodic) {
        a = (i + nx - 1) % nx; b = (i + 1) % nx;
        *sx = (h[j * nx + b] - h[j * nx + a]) / (2.0 * dx);
        a = (j + ny - 1) % ny; b = (j + 1) % ny;
        *sy = (h[b * nx + i] - h[a * nx + i]) / (2.0 * dx);
        return;
    }
    *sx = 0.0;
    *sy = 0.0;
    if (nx > 1) {
        a = i > 0 ? i - 1 : i; b = i < nx - 1 ? i + 1 : i;
        *sx = (h[j * nx + b] - h[j * nx + a]) / ((double)(b - a) * dx);
    }
    if (ny > 1) {
        a = j > 0 ? j - 1 : j; b = j < ny - 1 ? j + 1 : j;
        *sy = (h[b * nx + i] - h[a * nx + i]) / ((double)(b - a) * dx);
    }
}

int orc_sample_probes(orc_ocean *o, const double *H, const double *B, const double *xy, int64_t n, double *out) {
    if (!H || !B || (!xy && n > 0) || (!out && n > 0)) return fail(o, "null input");
    const int64_t N = o->N;
    const double dxf = o->L / (double)N;
    for (int64_t q = 0; q < n; ++q) {
        const double x = xy[2 * q], y = xy[2 * q + 1];
        const double *h = H;
        int64_t nx = N, ny = N, i0, j0;
        double fx, fy, dx = dxf;
        int periodic = 1;
        int64_t off = 0;
        int found = 0;
        for (int p = 0; p < o->np && !found; ++p) {
            const patch_t *pt = &o->pt[p];
            double u = (x - pt->ax) * UNIT / (double)pt->dxu - (double)pt->wx - 0.5;
            double v = (y - pt->ay) * UNIT / (double)pt->dxu - (double)pt->wy - 0.5;
            if (u >= 0.0 && v >= 0.0 && u <= (double)(pt->nx - 1) && v <= (double)(pt->ny - 1)) {
                found = 1;
                h = B + off;
                nx = pt->nx;
                ny = pt->ny;
                dx = pt->dx;
                periodic = 0;
                i0 = (int64_t)floor(u);
                j0 = (int64_t)floor(v);
                if (i0 > nx - 2) i0 = nx > 1 ? nx - 2 : 0;
                if (j0 > ny - 2) j0 = ny > 1 ? ny - 2 : 0;
                fx = u - (double)i0;
                fy = v - (double)j0;
            }
            off += (int64_t)pt->nx * pt->ny;
        }
        if (!found) {
            double u = x / dxf, v = y / dxf;
            double fu = floor(u), fv = floor(v);
            fx = u - fu;
            fy = v - fv;
            i0 = pmod((int64_t)fu, N);
            j0 = pmod((int64_t)fv, N);
        }
        double hv = 0.0, sxv = 0.0, syv = 0.0;
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                int64_t i = i0 + di, j = j0 + dj;
                if (periodic) { i %= nx; j %= ny; }
                else {
                    if (i > nx - 1) i = nx - 1;
                    if (j > ny - 1) j = ny - 1;
                }
                double w = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy);
                double sx, sy;
                fd_slopes(h, nx, ny, periodic, i, j, dx, &sx, &sy);
                hv += w * h[j * nx + i];
                sxv += w * sx;
                syv += w * sy;
            }
        double inv = 1.0 / sqrt(1.0 + sxv * sxv + syv * syv);
        out[4 * q + 0] = hv;
        out[4 * q + 1] = -sxv * inv;
        out[4 * q + 2] = -syv * inv;
        out[4 * q + 3] = inv;
    }
    return 0;
}

/* Splat caller-placed particles (canonical records) into a patch map at the
 * current step; used by the closed-form pins. */
/* Replace the particle state by caller-supplied records (ten integer
 * columns, the layout of orc_particles) as the state after step n, with the
 * windows and bin histograms of that step; the counters are left as they
 * are.  Test infrastructure for timing a full frame of a large scene without
 * re-running its whole history: the next orc_step continues from step n. */
int orc_load(orc_ocean *o, int64_t n, const int64_t *recs, int64_t count) {
    if (!o->have_spec) return fail(o, "set_spectrum first");
    if (n < 0 || count < 0) return fail(o, "step and count must be >= 0");
    prt_t *P = (prt_t *)malloc(sizeof(prt_t) * (size_t)(count > 0 ? count : 1));
    if (!P) return fail(o, "out of memory");
    for (int64_t k = 0; k < count; ++k) {
        const int64_t *d = recs + 10 * k;
        prt_t *q = &P[k];
        q->patch = (int32_t)d[0];
        q->bucket = (int32_t)d[1];
        q->kind = (int32_t)d[2];
        q->level = (int32_t)d[3];
        q->code = (int32_t)d[4];
        q->birth = d[5];
        q->ox = d[6];
        q->oy = d[7];
        q->src = (int32_t)d[8];
        q->slot = (int32_t)d[9];
        if (q->patch < 0 || q->patch >= o->np || q->bucket < 0 || q->bucket >= o->nb || q->code < 0 ||
            q->code >= NCODE || q->birth > n || q->kind < 0 || q->kind > 2 ||
            (q->kind >= 1 && (q->src < 0 || q->src >= o->ns))) {
            free(P);
            return fail(o, "record out of range");
        }
    }
    free(o->P);
    o->P = P;
    o->nP = count;
    o->capP = count > 0 ? count : 1;
    o->n = n;
    o->stepped = 1;
    update_windows(o, n);
    rebuild_hist(o);
    return 0;
}

int orc_splat(orc_ocean *o, int32_t p, const int64_t *recs, int64_t n, double *raw) {
    if (p < 0 || p >= o->np) return fail(o, "patch out of range");
    const patch_t *pt = &o->pt[p];
    memset(raw, 0, sizeof(double) * (size_t)pt->nx * pt->ny);
    int64_t wmax = pt->nx > pt->ny ? pt->nx : pt->ny;
    double *wxv = (double *)malloc(sizeof(double) * (size_t)(wmax + 8));
    double *wyv = (double *)malloc(sizeof(double) * (size_t)(wmax + 8));
    prt_t *keep = (prt_t *)malloc(sizeof(prt_t) * (size_t)(n > 0 ? n : 1));
    int64_t nk = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t *d = recs + 10 * k;
        prt_t q;
        q.patch = (int32_t)d[0];
        q.bucket = (int32_t)d[1];
        q.kind = (int32_t)d[2];
        q.level = (int32_t)d[3];
        q.code = (int32_t)d[4];
        q.birth = d[5];
        q.ox = d[6];
        q.oy = d[7];
        q.src = (int32_t)d[8];
        q.slot = (int32_t)d[9];
        if (q.patch != p || q.bucket < 0 || q.bucket >= o->nb || q.code < 0 || q.code >= NCODE) continue;
        if (q.kind < 0 || q.kind > 2 || (q.kind >= 1 && (q.src < 0 || q.src >= o->ns))) continue;
        if (o->synth == 1) keep[nk++] = q;
        else splat_particle(o, pt, raw, &q, wxv, wyv);
    }
    if (o->synth == 1) layer_synth(o, pt, raw, keep, nk, p);
    free(keep);
    free(wxv);
    free(wyv);
    return 0;
}

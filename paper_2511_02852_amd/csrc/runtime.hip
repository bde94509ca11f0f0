// runtime.hip -- host side of the hybrid-ocean library: the C ABI of
// include/hwo.h, the FP64 setup tables, device memory, launch sequencing and
// hipGraph replay of a frame.
//
// Setup tables (built once, in FP64, on the host; integer ones are exact):
//   spectrum   Eq 2-4 (alpha, w_p, gamma), Eq 5-6 spreading
//   buckets    log-spaced wavelength edges or the equal-energy partition of
//              [0.5 w_p, 2.5 w_p], w_i = geometric mean of the edge
//              frequencies, r_i = pi g / w_i^2, c_i = g / w_i (Sec 3.2)
//   directions 64 bins, integer weights round(Dir dtheta 2^30) (times the
//              side pair's |cos| when obliquity-weighted), codes in units
//              of 2 pi / 10368; CDF by a wave64 scan on the GPU; for
//              stratified groups the factor sqrt(2 pi Dir) per code
//   velocity   round(c_i dt (cos, sin) 2^32) per code, int32
//   rates      round(eta 4 L dt w_i^3 / (pi^3 g) kappa 2^32) per side pair
//              (Eq 18; kappa = 1, or the pair's mean obliquity)
//   amplitude  sqrt(2 S_J(w_i) dw_i / eta) (Eq 7, importance-sampled)
//   sources    closest-radius bucket, ring offsets / multipliers, emission
//              cadence, crest volume = swept volume, subdivision ages
// h0(k) and the FFT twiddles are generated on the GPU in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hwo.h"
#include "hwo_dev.h"

using namespace hwo;

namespace {

constexpr double kUnit = 1048576.0;
constexpr double kTwo32 = 4294967296.0;
constexpr double kTwo30 = 1073741824.0;
constexpr int kStages = 14;
enum { ST_PARAMS = 0, ST_FFT_A, ST_FFT_B, ST_COUNT, ST_SCAN, ST_SCATTER, ST_SPLAT, ST_PLAN, ST_REDUCE, ST_BINPLAN,
       ST_DEPX, ST_FILTY, ST_LSUM, ST_NORMALS };

int64_t pmod(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}
int64_t ipow3(int k) {
  int64_t v = 1;
  for (int i = 0; i < k; ++i) v *= 3;
  return v;
}

struct TimedLaunch {
  int stage;
  hipEvent_t a, b;
};

}  // namespace

struct hwo_ocean {
  hwo_config cfg{};
  hwo_spectrum sp{};
  bool have_spec = false, finalized = false;
  std::vector<hwo_patch> patches;
  std::vector<hwo_source> sources;
  std::vector<int32_t> bin_cells;
  // spectrum / buckets
  double alpha = 0, wp = 0, gamma = 0;
  int nb = 0, lmax = 0;
  double w[kMaxBuckets], dw[kMaxBuckets], r[kMaxBuckets], c[kMaxBuckets];
  int32_t margin[kMaxBuckets];
  std::vector<uint32_t> qw;        // [nb][side pair][64]
  double kappa[kMaxBuckets][2];    // flux factor per side pair (1: the paper's count)
  std::vector<int32_t> codes;      // [64]
  int32_t wind_code = 0;           // wind direction in direction-code units
  std::vector<float> afac;         // [nb][kNCode] sqrt(2 pi Dir); stratified directions only
  // texel-layer synthesis tables
  std::vector<float> taps;         // 2R+1 raised-cosine taps per (patch, bucket)
  std::vector<int32_t> xt_base;    // first x tile per (patch, bucket), np*nb+1
  std::vector<int2> toff;          // [nb][kNCode] trough offsets (units)
  int64_t lt_total = 0;
  int32_t max_R = 0;
  std::vector<int2> V;             // [nb][kNCode]
  std::vector<float2> UC;          // [kNCode]
  // scene tables
  std::vector<PatchDev> pdev;
  std::vector<SourceDev> sdev;
  std::vector<float> ring_m;
  std::vector<float> ring_amp;     // [ns][kMaxRing] B_s m_s[j] (FP32 product, as on the device)
  std::vector<int2> ring_O;
  std::vector<int32_t> src_order;
  // device
  hipStream_t st = nullptr;
  bool own_stream = false;
  int device = 0;                  // device current when the stream was set up
  void *scratch = nullptr;         // that device's static probe staging (see probe_scratch)
  std::string scratch_err;         // why the scratch address could not be had, if so
  Dev dev{};
  std::vector<void *> allocs;
  float2 *h0T = nullptr, *tw = nullptr;
  uint32_t *cdf = nullptr, *cdfQ = nullptr;
  int update_grid = 1024;           // persistent grid of the counting pass (one round of resident blocks)
  int scatter_grid = 1024;          // and of the scatter pass
  int target_blocks = 1024;        // resident splat blocks the persistent grid aims for
  int splat_grid = 0;              // persistent splat blocks launched (0: four times target_blocks)
  int items_target = 4096;          // splat work items per frame the plan aims for (beyond one per tile; set per scene)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // batched form: the background FFT runs on a second branch of the frame
  // graph, joined before the splat (which blends with it)
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool capturing = false;
  bool fused = false;              // one-block scan + estimates + plan (small scenes)
  // timing
  bool timing = false;
  std::vector<TimedLaunch> tl;
  double stage_ms[kStages] = {0};
  int64_t stage_n[kStages] = {0};
  int64_t n_host = 0;
  std::string err;

  int fail(int code, const std::string &m) {
    err = m;
    return code;
  }
  int hip_fail(hipError_t e, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return HWO_EDEVICE;
  }
  void *alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (cfg.dev_alloc) {
      p = cfg.dev_alloc(bytes, cfg.alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
    if (p) allocs.push_back(p);
    return p;
  }
  void release_all() {
    for (void *p : allocs) {
      if (cfg.dev_alloc) {
        if (cfg.dev_free) cfg.dev_free(p, cfg.alloc_ctx);
      } else {
        (void)hipFree(p);
      }
    }
    allocs.clear();
  }
};

#define HWO_CHECK(expr)                                   \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return o->hip_fail(e_, #expr);  \
  } while (0)

// ---------------------------------------------------------------- static scratch
// Staging memory of hwo_sample_probes_static, for callers that cannot
// allocate: probe positions in the first half, results in the second.  Each
// GPU holds its own copy of this array for the life of the process; its
// address on a device comes from hipGetSymbolAddress with that device
// current (the array's name is not a device address in host code).  Every
// handle on one GPU shares that GPU's copy.
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr int64_t kScratchProbes = (int64_t)(kScratchBytes / 2 / 16);   // 16 B in and 16 B out per probe
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kScratchDevices] = {};

// Device address of the current device's scratch, looked up once per device.
static hipError_t probe_scratch(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------- spectrum
static double jonswap_h(const hwo_ocean *o, double w) {
  if (w <= 0.0) return 0.0;
  double sigma = (w <= o->wp) ? 0.07 : 0.09;
  double d = w - o->wp;
  double r = exp(-(d * d) / (2.0 * sigma * sigma * o->wp * o->wp));
  double x = o->wp / w;
  double x4 = x * x * x * x;
  return o->alpha * o->cfg.g * o->cfg.g * pow(w, -5.0) * exp(-1.25 * x4) * pow(o->gamma, r);
}

// Equal-energy partition of [0.5 w_p, 2.5 w_p] into n buckets (Sec 3.3):
// ascending edges with equal integrals of S_J between neighbours.  The
// cumulative integral is composite Simpson over 65536 panels; an edge is
// placed by linear interpolation of the cumulative integral inside the panel
// that contains its target.
static void equal_energy_edges(const hwo_ocean *o, int n, double *e) {
  const int K = 65536;
  const double a = 0.5 * o->wp, b = 2.5 * o->wp, h = (b - a) / (double)K;
  std::vector<double> C((size_t)K + 1);
  C[0] = 0.0;
  for (int k = 0; k < K; ++k) {
    const double x = a + (double)k * h;
    C[k + 1] = C[k] + h / 6.0 * (jonswap_h(o, x) + 4.0 * jonswap_h(o, x + 0.5 * h) + jonswap_h(o, x + h));
  }
  e[0] = a;
  e[n] = b;
  int k = 0;
  for (int i = 1; i < n; ++i) {
    const double tau = C[K] * (double)i / (double)n;
    while (k < K - 1 && C[k + 1] <= tau) ++k;
    e[i] = a + (double)k * h + h * ((tau - C[k]) / (C[k + 1] - C[k]));
  }
}

static double spread_h(const hwo_ocean *o, double w) {
  if (o->sp.spread_s >= 0.0) return o->sp.spread_s;
  double mu = (w <= o->wp) ? 5.0 : -2.5;
  return 16.0 * pow(w / o->wp, mu);
}

static double dir_h(double s, double theta) {
  double norm = tgamma(s + 1.0) / (2.0 * sqrt(M_PI) * tgamma(s + 0.5));
  double cth = cos(0.5 * theta);
  if (cth < 0.0) cth = -cth;
  return norm * pow(cth, 2.0 * s);
}

extern "C" {

int hwo_create_ocean(const hwo_config *cfg, hwo_ocean **out) {
  if (!cfg || !out) return HWO_EINVAL;
  *out = nullptr;
  const int N = cfg->fft_n;
  if (N < 16 || N > 4096 || (N & (N - 1)) != 0) return HWO_EINVAL;
  if (!(cfg->fft_L > 0) || !(cfg->g > 0) || !(cfg->dt > 0)) return HWO_EINVAL;
  if (cfg->max_particles < 0 || cfg->max_particles > ((int64_t)1 << 30)) return HWO_EINVAL;
  if (cfg->synth != 0 && cfg->synth != 1) return HWO_EINVAL;
  if (cfg->normals != 0 && cfg->normals != 1) return HWO_EINVAL;
  if (cfg->bg_fields != 0 && cfg->bg_fields != 1) return HWO_EINVAL;
  if (cfg->kernel != 0 && cfg->kernel != 1) return HWO_EINVAL;
  if (cfg->kernel == 1 && cfg->synth != 0) return HWO_EINVAL;
  if (cfg->fft_mfma16 != 0 && cfg->fft_mfma16 != 1) return HWO_EINVAL;
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return HWO_EINVAL;
  hwo_ocean *o = new hwo_ocean();
  o->cfg = *cfg;
  *out = o;
  return HWO_OK;
}

void hwo_destroy_ocean(hwo_ocean *o) {
  if (!o) return;
  if (o->st) (void)hipStreamSynchronize(o->st);
  if (o->exec) (void)hipGraphExecDestroy(o->exec);
  if (o->graph) (void)hipGraphDestroy(o->graph);
  if (o->ev_fork) (void)hipEventDestroy(o->ev_fork);
  if (o->ev_join) (void)hipEventDestroy(o->ev_join);
  if (o->st2) (void)hipStreamDestroy(o->st2);
  for (auto &t : o->tl) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  o->release_all();
  if (o->own_stream && o->st) (void)hipStreamDestroy(o->st);
  delete o;
}

const char *hwo_last_error(const hwo_ocean *o) { return o ? o->err.c_str() : "null handle"; }

int hwo_set_spectrum(hwo_ocean *o, const hwo_spectrum *sp) {
  if (!o || !sp) return HWO_EINVAL;
  if (o->have_spec) return o->fail(HWO_ESTATE, "spectrum already set");
  if (!(sp->U10 > 0) || !(sp->fetch > 0)) return o->fail(HWO_EINVAL, "U10 and fetch must be positive");
  if (sp->n_buckets < 1 || sp->n_buckets > kMaxBuckets) return o->fail(HWO_EINVAL, "n_buckets out of range");
  if (sp->bucket_mode != 0 && sp->bucket_mode != 1) return o->fail(HWO_EINVAL, "bucket_mode must be 0 or 1");
  if (sp->dir_mode != 0 && sp->dir_mode != 1) return o->fail(HWO_EINVAL, "dir_mode must be 0 or 1");
  if (sp->flux_mode != 0 && sp->flux_mode != 1) return o->fail(HWO_EINVAL, "flux_mode must be 0 or 1");
  if (sp->flux_mode == 1 && sp->dir_mode != 0)
    return o->fail(HWO_EINVAL, "obliquity-weighted injection needs dir_mode 0");
  if (sp->bucket_mode == 0 && (!(sp->lambda_min > 0) || !(sp->lambda_max > sp->lambda_min)))
    return o->fail(HWO_EINVAL, "bad lambda range");
  if (!(sp->eta > 0)) return o->fail(HWO_EINVAL, "eta must be positive");
  if (sp->max_level < 0 || sp->max_level > kMaxLevel) return o->fail(HWO_EINVAL, "max_level out of range");
  if (!(sp->subdiv_frac > 0)) return o->fail(HWO_EINVAL, "subdiv_frac must be positive");
  if (sp->h0_mode != 0 && sp->h0_mode != 1) return o->fail(HWO_EINVAL, "h0_mode must be 0 or 1");
  const double g = o->cfg.g, dt = o->cfg.dt;
  const double U10 = sp->U10, fetch = sp->fetch;
  o->sp = *sp;
  o->nb = sp->n_buckets;
  o->lmax = sp->max_level;
  // Eq 4
  o->alpha = 0.076 * pow(U10 * U10 / (fetch * g), 0.22);
  o->wp = 22.0 * pow(g * g / (U10 * fetch), 1.0 / 3.0);
  o->gamma = (sp->gamma > 0.0) ? sp->gamma : 7.0 * pow(g * fetch / (U10 * U10), -0.142);
  // buckets: edge frequencies descending (bucket 0 holds the shortest waves)
  double we[kMaxBuckets + 1];
  if (sp->bucket_mode == 0) {
    for (int j = 0; j <= o->nb; ++j) {
      double le = sp->lambda_min * pow(sp->lambda_max / sp->lambda_min, (double)j / (double)o->nb);
      we[j] = sqrt(2.0 * M_PI * g / le);
    }
  } else {
    double e[kMaxBuckets + 1];
    equal_energy_edges(o, o->nb, e);
    for (int j = 0; j <= o->nb; ++j) we[j] = e[o->nb - j];
  }
  for (int i = 0; i < o->nb; ++i) {
    double w = sqrt(we[i] * we[i + 1]);
    o->w[i] = w;
    o->dw[i] = we[i] - we[i + 1];
    o->r[i] = M_PI * g / (w * w);
    o->c[i] = g / w;
    o->margin[i] = (int32_t)ceil(2.0 * o->r[i] * kUnit);
    if (o->c[i] * dt >= 0.5) return o->fail(HWO_EINVAL, "bucket speed too high for the fixed-point step");
    if (2.0 * o->r[i] * kUnit > 1.0e9) return o->fail(HWO_EINVAL, "bucket radius too large");
  }
  // direction codes and integer weights
  const int wind_code = (int)pmod(llround(sp->wind_dir * (double)kNCode / (2.0 * M_PI)), kNCode);
  o->codes.resize(kDirBins);
  for (int b = 0; b < kDirBins; ++b)
    o->codes[b] = (int32_t)pmod((int64_t)wind_code + kNCode / 2 + (int64_t)(2 * b + 1) * (kNCode / (2 * kDirBins)),
                                kNCode);
  // One table per side pair (0: the sides normal to x).  Obliquity weighting
  // lets a wave heading phi cross the x sides at the rate c |cos phi| (|sin phi|
  // for y): that pair's directions follow Dir |cos phi| and its group count is
  // scaled by kappa, the mean of |cos phi| under Dir.
  o->qw.assign((size_t)o->nb * 2 * kDirBins, 0);
  const double dth = 2.0 * M_PI / (double)kDirBins;
  for (int i = 0; i < o->nb; ++i) {
    double s = spread_h(o, o->w[i]);
    for (int pair = 0; pair < 2; ++pair) {
      int64_t tot = 0;
      double num = 0.0, den = 0.0;
      for (int b = 0; b < kDirBins; ++b) {
        double th = -M_PI + ((double)b + 0.5) * dth;
        double dv = dir_h(s, th);
        double phi = 2.0 * M_PI * (double)o->codes[b] / (double)kNCode;
        double ob = fabs(pair == 0 ? cos(phi) : sin(phi));
        num += dv * ob;
        den += dv;
        int64_t qb = llround((sp->flux_mode ? dv * ob : dv) * dth * kTwo30);
        o->qw[((size_t)i * 2 + pair) * kDirBins + b] = (uint32_t)qb;
        tot += qb;
      }
      o->kappa[i][pair] = sp->flux_mode ? num / den : 1.0;
      if (tot <= 0 || tot >= ((int64_t)1 << 32)) return o->fail(HWO_EINVAL, "degenerate direction distribution");
    }
  }
  o->wind_code = wind_code;
  // Stratified directions: a particle of bucket i heading along theta carries
  // A_i * sqrt(2 pi Dir(theta - wind)), so that over a group of N_theta equal
  // sectors its squared amplitude sums to the bucket's share S(w_i) dw_i (Eq 7
  // with dtheta = 2 pi / N_theta).
  o->afac.clear();
  if (sp->dir_mode == 1) {
    o->afac.resize((size_t)o->nb * kNCode);
    for (int i = 0; i < o->nb; ++i) {
      double s = spread_h(o, o->w[i]);
      for (int code = 0; code < kNCode; ++code) {
        double th = 2.0 * M_PI * (double)code / (double)kNCode - sp->wind_dir;
        o->afac[(size_t)i * kNCode + code] = (float)sqrt(2.0 * M_PI * dir_h(s, th));
      }
    }
  }
  // velocity per step and unit vectors
  o->V.resize((size_t)o->nb * kNCode);
  o->UC.resize(kNCode);
  for (int code = 0; code < kNCode; ++code) {
    double ang = 2.0 * M_PI * (double)code / (double)kNCode;
    o->UC[code] = make_float2((float)cos(ang), (float)sin(ang));
  }
  for (int i = 0; i < o->nb; ++i) {
    double cdt = o->c[i] * dt;
    for (int code = 0; code < kNCode; ++code) {
      double ang = 2.0 * M_PI * (double)code / (double)kNCode;
      int64_t vx = llround(cdt * cos(ang) * kTwo32);
      int64_t vy = llround(cdt * sin(ang) * kTwo32);
      o->V[(size_t)i * kNCode + code] = make_int2((int32_t)vx, (int32_t)vy);
    }
  }
  // stream, h0, twiddles, CDF
  if (o->cfg.stream) {
    o->st = (hipStream_t)o->cfg.stream;
  } else {
    HWO_CHECK(hipStreamCreateWithFlags(&o->st, hipStreamNonBlocking));
    o->own_stream = true;
  }
  HWO_CHECK(hipGetDevice(&o->device));
  {
    // only hwo_sample_probes_static needs it; it reports a failure here
    const hipError_t e = probe_scratch(o->device, &o->scratch);
    if (e != hipSuccess) o->scratch_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
  }
  const int N = o->cfg.fft_n;
  o->h0T = (float2 *)o->alloc(sizeof(float2) * (size_t)N * N);
  o->tw = (float2 *)o->alloc(sizeof(float2) * (size_t)N);
  uint32_t *qd = (uint32_t *)o->alloc(sizeof(uint32_t) * o->qw.size());
  o->cdf = (uint32_t *)o->alloc(sizeof(uint32_t) * o->qw.size());
  o->cdfQ = (uint32_t *)o->alloc(sizeof(uint32_t) * (size_t)o->nb * 2);
  if (!o->h0T || !o->tw || !qd || !o->cdf || !o->cdfQ) return o->fail(HWO_ENOMEM, "device allocation failed");
  Dev d{};
  d.N = N;
  d.L = o->cfg.fft_L;
  d.g = g;
  d.nb = o->nb;
  d.seed = o->cfg.seed;
  launch_h0(d, o->h0T, o->tw, o->alpha, o->wp, o->gamma, sp->spread_s, sp->wind_dir, sp->h0_mode, o->st);
  HWO_CHECK(hipGetLastError());
  HWO_CHECK(hipMemcpyAsync(qd, o->qw.data(), sizeof(uint32_t) * o->qw.size(), hipMemcpyHostToDevice, o->st));
  launch_cdf(d, qd, o->cdf, o->cdfQ, o->st);
  HWO_CHECK(hipGetLastError());
  HWO_CHECK(hipStreamSynchronize(o->st));
  o->have_spec = true;
  return HWO_OK;
}

int hwo_add_patch(hwo_ocean *o, const hwo_patch *p, int32_t *id) {
  if (!o || !p) return HWO_EINVAL;
  if (!o->have_spec) return o->fail(HWO_ESTATE, "set_spectrum first");
  if (o->finalized) return o->fail(HWO_ESTATE, "scene is fixed after the first step");
  if ((int)o->patches.size() >= kMaxPatches) return o->fail(HWO_ERANGE, "too many patches");
  if (p->nx < 1 || p->ny < 1 || p->nx > 4096 || p->ny > 4096 || !(p->dx > 0))
    return o->fail(HWO_EINVAL, "bad patch size");
  const double dxu = p->dx * kUnit;
  if (dxu != floor(dxu) || ((int64_t)dxu) % 2 != 0 || dxu > 1.0e8)
    return o->fail(HWO_EINVAL, "dx must be an even multiple of 2^-20 m");
  if ((double)p->nx * dxu > 1.5e9 || (double)p->ny * dxu > 1.5e9) return o->fail(HWO_EINVAL, "patch too large");
  if (p->follow < -1) return o->fail(HWO_EINVAL, "bad follow id");
  const double eta = (p->eta > 0.0) ? p->eta : o->sp.eta;
  if (o->sp.dir_mode == 1 && (eta != floor(eta) || eta > (double)kNCode))
    return o->fail(HWO_EINVAL, "stratified directions need a whole number of particles per group");
  if (id) *id = (int32_t)o->patches.size();
  o->patches.push_back(*p);
  return HWO_OK;
}

int hwo_add_source(hwo_ocean *o, const hwo_source *s, int32_t *id) {
  if (!o || !s) return HWO_EINVAL;
  if (!o->have_spec) return o->fail(HWO_ESTATE, "set_spectrum first");
  if (o->finalized) return o->fail(HWO_ESTATE, "scene is fixed after the first step");
  if ((int)o->sources.size() >= kMaxSources) return o->fail(HWO_ERANGE, "too many sources");
  if (s->patch < 0 || s->patch >= (int)o->patches.size()) return o->fail(HWO_EINVAL, "source patch out of range");
  if (!(s->radius > 0) || !(s->draft >= 0)) return o->fail(HWO_EINVAL, "bad source radius/draft");
  if (s->ring_n < 1 || s->ring_n > kMaxRing || 128 % s->ring_n != 0)
    return o->fail(HWO_EINVAL, "ring_n must divide 128");
  if (!(s->heave_amp >= 0) || (s->heave_amp > 0 && !(s->heave_period > 0)))
    return o->fail(HWO_EINVAL, "bad heave amplitude/period");
  if (id) *id = (int32_t)o->sources.size();
  o->sources.push_back(*s);
  return HWO_OK;
}

int hwo_set_bins(hwo_ocean *o, const int32_t *bin_cells, int32_t n) {
  if (!o || !bin_cells) return HWO_EINVAL;
  if (!o->have_spec) return o->fail(HWO_ESTATE, "set_spectrum first");
  if (o->finalized) return o->fail(HWO_ESTATE, "bins are fixed after the first step");
  if (n != o->nb) return o->fail(HWO_EINVAL, "need one bin size per bucket");
  for (int i = 0; i < n; ++i)
    if (bin_cells[i] < 1 || bin_cells[i] > 4096) return o->fail(HWO_EINVAL, "bin size out of range");
  o->bin_cells.assign(bin_cells, bin_cells + n);
  return HWO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- finalize
static int build_scene_tables(hwo_ocean *o) {
  const double g = o->cfg.g, dt = o->cfg.dt;
  const int np = (int)o->patches.size(), ns = (int)o->sources.size(), nb = o->nb;
  if (o->bin_cells.empty()) o->bin_cells.assign(nb, 16);
  for (int p = 0; p < np; ++p)
    if (o->patches[p].follow >= ns) return o->fail(HWO_EINVAL, "patch follows a missing source");
  // sources sorted by patch (stable)
  o->src_order.resize(ns);
  for (int s = 0; s < ns; ++s) o->src_order[s] = s;
  std::stable_sort(o->src_order.begin(), o->src_order.end(),
                   [&](int a, int b) { return o->sources[a].patch < o->sources[b].patch; });
  o->pdev.assign(np, PatchDev{});
  int64_t bins = 0, tiles = 0, cells = 0;
  const bool layers = o->cfg.synth == 1;
  o->taps.clear();
  o->xt_base.clear();
  o->lt_total = 0;
  o->max_R = 0;
  int64_t xtiles = 0;
  const double dxf = o->cfg.fft_L / (double)o->cfg.fft_n;
  for (int p = 0; p < np; ++p) {
    const hwo_patch &hp = o->patches[p];
    PatchDev &P = o->pdev[p];
    P.ax = hp.anchor_x;
    P.ay = hp.anchor_y;
    P.dx = hp.dx;
    P.nx = hp.nx;
    P.ny = hp.ny;
    P.dxu = (int32_t)(hp.dx * kUnit);
    P.follow = hp.follow;
    const double eta = (hp.eta > 0.0) ? hp.eta : o->sp.eta;
    if (o->sp.dir_mode == 1 && (eta != floor(eta) || eta > (double)kNCode))
      return o->fail(HWO_EINVAL, "stratified directions need a whole number of particles per group");
    P.ntheta = (int32_t)eta;
    const double rmax = o->r[nb - 1];
    const double lmin = (double)(hp.nx < hp.ny ? hp.nx : hp.ny) * hp.dx / 4.0;
    P.band = (float)((hp.blend_band > 0.0) ? hp.blend_band : (rmax < lmin ? rmax : lmin));
    P.inv_band = 1.0f / P.band;
    P.ratio = (float)(hp.dx / dxf);
    const double Lx = (double)hp.nx * hp.dx, Ly = (double)hp.ny * hp.dx;
    P.bin_lo = (int32_t)bins;
    for (int i = 0; i < nb; ++i) {
      const double w = o->w[i];
      P.A[i] = (float)sqrt(2.0 * jonswap_h(o, w) * o->dw[i] / eta);
      const double gx = 4.0 * Ly * dt * w * w * w / (M_PI * M_PI * M_PI * g);
      const double gy = 4.0 * Lx * dt * w * w * w / (M_PI * M_PI * M_PI * g);
      P.Rx[i] = (uint64_t)llround(eta * gx * o->kappa[i][0] * kTwo32);
      P.Ry[i] = (uint64_t)llround(eta * gy * o->kappa[i][1] * kTwo32);
      if (P.Rx[i] > ((uint64_t)1 << 52) || P.Ry[i] > ((uint64_t)1 << 52))
        return o->fail(HWO_EINVAL, "injection rate too high");
      const int64_t binu = (int64_t)o->bin_cells[i] * P.dxu;
      if (binu >= ((int64_t)1 << 31)) return o->fail(HWO_EINVAL, "bin too large");
      P.binu[i] = (int32_t)binu;
      // division by the bin edge as a multiplication (exact for every 32-bit
      // dividend: Lemire, Kaser and Kurz, "Faster remainder by direct
      // computation", 2019); binu >= 2 here
      P.binm[i] = UINT64_MAX / (uint64_t)binu + 1;
      const int64_t m = o->margin[i];
      // a live particle lies within the window plus the margin, so its offset
      // from any cell of the patch is below nx dxu + m, which the splat forms
      // in 32 bits
      if ((int64_t)std::max(hp.nx, hp.ny) * P.dxu + m >= ((int64_t)1 << 31))
        return o->fail(HWO_EINVAL, "patch plus the bucket's survival margin exceed 2^31 position units");
      P.nbx[i] = (int32_t)(floor_div((int64_t)hp.nx * P.dxu + 2 * m, binu) + 1);
      P.nby[i] = (int32_t)(floor_div((int64_t)hp.ny * P.dxu + 2 * m, binu) + 1);
      P.binbase[i] = (int32_t)bins;
      bins += (int64_t)P.nbx[i] * P.nby[i];
      // a 64-cell splat tile must reach its crests through at most 32 bin rows
      if ((63 * (int64_t)P.dxu + 2 * m) / binu + 2 > 32)
        return o->fail(HWO_EINVAL, "bin edge too small for the bucket radius (a tile would need > 32 bin rows)");
      if (bins > ((int64_t)1 << 28)) return o->fail(HWO_EINVAL, "too many bins");
      if (layers) {
        // layer = patch + R cells each side, R = ceil(r / dx) - 1 (taps w(k dx) > 0 for |k| <= R)
        const int64_t Rl = std::max<int64_t>(0, (int64_t)ceil(o->r[i] / hp.dx) - 1);
        if (Rl > 2048) return o->fail(HWO_EINVAL, "bucket radius too large for texel layers");
        P.lay_R[i] = (int32_t)Rl;
        P.lt_off[i] = o->lt_total;
        P.tap_off[i] = (int32_t)o->taps.size();
        o->lt_total += (int64_t)hp.nx * ((int64_t)hp.ny + 2 * Rl);
        for (int64_t k = -Rl; k <= Rl; ++k) {
          const double dk = (double)k * hp.dx;
          o->taps.push_back((float)(fabs(dk) >= o->r[i] ? 0.0 : 0.5 * (1.0 + cos(M_PI * dk / o->r[i]))));
        }
        o->xt_base.push_back((int32_t)xtiles);
        xtiles += (((int64_t)hp.ny + 2 * Rl + kTile - 1) / kTile) * (((int64_t)hp.nx + kTile - 1) / kTile);
        o->max_R = std::max(o->max_R, (int32_t)Rl);
        if (xtiles > ((int64_t)1 << 30) || o->lt_total > ((int64_t)1 << 34))
          return o->fail(HWO_EINVAL, "texel layers too large");
      }
    }
    P.bin_hi = (int32_t)bins;
    P.ntx = (hp.nx + kTile - 1) / kTile;
    P.nty = (hp.ny + kTile - 1) / kTile;
    P.tile0 = (int32_t)tiles;
    tiles += (int64_t)P.ntx * P.nty;
    if (tiles > ((int64_t)1 << 19)) return o->fail(HWO_EINVAL, "too many output tiles");
    P.cell0 = cells;
    cells += (int64_t)hp.nx * hp.ny;
  }
  if (layers) o->xt_base.push_back((int32_t)xtiles);
  // source ranges per patch in sorted order
  for (int p = 0; p < np; ++p) {
    int lo = 0;
    while (lo < ns && o->sources[o->src_order[lo]].patch < p) ++lo;
    int hi = lo;
    while (hi < ns && o->sources[o->src_order[hi]].patch == p) ++hi;
    o->pdev[p].src_lo = lo;
    o->pdev[p].src_hi = hi;
  }
  o->sdev.assign(ns, SourceDev{});
  o->ring_m.clear();
  o->ring_amp.assign((size_t)std::max(ns, 1) * kMaxRing, 0.f);
  o->ring_O.clear();
  for (int si = 0; si < ns; ++si) {
    const hwo_source &hs = o->sources[si];
    SourceDev &S = o->sdev[si];
    S.x0 = hs.x0;
    S.y0 = hs.y0;
    S.vx = hs.vx;
    S.vy = hs.vy;
    S.patch = hs.patch;
    S.ne = hs.ring_n;
    S.a0 = kNCode / hs.ring_n;
    S.ring0 = (int32_t)o->ring_m.size();
    const double R = hs.radius;
    const double speed = sqrt(hs.vx * hs.vx + hs.vy * hs.vy);
    const double heading = atan2(hs.vy, hs.vx);
    int best = 0;
    for (int i = 1; i < nb; ++i)
      if (fabs(o->r[i] - R) < fabs(o->r[best] - R)) best = i;
    S.bucket = best;
    const double rb = o->r[best], cb = o->c[best];
    double sum_abs = 0.0;
    for (int j = 0; j < hs.ring_n; ++j) {
      const double phi = 2.0 * M_PI * (double)j / (double)hs.ring_n;
      const double m = cos(phi - heading);
      sum_abs += fabs(m);
      o->ring_m.push_back((float)m);
      const int64_t ox = llround(R * cos(phi) * kUnit), oy = llround(R * sin(phi) * kUnit);
      o->ring_O.push_back(make_int2((int32_t)ox, (int32_t)oy));
    }
    if (speed > 0.0) {
      const double e = floor(0.5 * rb / (speed * dt));
      const int64_t E = e < 1.0 ? 1 : (int64_t)e;
      S.E = (int32_t)std::min<int64_t>(E, 1 << 30);
      S.B = (float)(2.0 * R * speed * (double)E * dt * hs.draft / (rb * rb * sum_abs));
    } else {
      S.E = 0;
      S.B = 0.f;
    }
    for (int j = 0; j < hs.ring_n; ++j)
      o->ring_amp[(size_t)si * kMaxRing + j] = S.B * o->ring_m[(size_t)S.ring0 + j];
    // vertical motion: a ring each time the previous one has travelled half
    // a radius; its crests carry pi R^2 dz, shared by the n_e particles
    S.Eh = 0;
    S.Bh = 0.0;
    S.hf = 0.0;
    if (hs.heave_amp > 0.0) {
      const double e = floor(0.5 * rb / (cb * dt));
      S.Eh = e < 1.0 ? 1 : (int32_t)std::min(e, (double)(1 << 30));
      S.Bh = M_PI * R * R * hs.heave_amp / ((double)hs.ring_n * rb * rb);
      S.hf = dt / hs.heave_period;
    }
    for (int L = 0; L < kMaxLevel; ++L) {
      const double alpha = 2.0 * M_PI / ((double)hs.ring_n * (double)ipow3(L));
      const double x = (o->sp.subdiv_frac * rb / alpha - R) / (cb * dt);
      int64_t T = (int64_t)floor(x) + 1;
      if (T < 0) T = 0;
      S.T[L] = (int32_t)std::min<int64_t>(T, (int64_t)1 << 30);
    }
  }
  o->dev.nbins = (int32_t)bins;
  o->dev.ntiles = (int32_t)tiles;
  // particle capacity
  int64_t cap = o->cfg.max_particles;
  if (cap == 0) {
    double est = 0.0;
    for (int p = 0; p < np; ++p) {
      const hwo_patch &hp = o->patches[p];
      const double span = (double)std::max(hp.nx, hp.ny) * hp.dx;
      for (int i = 0; i < nb; ++i) {
        const double rate = (double)(o->pdev[p].Rx[i] + o->pdev[p].Ry[i]) / kTwo32;
        const double steps = std::min((1.5 * span + 4.0 * o->r[i]) / (o->c[i] * dt), 4096.0);
        est += rate * steps;
      }
    }
    for (int si = 0; si < ns; ++si) {
      const SourceDev &S = o->sdev[si];
      if (S.E <= 0) continue;
      const hwo_patch &hp = o->patches[S.patch];
      const double span = (double)std::max(hp.nx, hp.ny) * hp.dx;
      const double steps = std::min((span + 4.0 * o->r[S.bucket]) / (o->c[S.bucket] * dt), 4096.0);
      est += (double)S.ne * ipow3(o->lmax) * (steps / S.E + 1.0);
    }
    cap = (int64_t)(1.5 * est) + 65536;
    cap = std::min<int64_t>(cap, (int64_t)1 << 30);
  }
  o->dev.cap = (int32_t)cap;
  (void)cells;
  return HWO_OK;
}

template <class T>
static T *upload(hwo_ocean *o, const std::vector<T> &v, int *rc) {
  T *p = (T *)o->alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!p) {
    *rc = o->fail(HWO_ENOMEM, "device allocation failed");
    return nullptr;
  }
  if (!v.empty()) {
    hipError_t e = hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, o->st);
    if (e != hipSuccess) *rc = o->hip_fail(e, "upload");
  }
  return p;
}

static int finalize(hwo_ocean *o) {
  if (o->finalized) return HWO_OK;
  if (!o->have_spec) return o->fail(HWO_ESTATE, "set_spectrum first");
  int rc = build_scene_tables(o);
  if (rc) return rc;
  Dev &d = o->dev;
  const int np = (int)o->patches.size(), ns = (int)o->sources.size(), nb = o->nb, N = o->cfg.fft_n;
  d.np = np;
  d.ns = ns;
  d.nb = nb;
  d.N = N;
  d.compact = o->cfg.compact ? 1 : 0;
  d.fft_mfma16 = o->cfg.fft_mfma16 && N >= 1024 ? 1 : 0;
  d.lmax = o->lmax;
  d.n_inj_slots = np * nb * 2;
  d.g = o->cfg.g;
  d.dt = o->cfg.dt;
  d.L = o->cfg.fft_L;
  d.dxf = o->cfg.fft_L / (double)N;
  d.seed = o->cfg.seed;
  rc = HWO_OK;
  d.patches = upload(o, o->pdev, &rc);
  d.sources = upload(o, o->sdev, &rc);
  d.src_order = upload(o, o->src_order, &rc);
  d.V = upload(o, o->V, &rc);
  {
    std::vector<int2> vbin((size_t)nb * kDirBins);
    for (int i = 0; i < nb; ++i)
      for (int k = 0; k < kDirBins; ++k) vbin[(size_t)i * kDirBins + k] = o->V[(size_t)i * kNCode + o->codes[k]];
    d.Vbin = upload(o, vbin, &rc);
  }
  d.UC = upload(o, o->UC, &rc);
  d.cdf = o->cdf;
  d.cdfQ = o->cdfQ;
  d.codes = upload(o, o->codes, &rc);
  d.afac = o->afac.empty() ? nullptr : upload(o, o->afac, &rc);
  d.wind_code = o->wind_code;
  std::vector<float> br(nb);
  std::vector<int32_t> bm(nb);
  for (int i = 0; i < nb; ++i) {
    br[i] = (float)o->r[i];
    bm[i] = o->margin[i];
  }
  d.bucket_r = upload(o, br, &rc);
  d.margin = upload(o, bm, &rc);
  d.ring_m = upload(o, o->ring_m, &rc);
  d.ring_amp = upload(o, o->ring_amp, &rc);
  d.ring_O = upload(o, o->ring_O, &rc);
  if (rc) return rc;
  int64_t cells = 0;
  for (auto &hp : o->patches) cells += (int64_t)hp.nx * hp.ny;
  const size_t rec = d.compact ? sizeof(RecCompact) : sizeof(RecWide);
  d.glob = (Globals *)o->alloc(sizeof(Globals));
  d.sp = (StepPatch *)o->alloc(sizeof(StepPatch) * std::max(np, 1));
  d.sp_next = (StepPatch *)o->alloc(sizeof(StepPatch) * std::max(np, 1));
  d.inj_off = (int32_t *)o->alloc(sizeof(int32_t) * (d.n_inj_slots + 1));
  d.em_off = (int32_t *)o->alloc(sizeof(int32_t) * (ns + 1));
  d.src_pos = (int2 *)o->alloc(sizeof(int2) * std::max(ns, 1));
  d.ctr = (unsigned long long *)o->alloc(sizeof(unsigned long long) * (size_t)std::max(np * nb * CNT_NUM, 1));
  d.ctr_next = (unsigned long long *)o->alloc(sizeof(unsigned long long) * (size_t)std::max(np * nb * CNT_NUM, 1));
  d.hist = (int32_t *)o->alloc(sizeof(int32_t) * ((size_t)d.nbins + 1));
  d.off = (int32_t *)o->alloc(sizeof(int32_t) * ((size_t)d.nbins + 1));
  d.cur = (int32_t *)o->alloc(sizeof(int32_t) * ((size_t)d.nbins + 1));
  d.bsum = (int32_t *)o->alloc(sizeof(int32_t) * (size_t)std::max(scan_blocks(d.nbins), 1));
  d.S0 = o->alloc(rec * (size_t)d.cap);
  d.S1 = o->alloc(rec * (size_t)d.cap);
  d.h0T = o->h0T;
  d.tw = o->tw;
  d.nfields = o->cfg.bg_fields ? 5 : 1;   // height, or height + slopes + choppy displacements
  d.FT = (float2 *)o->alloc(sizeof(float2) * (size_t)(N / 2 + 1) * N * d.nfields);
  d.H = (float *)o->alloc(sizeof(float) * (size_t)N * N * d.nfields);
  d.raw = (float *)o->alloc(sizeof(float) * (size_t)std::max<int64_t>(cells, 1));
  d.blend = (float *)o->alloc(sizeof(float) * (size_t)std::max<int64_t>(cells, 1));
  d.ncells = cells;
  if (o->cfg.normals) {
    d.nrm = (float *)o->alloc(sizeof(float) * 3 * (size_t)std::max<int64_t>(cells, 1));
    if (!d.nrm) return o->fail(HWO_ENOMEM, "device allocation failed");
    HWO_CHECK(hipMemsetAsync(d.nrm, 0, sizeof(float) * 3 * (size_t)std::max<int64_t>(cells, 1), o->st));
  }
  // splat work plan
  d.max_items = d.ntiles + 8192;
  d.chunk_load = 3500;   // least estimated cost per work item (several hundred particle visits)
  d.splat_kernel = 2;    // hybrid schedule: batches for small footprints, quadrants for large ones
  // Items beyond one per tile: about 16 parts per tile on average, between
  // 1024 and 4096.  Every extra part writes a 16 KiB partial tile that the
  // reduce reads back, so scenes with few dense tiles do better with fewer,
  // larger parts, while scenes with thousands of tiles of uneven load need
  // the larger budget to cut their heavy tiles.
  o->items_target = std::min(4096, std::max(1024, 16 * d.ntiles));
  d.tile_load = (uint32_t *)o->alloc(sizeof(uint32_t) * (size_t)std::max(d.ntiles, 1));
  d.tile_meas = (uint32_t *)o->alloc(sizeof(uint32_t) * (size_t)std::max(d.ntiles, 1));
  d.tile_model = (uint32_t *)o->alloc(sizeof(uint32_t) * (size_t)std::max(d.ntiles, 1));
  d.tile_ratio = (float *)o->alloc(sizeof(float) * (size_t)std::max(d.ntiles, 1));
  d.item_base = (int32_t *)o->alloc(sizeof(int32_t) * ((size_t)d.ntiles + 1));
  d.splat_ctl = (int32_t *)o->alloc(sizeof(int32_t) * 4);
  d.split_tiles = (int32_t *)o->alloc(sizeof(int32_t) * (size_t)std::max(d.ntiles, 1));
  d.item_desc = (int4 *)o->alloc(sizeof(int4) * (size_t)d.max_items);
  {
    std::vector<int32_t> tp((size_t)std::max(d.ntiles, 1), 0);
    for (int p = 0; p < np; ++p)
      for (int t = 0; t < o->pdev[p].ntx * o->pdev[p].nty; ++t) tp[(size_t)o->pdev[p].tile0 + t] = p;
    d.tile_patch = upload(o, tp, &rc);
    if (rc) return rc;
    // Bin rectangle each (tile, bucket) reads: crests within 2 r of the
    // tile's cell centres, in bins anchored at the window origin minus 2 r.
    // Static, because bins move with the window.
    std::vector<short4> rect((size_t)std::max(d.ntiles, 1) * nb);
    for (int p = 0; p < np; ++p) {
      const PatchDev &P = o->pdev[p];
      for (int t = 0; t < P.ntx * P.nty; ++t) {
        const int i0 = (t % P.ntx) * kTile, j0 = (t / P.ntx) * kTile;
        const int tw = std::min(kTile, P.nx - i0), th = std::min(kTile, P.ny - j0);
        for (int b = 0; b < nb; ++b) {
          const int64_t m = o->margin[b], binu = P.binu[b];
          const int64_t ax0 = (int64_t)i0 * P.dxu + P.dxu / 2, ay0 = (int64_t)j0 * P.dxu + P.dxu / 2;
          const int bx_lo = (int)(ax0 / binu);
          const int bx_hi = (int)std::min<int64_t>(P.nbx[b] - 1, (ax0 + (int64_t)(tw - 1) * P.dxu + 2 * m) / binu);
          const int by_lo = (int)(ay0 / binu);
          const int by_hi = (int)std::min<int64_t>(P.nby[b] - 1, (ay0 + (int64_t)(th - 1) * P.dxu + 2 * m) / binu);
          const int nrows = (bx_lo <= bx_hi && by_lo <= by_hi) ? by_hi - by_lo + 1 : 0;
          if (nrows > 32 || bx_hi > 32767) return o->fail(HWO_EINVAL, "bin rectangle too large");
          rect[((size_t)P.tile0 + t) * nb + b] = make_short4((short)bx_lo, (short)bx_hi, (short)by_lo, (short)nrows);
        }
      }
    }
    d.tile_rect = upload(o, rect, &rc);
    if (rc) return rc;
  }
  if (!d.item_desc) return o->fail(HWO_ENOMEM, "device allocation failed");
  d.partials = (float *)o->alloc(sizeof(float) * (size_t)kTile * kTile * (size_t)d.max_items);
  d.synth = o->cfg.synth;
  d.radial = o->cfg.kernel;
  if (d.synth == 1 && np > 0) {
    d.n_xtiles = o->xt_base.back();
    // trough offsets round(r (cos, sin) 2^20): the texel a trough lands in is an integer decision
    o->toff.resize((size_t)nb * kNCode);
    for (int b = 0; b < nb; ++b)
      for (int code = 0; code < kNCode; ++code) {
        const double ang = 2.0 * M_PI * (double)code / (double)kNCode;
        o->toff[(size_t)b * kNCode + code] =
            make_int2((int32_t)llround(o->r[b] * cos(ang) * kUnit), (int32_t)llround(o->r[b] * sin(ang) * kUnit));
      }
    d.lt = (float *)o->alloc(sizeof(float) * (size_t)std::max<int64_t>(o->lt_total, 1));
    // heavy x tiles are cut into up to four parts; the partial tiles take
    // 64 KiB per x tile, so very large scenes keep one part per tile
    d.xparts = ((int64_t)d.n_xtiles * 4 * kTile * kTile * 4 <= ((int64_t)1 << 30)) ? 4 : 1;
    d.xt_nparts = (int32_t *)o->alloc(sizeof(int32_t) * (size_t)std::max(d.n_xtiles, 1));
    d.xpartial = (float *)o->alloc(sizeof(float) * (size_t)std::max(d.n_xtiles, 1) * d.xparts * kTile * kTile);
    if (!d.xt_nparts || !d.xpartial) return o->fail(HWO_ENOMEM, "device allocation failed");
    d.yplanes = (float *)o->alloc(sizeof(float) * (size_t)nb * (size_t)std::max<int64_t>(cells, 1));
    d.taps = upload(o, o->taps, &rc);
    d.xt_base = upload(o, o->xt_base, &rc);
    d.toff = upload(o, o->toff, &rc);
    if (rc) return rc;
    if (!d.lt || !d.yplanes) return o->fail(HWO_ENOMEM, "device allocation failed");
    // both passes stage (64 + 2R + 17) x 64 floats (the register-blocked FIR
    // reads up to 16 rows / columns past the strip, zero padded) and the taps
    // padded to a multiple of 16
    const int64_t ls = sizeof(float) * (((int64_t)kTile + 2 * o->max_R + 17) * kTile + 2 * o->max_R + 17);
    if (ls > 159 * 1024) return o->fail(HWO_EINVAL, "texel-layer passes do not fit in LDS (bucket radius too large)");   // 1 KiB for static LDS
    d.lsmem = (int32_t)ls;
    HWO_CHECK(prepare_layers(d));
    HWO_CHECK(hipMemsetAsync(d.lt, 0, sizeof(float) * (size_t)std::max<int64_t>(o->lt_total, 1), o->st));
    HWO_CHECK(hipMemsetAsync(d.xt_nparts, 0, sizeof(int32_t) * (size_t)std::max(d.n_xtiles, 1), o->st));
    HWO_CHECK(hipMemsetAsync(d.yplanes, 0, sizeof(float) * (size_t)nb * (size_t)std::max<int64_t>(cells, 1), o->st));
  }
  if (!d.tile_load || !d.tile_meas || !d.tile_model || !d.tile_ratio || !d.item_base || !d.splat_ctl ||
      !d.split_tiles || !d.partials)
    return o->fail(HWO_ENOMEM, "device allocation failed");
  if (!d.glob || !d.sp || !d.sp_next || !d.ctr_next || !d.inj_off || !d.em_off || !d.src_pos || !d.ctr || !d.hist ||
      !d.off || !d.cur ||
      !d.bsum || !d.S0 || !d.S1 || !d.FT || !d.H || !d.raw || !d.blend)
    return o->fail(HWO_ENOMEM, "device allocation failed");
  HWO_CHECK(hipMemsetAsync(d.glob, 0, sizeof(Globals), o->st));
  d.splat_prof = (unsigned long long *)o->alloc(sizeof(unsigned long long) * PROF_N);
  if (!d.splat_prof) return o->fail(HWO_ENOMEM, "device allocation failed");
  HWO_CHECK(hipMemsetAsync(d.splat_prof, 0, sizeof(unsigned long long) * PROF_N, o->st));
  HWO_CHECK(hipMemsetAsync(d.sp, 0, sizeof(StepPatch) * std::max(np, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.ctr, 0, sizeof(unsigned long long) * (size_t)std::max(np * nb * CNT_NUM, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.ctr_next, 0, sizeof(unsigned long long) * (size_t)std::max(np * nb * CNT_NUM, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.sp_next, 0, sizeof(StepPatch) * std::max(np, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.hist, 0, sizeof(int32_t) * ((size_t)d.nbins + 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.off, 0, sizeof(int32_t) * ((size_t)d.nbins + 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.cur, 0, sizeof(int32_t) * ((size_t)d.nbins + 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.raw, 0, sizeof(float) * (size_t)std::max<int64_t>(cells, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.blend, 0, sizeof(float) * (size_t)std::max<int64_t>(cells, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.H, 0, sizeof(float) * (size_t)N * N * d.nfields, o->st));
  HWO_CHECK(hipMemsetAsync(d.tile_load, 0, sizeof(uint32_t) * (size_t)std::max(d.ntiles, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.tile_meas, 0, sizeof(uint32_t) * (size_t)std::max(d.ntiles, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.tile_model, 0, sizeof(uint32_t) * (size_t)std::max(d.ntiles, 1), o->st));
  HWO_CHECK(hipMemsetD32Async((hipDeviceptr_t)d.tile_ratio, 0x3F800000, (size_t)std::max(d.ntiles, 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.item_base, 0, sizeof(int32_t) * ((size_t)d.ntiles + 1), o->st));
  HWO_CHECK(hipMemsetAsync(d.splat_ctl, 0, sizeof(int32_t) * 4, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  int dev_id = 0, cus = 256;
  (void)hipGetDevice(&dev_id);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id);
  o->update_grid = std::max(64, update_blocks_per_cu(d.compact, false) * cus);
  o->scatter_grid = std::max(64, update_blocks_per_cu(d.compact, true) * cus);
  o->target_blocks = std::max(64, 4 * cus);
  if (o->cfg.batched) {
    o->fused = bin_plan_fits(d.nbins, d.ntiles, d.nb);
    HWO_CHECK(hipStreamCreateWithFlags(&o->st2, hipStreamNonBlocking));
    HWO_CHECK(hipEventCreateWithFlags(&o->ev_fork, hipEventDisableTiming));
    HWO_CHECK(hipEventCreateWithFlags(&o->ev_join, hipEventDisableTiming));
  }
  o->finalized = true;
  return HWO_OK;
}

// ---------------------------------------------------------------- stepping
struct PatchArg {
  int p0, p1;     // patch range
  int b0, b1;     // bin range
  bool first, last;
  int t0, t1;     // output tile range
};

// Launch the kernels of one stage (for one launch group of patches).
static void launch_stage(hwo_ocean *o, int stage, const PatchArg *g) {
  const Dev &d = o->dev;
  switch (stage) {
    case ST_PARAMS: launch_params(d, o->st); break;
    case ST_FFT_A: launch_fft_a(d, o->st); break;
    case ST_FFT_B: launch_fft_b(d, o->st); break;
    case ST_COUNT: launch_update(d, g->p0, g->p1, false, o->update_grid, o->st); break;
    case ST_SCAN: launch_scan(d, g->b0, g->b1, g->first, g->last, o->st); break;
    case ST_SCATTER: launch_update(d, g->p0, g->p1, true, o->scatter_grid, o->st); break;
    case ST_PLAN: launch_splat_plan(d, g->t0, g->t1 - g->t0, o->items_target, o->st); break;
    case ST_SPLAT:
      launch_splat_tiles(d, g->t0, g->t1 - g->t0,
                         std::max(1, std::min(o->splat_grid > 0 ? o->splat_grid : 4 * o->target_blocks, d.max_items)),
                         o->st);
      break;
    case ST_REDUCE: launch_splat_reduce(d, g->t0, g->t1 - g->t0, o->st); break;
    case ST_BINPLAN: launch_bin_plan(d, d.nbins, d.ntiles, o->items_target, o->st); break;
    case ST_DEPX: launch_deposit_x(d, nullptr, 0, o->st); break;
    case ST_FILTY: launch_filter_y(d, 0, d.ntiles, o->st); break;
    case ST_LSUM: launch_layer_sum(d, 0, d.np, d.ncells, d.raw, d.blend, 0, o->st); break;
    case ST_NORMALS: launch_normals(d, o->st); break;
    default: break;
  }
}

static void timed(hwo_ocean *o, int stage, const PatchArg *g) {
  if (!o->timing) {
    launch_stage(o, stage, g);
    return;
  }
  TimedLaunch t;
  t.stage = stage;
  (void)hipEventCreate(&t.a);
  (void)hipEventCreate(&t.b);
  (void)hipEventRecord(t.a, o->st);
  launch_stage(o, stage, g);
  (void)hipEventRecord(t.b, o->st);
  o->tl.push_back(t);
}

// Launch groups: the whole ocean (batched) or one group per patch.
static std::vector<PatchArg> launch_groups(const hwo_ocean *o) {
  const Dev &d = o->dev;
  std::vector<PatchArg> groups;
  if (d.np == 0) return groups;   // no patches: no particle or splat launches
  if (o->cfg.batched) {
    groups.push_back({0, d.np, 0, d.nbins, true, true, 0, 0});
  } else {
    for (int p = 0; p < d.np; ++p)
      groups.push_back({p, p + 1, o->pdev[p].bin_lo, o->pdev[p].bin_hi, p == 0, p == d.np - 1, 0, 0});
  }
  for (auto &gp : groups) {
    const PatchDev &P0 = o->pdev[gp.p0];
    const PatchDev &P1 = o->pdev[gp.p1 - 1];
    gp.t0 = P0.tile0;
    gp.t1 = P1.tile0 + P1.ntx * P1.nty;
  }
  return groups;
}

static void run_step(hwo_ocean *o) {
  // While a frame graph is captured the FFT forks onto st2 after the step
  // parameters (it needs the step index) and joins before the first splat.
  // The branch is captured after the particle kernels it runs beside; that
  // capture order gives the faster graph schedule.
  const bool fork = o->capturing && o->st2;
  timed(o, ST_PARAMS, nullptr);
  if (fork) {
    (void)hipEventRecord(o->ev_fork, o->st);
  } else {
    timed(o, ST_FFT_A, nullptr);
    timed(o, ST_FFT_B, nullptr);
  }
  bool joined = !fork;
  auto join = [&]() {
    if (joined) return;
    (void)hipStreamWaitEvent(o->st2, o->ev_fork, 0);
    launch_fft_a(o->dev, o->st2);
    launch_fft_b(o->dev, o->st2);
    (void)hipEventRecord(o->ev_join, o->st2);
    (void)hipStreamWaitEvent(o->st, o->ev_join, 0);
    joined = true;
  };
  if (o->dev.np > 0) {
    const std::vector<PatchArg> groups = launch_groups(o);
    const bool layers = o->dev.synth == 1;
    if (o->fused) {
      // one group: the plan needs only the bin offsets, so it precedes the scatter
      timed(o, ST_COUNT, &groups[0]);
      timed(o, ST_BINPLAN, &groups[0]);
      timed(o, ST_SCATTER, &groups[0]);
    } else {
      for (const auto &gp : groups) {
        timed(o, ST_COUNT, &gp);
        timed(o, ST_SCAN, &gp);
        timed(o, ST_SCATTER, &gp);
      }
    }
    if (layers) {
      // texel layers of all patches: deposit and pass along x, pass along y,
      // then (with the background) the layer sum and blend
      timed(o, ST_DEPX, nullptr);
      timed(o, ST_FILTY, nullptr);
      join();
      timed(o, ST_LSUM, nullptr);
    } else if (o->fused) {
      join();
      timed(o, ST_SPLAT, &groups[0]);
      timed(o, ST_REDUCE, &groups[0]);
    } else {
      for (const auto &gp : groups) {
        timed(o, ST_PLAN, &gp);
        join();
        timed(o, ST_SPLAT, &gp);
        timed(o, ST_REDUCE, &gp);
      }
    }
    if (o->cfg.normals) timed(o, ST_NORMALS, nullptr);
  }
  join();
}

static int collect_timing(hwo_ocean *o) {
  if (o->tl.empty()) return HWO_OK;
  HWO_CHECK(hipStreamSynchronize(o->st));
  for (auto &t : o->tl) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    o->stage_ms[t.stage] += ms;
    o->stage_n[t.stage] += 1;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  o->tl.clear();
  return HWO_OK;
}

extern "C" {

int hwo_step(hwo_ocean *o, int32_t nsteps) {
  if (!o) return HWO_EINVAL;
  if (nsteps < 0) return o->fail(HWO_EINVAL, "nsteps must be >= 0");
  int rc = finalize(o);
  if (rc) return rc;
  if (o->n_host + nsteps > ((int64_t)1 << 31) - 1) return o->fail(HWO_ERANGE, "step index overflow");
  const bool use_graph = o->cfg.batched && !o->timing;
  for (int32_t k = 0; k < nsteps; ++k) {
    if (use_graph) {
      if (!o->exec) {
        HWO_CHECK(hipStreamBeginCapture(o->st, hipStreamCaptureModeThreadLocal));
        o->capturing = true;
        run_step(o);
        o->capturing = false;
        HWO_CHECK(hipStreamEndCapture(o->st, &o->graph));
        HWO_CHECK(hipGraphInstantiate(&o->exec, o->graph, nullptr, nullptr, 0));
      }
      HWO_CHECK(hipGraphLaunch(o->exec, o->st));
    } else {
      run_step(o);
      HWO_CHECK(hipGetLastError());
    }
    o->n_host += 1;
    if (o->timing && o->tl.size() > 4096) {
      rc = collect_timing(o);
      if (rc) return rc;
    }
  }
  return HWO_OK;
}

int hwo_sync(hwo_ocean *o) {
  if (!o) return HWO_EINVAL;
  if (o->st) HWO_CHECK(hipStreamSynchronize(o->st));
  return HWO_OK;
}

int64_t hwo_step_index(const hwo_ocean *o) { return o ? o->n_host : -1; }

int hwo_read_heightmaps(hwo_ocean *o, int32_t which, int32_t layer, float *dst, int64_t dst_elems,
                        int32_t dst_is_device) {
  if (!o || !dst) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  const Dev &d = o->dev;
  const float *src;
  int64_t n;
  if (which == -1) {
    if (layer < 0 || layer > 4) return o->fail(HWO_EINVAL, "background layer must be 0..4");
    if (layer >= d.nfields) return o->fail(HWO_ESTATE, "slope and displacement fields are not enabled (hwo_config.bg_fields)");
    src = d.H + (size_t)layer * d.N * d.N;
    n = (int64_t)d.N * d.N;
  } else {
    if (which < 0 || which >= d.np) return o->fail(HWO_ERANGE, "patch out of range");
    if (layer < 0 || layer > 4) return o->fail(HWO_EINVAL, "layer must be 0..4");
    if (layer >= 2 && !d.nrm) return o->fail(HWO_ESTATE, "normals are not enabled (hwo_config.normals)");
    const PatchDev &P = o->pdev[which];
    src = (layer == 0 ? d.blend : layer == 1 ? d.raw : d.nrm + (size_t)(layer - 2) * d.ncells) + P.cell0;
    n = (int64_t)P.nx * P.ny;
  }
  if (dst_elems < n) return o->fail(HWO_ERANGE, "destination too small");
  HWO_CHECK(hipMemcpyAsync(dst, src, sizeof(float) * (size_t)n,
                           dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  return HWO_OK;
}

int hwo_read_counts(hwo_ocean *o, int32_t patch, int64_t *dst, int64_t dst_elems) {
  if (!o || !dst) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  const Dev &d = o->dev;
  if (patch < 0 || patch >= d.np) return o->fail(HWO_ERANGE, "patch out of range");
  if (dst_elems < 6 * (int64_t)d.nb) return o->fail(HWO_ERANGE, "destination too small");
  const PatchDev &P = o->pdev[patch];
  std::vector<unsigned long long> ctr((size_t)d.nb * CNT_NUM);
  std::vector<int32_t> off((size_t)(P.bin_hi - P.bin_lo) + 1);
  Globals g{};
  HWO_CHECK(hipMemcpyAsync(ctr.data(), d.ctr + (size_t)patch * d.nb * CNT_NUM, sizeof(unsigned long long) * ctr.size(),
                           hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipMemcpyAsync(off.data(), d.off + P.bin_lo, sizeof(int32_t) * off.size(), hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipMemcpyAsync(&g, d.glob, sizeof(Globals), hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  const bool stepped = o->n_host > 0;
  for (int b = 0; b < d.nb; ++b) {
    const int lo = P.binbase[b] - P.bin_lo, hi = lo + P.nbx[b] * P.nby[b];
    dst[6 * b + 0] = stepped ? (int64_t)off[hi] - off[lo] : 0;
    dst[6 * b + 1] = (int64_t)ctr[(size_t)b * CNT_NUM + CNT_INJ];
    dst[6 * b + 2] = (int64_t)ctr[(size_t)b * CNT_NUM + CNT_EMIT];
    dst[6 * b + 3] = (int64_t)ctr[(size_t)b * CNT_NUM + CNT_SUB];
    dst[6 * b + 4] = (int64_t)ctr[(size_t)b * CNT_NUM + CNT_DIED];
    dst[6 * b + 5] = (int64_t)g.dropped;
  }
  if (g.err) return o->fail(HWO_ERANGE, "a window left the fixed-point position range");
  if (g.dropped) return o->fail(HWO_EOVERFLOW, "particle capacity exceeded");
  return HWO_OK;
}

int hwo_read_buckets(const hwo_ocean *o, double *dst, int32_t n) {
  if (!o || !dst) return HWO_EINVAL;
  if (!o->have_spec) return HWO_ESTATE;
  if (n < 4 * o->nb) return HWO_ERANGE;
  for (int i = 0; i < o->nb; ++i) {
    dst[4 * i + 0] = o->w[i];
    dst[4 * i + 1] = o->dw[i];
    dst[4 * i + 2] = o->r[i];
    dst[4 * i + 3] = o->c[i];
  }
  return HWO_OK;
}

int hwo_tile_dims(hwo_ocean *o, int32_t patch, int32_t bucket, int64_t *dims) {
  if (!o || !dims) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  if (patch < 0 || patch >= o->dev.np || bucket < 0 || bucket >= o->nb) return o->fail(HWO_ERANGE, "out of range");
  const PatchDev &P = o->pdev[patch];
  dims[0] = o->bin_cells[bucket];
  dims[1] = P.nbx[bucket];
  dims[2] = P.nby[bucket];
  return HWO_OK;
}

int hwo_read_tiles(hwo_ocean *o, int32_t patch, int32_t bucket, int64_t *dst, int64_t n) {
  if (!o || !dst) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  if (patch < 0 || patch >= o->dev.np || bucket < 0 || bucket >= o->nb) return o->fail(HWO_ERANGE, "out of range");
  const PatchDev &P = o->pdev[patch];
  const int64_t nh = (int64_t)P.nbx[bucket] * P.nby[bucket];
  if (n < nh) return o->fail(HWO_ERANGE, "destination too small");
  std::vector<int32_t> off((size_t)nh + 1);
  HWO_CHECK(hipMemcpyAsync(off.data(), o->dev.off + P.binbase[bucket], sizeof(int32_t) * off.size(),
                           hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  for (int64_t k = 0; k < nh; ++k) dst[k] = o->n_host > 0 ? (int64_t)off[k + 1] - off[k] : 0;
  return HWO_OK;
}

int hwo_read_particles(hwo_ocean *o, int64_t *dst, int64_t max_recs, int64_t *n_out) {
  if (!o || !n_out) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  const Dev &d = o->dev;
  Globals g{};
  HWO_CHECK(hipMemcpyAsync(&g, d.glob, sizeof(Globals), hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  const int64_t n = o->n_host > 0 ? g.n_live : 0;
  *n_out = n;
  if (!dst) return HWO_OK;
  if (max_recs < n) return o->fail(HWO_ERANGE, "destination too small");
  const void *S = (g.n & 1) ? d.S1 : d.S0;
  const int64_t step = g.n;
  if (d.compact) {
    std::vector<RecCompact> h((size_t)n);
    if (n) HWO_CHECK(hipMemcpy(h.data(), S, sizeof(RecCompact) * n, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < n; ++k) {
      const RecCompact &r = h[k];
      const uint32_t m = r.meta;
      const int64_t age = (int64_t)(((uint32_t)step - (r.bc & 0xFFFFu)) & 0xFFFFu);
      int64_t *q = dst + 10 * k;
      q[0] = m_patch(m); q[1] = m_bucket(m); q[2] = m_kind(m) + (m_heave(m) ? 1 : 0); q[3] = m_level(m);
      q[4] = r.bc >> 16; q[5] = step - age; q[6] = r.ox; q[7] = r.oy;
      q[8] = m_src(m) == kNoSource ? -1 : (int64_t)m_src(m); q[9] = m_slot(m);
    }
  } else {
    std::vector<RecWide> h((size_t)n);
    if (n) HWO_CHECK(hipMemcpy(h.data(), S, sizeof(RecWide) * n, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < n; ++k) {
      const RecWide &r = h[k];
      const uint32_t m = r.meta;
      int64_t *q = dst + 10 * k;
      q[0] = m_patch(m); q[1] = m_bucket(m); q[2] = m_kind(m) + (m_heave(m) ? 1 : 0); q[3] = m_level(m);
      q[4] = r.code; q[5] = r.birth; q[6] = r.ox; q[7] = r.oy;
      q[8] = m_src(m) == kNoSource ? -1 : (int64_t)m_src(m); q[9] = m_slot(m);
    }
  }
  return HWO_OK;
}

int hwo_test_splat(hwo_ocean *o, int32_t patch, const int64_t *recs, int64_t n, float *dst, int64_t dst_elems) {
  if (!o || (!recs && n > 0) || !dst || n < 0 || n > (1 << 24)) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  const Dev &d = o->dev;
  if (patch < 0 || patch >= d.np) return o->fail(HWO_ERANGE, "patch out of range");
  const PatchDev &P = o->pdev[patch];
  const int64_t cells = (int64_t)P.nx * P.ny;
  if (dst_elems < cells) return o->fail(HWO_ERANGE, "destination too small");
  // the window of the current step is needed; make sure sp[] is filled
  if (o->n_host == 0) return o->fail(HWO_ESTATE, "step at least once before splatting");
  const int64_t step = o->n_host;
  std::vector<uint8_t> host;
  const size_t rs = d.compact ? sizeof(RecCompact) : sizeof(RecWide);
  host.resize(rs * (size_t)std::max<int64_t>(n, 1));
  for (int64_t k = 0; k < n; ++k) {
    const int64_t *q = recs + 10 * k;
    if (q[0] != patch || q[1] < 0 || q[1] >= o->nb || q[2] < 0 || q[2] > 2 || q[4] < 0 || q[4] >= kNCode ||
        q[3] < 0 || q[3] > kMaxLevel || q[5] > step || step - q[5] > kAgeMax)
      return o->fail(HWO_EINVAL, "bad particle record");
    const bool ring = q[2] >= 1;
    if (ring && (q[8] < 0 || q[8] >= d.ns || q[9] < 0 || q[9] >= o->sdev[q[8]].ne))
      return o->fail(HWO_EINVAL, "bad ring particle record");
    if (q[2] == 2 && o->sdev[q[8]].Eh == 0) return o->fail(HWO_EINVAL, "vertical-motion ring of a source without heave");
    const uint32_t src = ring ? (uint32_t)q[8] : kNoSource;
    const uint32_t meta = pack_meta((uint32_t)q[3], ring ? 1u : 0u, (uint32_t)q[1], (uint32_t)q[0], src,
                                    ring ? (uint32_t)q[9] : 0u) | (q[2] == 2 ? kHeaveBit : 0u);
    if (d.compact) {
      RecCompact r;
      r.ox = (int32_t)q[6]; r.oy = (int32_t)q[7];
      r.bc = ((uint32_t)q[5] & 0xFFFFu) | ((uint32_t)q[4] << 16);
      r.meta = meta;
      memcpy(host.data() + rs * k, &r, rs);
    } else {
      RecWide r;
      r.ox = (int32_t)q[6]; r.oy = (int32_t)q[7]; r.birth = (int32_t)q[5]; r.code = (int32_t)q[4];
      r.meta = meta;
      float amp;
      if (q[2] == 0) amp = P.A[q[1]] * (o->afac.empty() ? 1.f : o->afac[(size_t)q[1] * kNCode + q[4]]);
      else if (q[2] == 2) {
        const SourceDev &S = o->sdev[q[8]];
        const double T = o->sources[q[8]].heave_period;
        const double z0 = sin(2.0 * M_PI * ((double)(q[5] - S.Eh) * o->cfg.dt) / T);
        const double z1 = sin(2.0 * M_PI * ((double)q[5] * o->cfg.dt) / T);
        amp = (float)(S.Bh * (z0 - z1) / std::pow(3.0, (double)q[3]));
      }
      else {
        const SourceDev &S = o->sdev[q[8]];
        amp = S.B * o->ring_m[S.ring0 + q[9]];
        for (int l = 0; l < q[3]; ++l) amp *= (1.0f / 3.0f);
      }
      r.amp = amp; r.pad0 = 0; r.pad1 = 0;
      memcpy(host.data() + rs * k, &r, rs);
    }
  }
  void *drec = nullptr;
  float *dout = nullptr;
  HWO_CHECK(hipMalloc(&drec, host.size()));
  HWO_CHECK(hipMalloc((void **)&dout, sizeof(float) * (size_t)cells));
  hipError_t e = hipMemcpyAsync(drec, host.data(), host.size(), hipMemcpyHostToDevice, o->st);
  if (e == hipSuccess) {
    if (d.synth == 1) {
      launch_deposit_x(d, drec, (int)n, o->st);
      launch_filter_y(d, P.tile0, P.ntx * P.nty, o->st);
      launch_layer_sum(d, patch, patch + 1, cells, dout, nullptr, P.cell0, o->st);
    } else {
      launch_splat_direct(d, P.tile0, P.ntx * P.nty, drec, (int)n, dout, P.cell0, o->st);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(dst, dout, sizeof(float) * (size_t)cells, hipMemcpyDeviceToHost, o->st);
  if (e == hipSuccess) e = hipStreamSynchronize(o->st);
  (void)hipFree(drec);
  (void)hipFree(dout);
  if (e != hipSuccess) return o->hip_fail(e, "test_splat");
  return HWO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- snapshot
// A step boundary is fully described by the step index, the globals, the
// per-bucket counters, the bin offsets of the last scan (the next step reads
// its particles through them), the live particle records and the splat's
// partition feedback; everything else is rebuilt from the step index or the
// scene.  The image starts with a header and a fingerprint of the scene.
namespace {
constexpr uint64_t kSnapMagic = 0x48574f534e415031ull;   // "HWOSNAP1"
struct SnapHeader {
  uint64_t magic;
  uint64_t scene;              // fingerprint of the scene tables
  int64_t n_host;
  int32_t np, nb, nbins, ntiles, cap, compact, n_live, pad;
};

uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

uint64_t scene_fingerprint(const hwo_ocean *o) {
  uint64_t h = 0xcbf29ce484222325ull;
  const hwo_config &c = o->cfg;
  h = fnv(h, &c.fft_n, sizeof c.fft_n);
  h = fnv(h, &c.fft_L, sizeof c.fft_L);
  h = fnv(h, &c.g, sizeof c.g);
  h = fnv(h, &c.dt, sizeof c.dt);
  h = fnv(h, &c.seed, sizeof c.seed);
  h = fnv(h, &c.compact, sizeof c.compact);
  h = fnv(h, o->w, sizeof(double) * (size_t)o->nb);
  h = fnv(h, o->pdev.data(), sizeof(PatchDev) * o->pdev.size());   // value-initialised: no stray padding
  h = fnv(h, o->sdev.data(), sizeof(SourceDev) * o->sdev.size());
  return h;
}

int64_t snapshot_bytes(const Dev &d, int32_t n_live) {
  return (int64_t)sizeof(SnapHeader) + (int64_t)sizeof(Globals) +
         (int64_t)sizeof(unsigned long long) * d.np * d.nb * CNT_NUM + (int64_t)sizeof(int32_t) * (d.nbins + 1) +
         (int64_t)(2 * sizeof(uint32_t) + sizeof(float)) * d.ntiles +
         (int64_t)(d.compact ? sizeof(RecCompact) : sizeof(RecWide)) * n_live;
}
}  // namespace

extern "C" {

int hwo_snapshot_size(hwo_ocean *o, int64_t *bytes) {
  if (!o || !bytes) return HWO_EINVAL;
  if (!o->finalized || o->n_host == 0) return o->fail(HWO_ESTATE, "snapshot needs a completed step");
  Globals g{};
  HWO_CHECK(hipMemcpyAsync(&g, o->dev.glob, sizeof(Globals), hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  *bytes = snapshot_bytes(o->dev, g.n_live);
  return HWO_OK;
}

int hwo_snapshot(hwo_ocean *o, void *dst, int64_t dst_bytes) {
  if (!o || !dst) return HWO_EINVAL;
  if (!o->finalized || o->n_host == 0) return o->fail(HWO_ESTATE, "snapshot needs a completed step");
  int rc = collect_timing(o);
  if (rc) return rc;
  const Dev &d = o->dev;
  Globals g{};
  HWO_CHECK(hipMemcpyAsync(&g, d.glob, sizeof(Globals), hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  if (dst_bytes < snapshot_bytes(d, g.n_live)) return o->fail(HWO_ERANGE, "snapshot buffer too small");
  char *p = (char *)dst;
  SnapHeader hd{kSnapMagic, scene_fingerprint(o), o->n_host, d.np, d.nb, d.nbins, d.ntiles, d.cap, d.compact,
                g.n_live, 0};
  memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  memcpy(p, &g, sizeof g);
  p += sizeof g;
  const size_t rb = d.compact ? sizeof(RecCompact) : sizeof(RecWide);
  const void *S = (g.n & 1) ? d.S1 : d.S0;
  const size_t nctr = sizeof(unsigned long long) * (size_t)d.np * d.nb * CNT_NUM;
  HWO_CHECK(hipMemcpyAsync(p, d.ctr, nctr, hipMemcpyDeviceToHost, o->st));
  p += nctr;
  HWO_CHECK(hipMemcpyAsync(p, d.off, sizeof(int32_t) * ((size_t)d.nbins + 1), hipMemcpyDeviceToHost, o->st));
  p += sizeof(int32_t) * ((size_t)d.nbins + 1);
  HWO_CHECK(hipMemcpyAsync(p, d.tile_meas, sizeof(uint32_t) * (size_t)d.ntiles, hipMemcpyDeviceToHost, o->st));
  p += sizeof(uint32_t) * (size_t)d.ntiles;
  HWO_CHECK(hipMemcpyAsync(p, d.tile_model, sizeof(uint32_t) * (size_t)d.ntiles, hipMemcpyDeviceToHost, o->st));
  p += sizeof(uint32_t) * (size_t)d.ntiles;
  HWO_CHECK(hipMemcpyAsync(p, d.tile_ratio, sizeof(float) * (size_t)d.ntiles, hipMemcpyDeviceToHost, o->st));
  p += sizeof(float) * (size_t)d.ntiles;
  if (g.n_live > 0) HWO_CHECK(hipMemcpyAsync(p, S, rb * (size_t)g.n_live, hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  return HWO_OK;
}

int hwo_restore(hwo_ocean *o, const void *src, int64_t src_bytes) {
  if (!o || !src || src_bytes < (int64_t)(sizeof(SnapHeader) + sizeof(Globals))) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  rc = collect_timing(o);
  if (rc) return rc;
  const Dev &d = o->dev;
  SnapHeader hd;
  Globals g;
  const char *p = (const char *)src;
  memcpy(&hd, p, sizeof hd);
  p += sizeof hd;
  memcpy(&g, p, sizeof g);
  p += sizeof g;
  if (hd.magic != kSnapMagic) return o->fail(HWO_EINVAL, "not a snapshot");
  if (hd.scene != scene_fingerprint(o) || hd.np != d.np || hd.nb != d.nb || hd.nbins != d.nbins ||
      hd.ntiles != d.ntiles || hd.compact != d.compact)
    return o->fail(HWO_EINVAL, "snapshot of a different scene or record form");
  if (hd.n_live < 0 || hd.n_live > d.cap || hd.n_live != g.n_live || g.n != hd.n_host || hd.n_host < 1)
    return o->fail(HWO_EINVAL, "inconsistent snapshot");
  if (src_bytes < snapshot_bytes(d, hd.n_live)) return o->fail(HWO_EINVAL, "truncated snapshot");
  HWO_CHECK(hipStreamSynchronize(o->st));
  const size_t rb = d.compact ? sizeof(RecCompact) : sizeof(RecWide);
  void *S = (g.n & 1) ? d.S1 : d.S0;
  HWO_CHECK(hipMemcpyAsync(d.glob, &g, sizeof g, hipMemcpyHostToDevice, o->st));
  const size_t nctr = sizeof(unsigned long long) * (size_t)d.np * d.nb * CNT_NUM;
  HWO_CHECK(hipMemcpyAsync(d.ctr, p, nctr, hipMemcpyHostToDevice, o->st));
  p += nctr;
  HWO_CHECK(hipMemcpyAsync(d.off, p, sizeof(int32_t) * ((size_t)d.nbins + 1), hipMemcpyHostToDevice, o->st));
  p += sizeof(int32_t) * ((size_t)d.nbins + 1);
  HWO_CHECK(hipMemcpyAsync(d.tile_meas, p, sizeof(uint32_t) * (size_t)d.ntiles, hipMemcpyHostToDevice, o->st));
  p += sizeof(uint32_t) * (size_t)d.ntiles;
  HWO_CHECK(hipMemcpyAsync(d.tile_model, p, sizeof(uint32_t) * (size_t)d.ntiles, hipMemcpyHostToDevice, o->st));
  p += sizeof(uint32_t) * (size_t)d.ntiles;
  HWO_CHECK(hipMemcpyAsync(d.tile_ratio, p, sizeof(float) * (size_t)d.ntiles, hipMemcpyHostToDevice, o->st));
  p += sizeof(float) * (size_t)d.ntiles;
  if (hd.n_live > 0) HWO_CHECK(hipMemcpyAsync(S, p, rb * (size_t)hd.n_live, hipMemcpyHostToDevice, o->st));
  // windows of the restored step (for probes and test splats before the next
  // step) and of the next one; the next step's histogram and counts of the
  // restored particles, which a scatter would have found
  if (d.np > 0) {
    launch_windows(d, o->st);
    HWO_CHECK(hipMemsetAsync(d.hist, 0, sizeof(int32_t) * ((size_t)d.nbins + 1), o->st));
    HWO_CHECK(hipMemsetAsync(d.ctr_next, 0, nctr, o->st));
    launch_predict(d, 0, d.np, o->update_grid, o->st);
    HWO_CHECK(hipGetLastError());
  }
  HWO_CHECK(hipStreamSynchronize(o->st));
  o->n_host = hd.n_host;
  return HWO_OK;
}

int hwo_sample_probes(hwo_ocean *o, const double *xy, int64_t n, float *out, int32_t on_device) {
  if (!o || n < 0 || n > (1 << 24) || (n > 0 && (!xy || !out))) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  if (o->n_host == 0) return o->fail(HWO_ESTATE, "step at least once before sampling");
  if (n == 0) return HWO_OK;
  const Dev &d = o->dev;
  const void *dxy = xy;
  void *dout = out;
  void *txy = nullptr, *tout = nullptr;
  hipError_t e = hipSuccess;
  if (!on_device) {
    e = hipMalloc(&txy, sizeof(double) * 2 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&tout, sizeof(float) * 4 * (size_t)n);
    if (e == hipSuccess)
      e = hipMemcpyAsync(txy, xy, sizeof(double) * 2 * (size_t)n, hipMemcpyHostToDevice, o->st);
    dxy = txy;
    dout = tout;
  }
  if (e == hipSuccess) {
    launch_probes(d, dxy, (int)n, dout, o->st);
    e = hipGetLastError();
  }
  if (e == hipSuccess && !on_device)
    e = hipMemcpyAsync(out, tout, sizeof(float) * 4 * (size_t)n, hipMemcpyDeviceToHost, o->st);
  if (e == hipSuccess) e = hipStreamSynchronize(o->st);
  if (txy) (void)hipFree(txy);
  if (tout) (void)hipFree(tout);
  if (e != hipSuccess) return o->hip_fail(e, "sample_probes");
  return HWO_OK;
}

int hwo_sample_probes_static(hwo_ocean *o, const double *xy, int64_t n, float *out) {
  if (!o || n < 0 || (n > 0 && (!xy || !out))) return HWO_EINVAL;
  if (n > kScratchProbes) return o->fail(HWO_ERANGE, "more probes than the static scratch holds (131072)");
  // no finalize here: building the device state allocates
  if (!o->finalized || o->n_host == 0) return o->fail(HWO_ESTATE, "step at least once before sampling");
  if (!o->scratch) return o->fail(HWO_EDEVICE, "static scratch unavailable: " + o->scratch_err);
  if (n == 0) return HWO_OK;
  unsigned char *base = (unsigned char *)o->scratch;
  void *sxy = base, *sout = base + kScratchBytes / 2;
  hipError_t e = hipMemcpyAsync(sxy, xy, sizeof(double) * 2 * (size_t)n, hipMemcpyHostToDevice, o->st);
  if (e == hipSuccess) {
    launch_probes(o->dev, sxy, (int)n, sout, o->st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, sout, sizeof(float) * 4 * (size_t)n, hipMemcpyDeviceToHost, o->st);
  if (e == hipSuccess) e = hipStreamSynchronize(o->st);
  if (e != hipSuccess) return o->hip_fail(e, "sample_probes_static");
  return HWO_OK;
}

int hwo_set_timing(hwo_ocean *o, int32_t enable) {
  if (!o) return HWO_EINVAL;
  int rc = collect_timing(o);
  if (rc) return rc;
  o->timing = enable != 0;
  for (int s = 0; s < kStages; ++s) {
    o->stage_ms[s] = 0.0;
    o->stage_n[s] = 0;
  }
  return HWO_OK;
}

int hwo_set_splat_profile(hwo_ocean *o, int32_t enable) {
  if (!o || (enable != 0 && enable != 1)) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  Dev &d = o->dev;
  HWO_CHECK(hipStreamSynchronize(o->st));
  HWO_CHECK(hipMemsetAsync(d.splat_prof, 0, sizeof(unsigned long long) * PROF_N, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  if (d.splat_profile != enable) {
    // the profiling splat is another kernel instance: capture the frame again
    d.splat_profile = enable;
    if (o->exec) (void)hipGraphExecDestroy(o->exec);
    if (o->graph) (void)hipGraphDestroy(o->graph);
    o->exec = nullptr;
    o->graph = nullptr;
  }
  return HWO_OK;
}

int hwo_read_splat_profile(hwo_ocean *o, double *dst, int32_t n) {
  if (!o || !dst || n < PROF_N) return HWO_EINVAL;
  if (!o->finalized) return o->fail(HWO_ESTATE, "no profile before the device state exists");
  const Dev &d = o->dev;
  unsigned long long h[PROF_N];
  HWO_CHECK(hipMemcpyAsync(h, d.splat_prof, sizeof(h), hipMemcpyDeviceToHost, o->st));
  HWO_CHECK(hipStreamSynchronize(o->st));
  for (int i = 0; i < PROF_N; ++i) dst[i] = (double)h[i];
  return HWO_OK;
}

int hwo_stage_times(hwo_ocean *o, double *ms, int64_t *launches, int32_t n) {
  if (!o || !ms || !launches || n < kStages) return HWO_EINVAL;
  int rc = collect_timing(o);
  if (rc) return rc;
  for (int s = 0; s < kStages; ++s) {
    ms[s] = o->stage_ms[s];
    launches[s] = o->stage_n[s];
  }
  return HWO_OK;
}

int hwo_time_stage(hwo_ocean *o, int32_t stage, int32_t reps, double *ms_per_rep) {
  if (!o || !ms_per_rep || reps < 1) return HWO_EINVAL;
  const bool splat_stage = stage == ST_PLAN || stage == ST_SPLAT || stage == ST_REDUCE;
  const bool layer_stage = stage == ST_DEPX || stage == ST_FILTY || stage == ST_LSUM;
  const bool normal_stage = stage == ST_NORMALS;
  if (stage != ST_FFT_A && stage != ST_FFT_B && !splat_stage && !layer_stage && !normal_stage)
    return o->fail(HWO_EINVAL, "stage is not repeatable (it advances or consumes state)");
  if (normal_stage && !o->cfg.normals) return o->fail(HWO_EINVAL, "normals are not enabled");
  if ((splat_stage && o->cfg.synth == 1) || (layer_stage && o->cfg.synth != 1))
    return o->fail(HWO_EINVAL, "stage is not part of this synthesis mode");
  if (o->n_host < 1) return o->fail(HWO_ESTATE, "time_stage needs a completed step");
  int rc = collect_timing(o);
  if (rc) return rc;
  const std::vector<PatchArg> groups = launch_groups(o);
  hipEvent_t a = nullptr, b = nullptr;
  HWO_CHECK(hipEventCreate(&a));
  HWO_CHECK(hipEventCreate(&b));
  HWO_CHECK(hipEventRecord(a, o->st));
  for (int k = 0; k < reps; ++k) {
    if (stage == ST_FFT_A || stage == ST_FFT_B || layer_stage || normal_stage) launch_stage(o, stage, nullptr);
    else
      for (const auto &gp : groups) launch_stage(o, stage, &gp);
  }
  HWO_CHECK(hipEventRecord(b, o->st));
  HWO_CHECK(hipEventSynchronize(b));
  float ms = 0.f;
  HWO_CHECK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  HWO_CHECK(hipGetLastError());
  *ms_per_rep = (double)ms / reps;
  return HWO_OK;
}

static void drop_graph(hwo_ocean *o) {
  if (o->exec) (void)hipGraphExecDestroy(o->exec);
  if (o->graph) (void)hipGraphDestroy(o->graph);
  o->exec = nullptr;
  o->graph = nullptr;
}

int hwo_get_plan(hwo_ocean *o, hwo_plan *out) {
  if (!o || !out) return HWO_EINVAL;
  int rc = finalize(o);
  if (rc) return rc;
  out->chunk_load = (int32_t)o->dev.chunk_load;
  out->items_target = o->items_target;
  out->splat_grid = o->splat_grid;
  out->splat_kernel = o->dev.splat_kernel;
  return HWO_OK;
}

int hwo_set_plan(hwo_ocean *o, const hwo_plan *p) {
  if (!o || !p) return HWO_EINVAL;
  if (p->chunk_load < 64 || p->chunk_load > (1 << 24) || p->items_target < 0 || p->items_target > 8192 ||
      p->splat_grid < 0 || p->splat_grid > 65535 || p->splat_kernel < 0 || p->splat_kernel > 2)
    return o->fail(HWO_EINVAL, "plan parameter out of range");
  int rc = finalize(o);
  if (rc) return rc;
  HWO_CHECK(hipStreamSynchronize(o->st));
  o->dev.chunk_load = (uint32_t)p->chunk_load;
  o->items_target = p->items_target;
  o->splat_grid = p->splat_grid;
  o->dev.splat_kernel = p->splat_kernel;
  drop_graph(o);   // the plan parameters are kernel arguments of the captured frame
  return HWO_OK;
}

// Milliseconds per (plan, splat, reduce) on the current frame, after two
// untimed rounds that let the partition feedback settle.
static int time_partition(hwo_ocean *o, int reps, double *ms) {
  const std::vector<PatchArg> groups = launch_groups(o);
  auto round = [&]() {
    for (const auto &gp : groups) {
      launch_stage(o, ST_PLAN, &gp);
      launch_stage(o, ST_SPLAT, &gp);
      launch_stage(o, ST_REDUCE, &gp);
    }
  };
  round();
  round();
  hipEvent_t a = nullptr, b = nullptr;
  HWO_CHECK(hipEventCreate(&a));
  HWO_CHECK(hipEventCreate(&b));
  HWO_CHECK(hipEventRecord(a, o->st));
  for (int k = 0; k < reps; ++k) round();
  HWO_CHECK(hipEventRecord(b, o->st));
  HWO_CHECK(hipEventSynchronize(b));
  float t = 0.f;
  HWO_CHECK(hipEventElapsedTime(&t, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  HWO_CHECK(hipGetLastError());
  *ms = (double)t / reps;
  return HWO_OK;
}

int hwo_autotune(hwo_ocean *o, int32_t reps, hwo_plan *best, double *best_ms, double *start_ms) {
  if (!o || !best || !best_ms || !start_ms || reps < 1) return HWO_EINVAL;
  if (o->cfg.synth == 1) return o->fail(HWO_EINVAL, "the texel-layer synthesis has no splat partition");
  if (o->n_host < 1) return o->fail(HWO_ESTATE, "autotune needs a completed step");
  int rc = collect_timing(o);
  if (rc) return rc;
  Dev &d = o->dev;
  const hwo_plan start{(int32_t)d.chunk_load, o->items_target, o->splat_grid, d.splat_kernel};
  auto apply = [&](const hwo_plan &p) {
    d.chunk_load = (uint32_t)p.chunk_load;
    o->items_target = p.items_target;
    o->splat_grid = p.splat_grid;
    d.splat_kernel = p.splat_kernel;
  };
  double t_start = 0.0;
  rc = time_partition(o, reps, &t_start);
  if (rc) return rc;
  *start_ms = t_start;
  hwo_plan best_plan = start;
  double t_best = t_start;
  const int room = std::min(8192, d.max_items - d.ntiles);
  const int tb = o->target_blocks;   // four per compute unit
  const std::vector<int32_t> chunks = {1000, 1750, 2500, 3500, 5000, 7000, 10000, 14000};
  const std::vector<int32_t> items = {256, 512, 1024, 2048, 4096, 8192};
  const std::vector<int32_t> grids = {tb / 2, tb, 2 * tb, 4 * tb, 8 * tb};
  // for each splat schedule, two sweeps of coordinate descent from the
  // starting partition
  for (int32_t kern = 0; kern < 3; ++kern) {
    hwo_plan cur = start;
    cur.splat_kernel = kern;
    apply(cur);
    double t_cur = t_start;
    if (kern != start.splat_kernel) {
      rc = time_partition(o, reps, &t_cur);
      if (rc) return rc;
    }
    for (int sweep = 0; sweep < 2; ++sweep) {
      for (int coord = 0; coord < 3; ++coord) {
        const std::vector<int32_t> &vals = coord == 0 ? chunks : coord == 1 ? items : grids;
        for (int32_t v : vals) {
          hwo_plan p = cur;
          if (coord == 0) p.chunk_load = v;
          if (coord == 1) {
            if (v > room) continue;
            p.items_target = v;
          }
          if (coord == 2) p.splat_grid = std::max(1, v);
          if (p.chunk_load == cur.chunk_load && p.items_target == cur.items_target && p.splat_grid == cur.splat_grid)
            continue;
          apply(p);
          double t = 0.0;
          rc = time_partition(o, reps, &t);
          if (rc) return rc;
          if (t < t_cur) {
            t_cur = t;
            cur = p;
          }
        }
        apply(cur);
      }
    }
    if (t_cur < t_best) {
      t_best = t_cur;
      best_plan = cur;
    }
  }
  const hwo_plan cur = best_plan;
  const double t_cur = t_best;
  apply(cur);
  drop_graph(o);
  // leave the frame's outputs from the chosen partition
  double t = 0.0;
  rc = time_partition(o, 1, &t);
  if (rc) return rc;
  *best = cur;
  *best_ms = t_cur;
  return HWO_OK;
}

int32_t hwo_record_bytes(const hwo_ocean *o) {
  if (!o) return 0;
  return o->cfg.compact ? (int32_t)sizeof(RecCompact) : (int32_t)sizeof(RecWide);
}

}  // extern "C"

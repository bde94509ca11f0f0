// fft.hip -- FFT background on gfx950.
//
// Background field (Sec 4.1 "FFT updates", spectrum of Sec 3.1 Eq 1-6):
//   H(x_j, t) = sum_k h~(k, t) e^{i k.x_j},
//   h~(k, t)  = h0(k) e^{-i w t} + conj(h0(-k)) e^{+i w t},  w = sqrt(g |k|),
// with h0(k) = 1/2 (xi_r + i xi_i) sqrt(S_k) dk, S_k = S_J(w) Dir(theta) g / (2 w k).
//
// h~ is Hermitian, so H is real.  Two passes, each one Stockham radix-8/4/2
// FFT per row in LDS:
//   pass A  for every kx index mx in [0, N/2]: evolve h~(mx, .) from rows mx
//           and -mx of h0 (stored transposed, so both reads are contiguous),
//           FFT along y, write F[mx][jy].
//   pass B  for every pair of output rows (jy_a, jy_b): rebuild the full
//           length-N x-spectrum from the half plane (F[N-mx] = conj F[mx]),
//           pack the two real transforms into one complex FFT
//           (Z = F_a + i F_b), write H[jy_a] = Re, H[jy_b] = Im.
// HBM bytes per point: h0 8 (read) + F 4 (write) + F 4 (read) + H 4 (write).
// h0 and the twiddles are generated in FP64 and stored FP32.
//
// Optional derived fields (blockIdx.y = field, one launch per pass for all):
// the slopes dH/dx, dH/dy (spectrum times i kx, i ky) and the choppy
// displacement sum -i (k/|k|) h~ e^{ik.x}; each is real, so the same two
// passes apply.  Their Nyquist rows and columns and k = 0 are dropped (an
// odd multiplier would make the Nyquist terms non-Hermitian).
#include "hwo_dev.h"

namespace hwo {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by +i
__device__ __forceinline__ float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }

// In-register DFTs with kernel e^{+2 pi i nk / R}.
__device__ __forceinline__ void dft2(float2 *v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
  float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  float2 s13 = cadd(a1, a3), d13 = cmuli(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}
__device__ __forceinline__ void dft4v(float2 *v) { dft4(v[0], v[1], v[2], v[3]); }
__device__ __forceinline__ void dft8(float2 *v) {
  const float h = 0.70710678118654752f;
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // twiddles w^k, w = e^{i pi / 4}
  float2 t1 = make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y));
  float2 t2 = cmuli(o2);
  float2 t3 = make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

template <int R> __device__ __forceinline__ void dftR(float2 *v);
template <> __device__ __forceinline__ void dftR<2>(float2 *v) { dft2(v); }
template <> __device__ __forceinline__ void dftR<4>(float2 *v) { dft4v(v); }
template <> __device__ __forceinline__ void dftR<8>(float2 *v) { dft8(v); }

// One Stockham stage of an N-point FFT held in LDS, T threads per transform.
// Butterfly j reads x[j + r N/R], applies e^{2 pi i r k / (Ns R)} (k = j mod Ns),
// and writes y[(j - k) R + k + r Ns].  All threads of the block must call it.
template <int N, int T, int R>
__device__ __forceinline__ void fft_stage(float2 *buf, int t, int Ns, const float2 *__restrict__ tw) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + T - 1) / T;
  float2 v[PER][R];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    int j = t + u * T;
    if (j < NB) {
      int k = j & (Ns - 1);
      int step = N / (Ns * R);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 x = buf[j + r * NB];
        if (r > 0 && Ns > 1) x = cmul(x, tw[r * k * step]);
        v[u][r] = x;
      }
      dftR<R>(v[u]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    int j = t + u * T;
    if (j < NB) {
      int k = j & (Ns - 1);
      int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[u][r];
    }
  }
  __syncthreads();
}

// Full inverse FFT (no scaling) of N points in LDS: radix-8 stages then one
// radix-4 or radix-2 stage for the remaining factor.
template <int N, int T>
__device__ __forceinline__ void fft_lds(float2 *buf, int t, const float2 *__restrict__ tw) {
  int Ns = 1;
  constexpr int L2 = __builtin_ctz(N);
  constexpr int n8 = L2 / 3;
  constexpr int rem = L2 - 3 * n8;
#pragma unroll
  for (int s = 0; s < n8; ++s) {
    fft_stage<N, T, 8>(buf, t, Ns, tw);
    Ns *= 8;
  }
  if (rem == 2) fft_stage<N, T, 4>(buf, t, Ns, tw);
  if (rem == 1) fft_stage<N, T, 2>(buf, t, Ns, tw);
}

// ---- radix-16 first stage on the matrix cores (optional)
// The first stage of the Stockham FFT (no twiddles) is a batch of 16-point
// DFTs, Y = F X with F[m][r] = e^{+2 pi i m r / 16}, i.e. in real form
// [Yr; Yi] = [[Fr, -Fi], [Fi, Fr]] [Xr; Xi]: for 32 butterflies at a time a
// 32 x 32 by 32 x 32 product, two 32x32x16 bf16 matrix-core products per
// operand pair.  FP32 operands are split into bf16 hi + lo parts; hi hi,
// hi lo and lo hi products are accumulated in FP32 (lo lo, ~2^-16 relative,
// is dropped).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16v __attribute__((ext_vector_type(16)));

// Butterflies j0 .. j0 + 31 (input x[j + r N/16], output y[16 j + m]) of one
// transform held in buf; the outputs are returned in registers (lane l: the
// m = 4 (l / 32) + {0..3} and 8 + 4 (l / 32) + {0..3} outputs of butterfly
// j0 + l % 32, real parts in d[0..7], imaginary in d[8..15]) so that the
// caller can write them after every wave has read its inputs.
template <int N>
__device__ __forceinline__ f32x16v dft16_mfma(const float2 *buf, int j0, int lane) {
  const int j = j0 + (lane & 31), kb = 8 * (lane >> 5);   // butterfly; first r of the lane's K slice
  // operands: A = the DFT matrix (rows i = m or 16 + m, columns r), split
  bf16x8 a0h, a0l, a1h, a1l, xrh, xrl, xih, xil;
  const int i = lane & 31, m = i & 15;
  const bool top = i < 16;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int r = kb + q;
    const float ph = (float)((m * r) & 15) * (1.0f / 16.0f);   // revolutions
    const float c = __builtin_amdgcn_cosf(ph), s = __builtin_amdgcn_sinf(ph);
    const float v0 = top ? c : s, v1 = top ? -s : c;   // columns r of [Fr; Fi] and [-Fi; Fr]
    const __bf16 h0 = (__bf16)v0, h1 = (__bf16)v1;
    a0h[q] = h0;
    a0l[q] = (__bf16)(v0 - (float)h0);
    a1h[q] = h1;
    a1l[q] = (__bf16)(v1 - (float)h1);
    const float2 x = buf[j + r * (N / 16)];
    const __bf16 xr = (__bf16)x.x, xi = (__bf16)x.y;
    xrh[q] = xr;
    xrl[q] = (__bf16)(x.x - (float)xr);
    xih[q] = xi;
    xil[q] = (__bf16)(x.y - (float)xi);
  }
  f32x16v acc;
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.f;
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, xrh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, xrl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0l, xrh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, xih, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, xil, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1l, xih, acc, 0, 0, 0);
  return acc;
}

// First stage (radix 16) of an N-point transform with T threads on the
// matrix cores; every thread of the block calls it.
template <int N, int T>
__device__ __forceinline__ void fft_stage16_mfma(float2 *buf, int t) {
  constexpr int G = N / 16 / 32;        // groups of 32 butterflies
  constexpr int W = T / 64;             // wavefronts per transform
  constexpr int PER = (G + W - 1) / W;  // groups per wavefront
  const int w = t >> 6, lane = t & 63;
  f32x16v out[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (w + u * W < G) out[u] = dft16_mfma<N>(buf, 32 * (w + u * W), lane);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (w + u * W < G) {
      const int j = 32 * (w + u * W) + (lane & 31);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        // D row i = 8 (q / 4) + 4 (l / 32) + q % 4 (q < 8: real part, row i + 16: imaginary part)
        const int mo = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        buf[16 * j + mo] = make_float2(out[u][q], out[u][q + 8]);
      }
    }
  }
  __syncthreads();
}

// Full inverse FFT with the radix-16 first stage on the matrix cores, then
// radix-8 stages and one radix-4 or radix-2 stage.
template <int N, int T>
__device__ __forceinline__ void fft_lds_m16(float2 *buf, int t, const float2 *__restrict__ tw) {
  fft_stage16_mfma<N, T>(buf, t);
  int Ns = 16;
  constexpr int L2 = __builtin_ctz(N) - 4;
  constexpr int n8 = L2 / 3;
  constexpr int rem = L2 - 3 * n8;
#pragma unroll
  for (int s = 0; s < n8; ++s) {
    fft_stage<N, T, 8>(buf, t, Ns, tw);
    Ns *= 8;
  }
  if (rem == 2) fft_stage<N, T, 4>(buf, t, Ns, tw);
  if (rem == 1) fft_stage<N, T, 2>(buf, t, Ns, tw);
}

template <int N, int T>
__device__ __forceinline__ void fft_row(float2 *buf, int t, const float2 *__restrict__ tw, bool m16) {
  if constexpr (N >= 1024 && T >= 64 && N / 512 >= T / 64) {
    if (m16) {
      fft_lds_m16<N, T>(buf, t, tw);
      return;
    }
  }
  fft_lds<N, T>(buf, t, tw);
}

template <int N> struct FftShape {
  static constexpr int T = (N / 8 < kThreads) ? (N / 8 < 1 ? 1 : N / 8) : kThreads;
  static constexpr int F = kThreads / T;      // transforms per block
};

__device__ __forceinline__ int signed_idx(int j, int N) { return j < N / 2 ? j : j - N; }

// Blocks b, b+8, b+16, ... share an XCD (round-robin dispatch); give them
// neighbouring work so their cache lines stay in one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  int per = nb / 8;
  if (per == 0 || (nb % 8) != 0) return b;
  return (b % 8) * per + b / 8;
}

template <int N>
__global__ __launch_bounds__(kThreads) void k_fft_a(Dev d) {
  constexpr int T = FftShape<N>::T, F = FftShape<N>::F;
  __shared__ float2 buf[F * N];
  const int f = threadIdx.x / T, t = threadIdx.x % T;
  const int mx = blockIdx.x * F + f;
  const int field = blockIdx.y;
  const bool active = mx <= N / 2;
  const float tn = (float)((double)d.glob->n * d.dt);
  const float dk = (float)(2.0 * M_PI / d.L);
  const float g = (float)d.g;
  float2 *row = buf + f * N;
  constexpr int E = N / T;   // elements per thread
  if (active) {
    const int mxn = (N - mx) & (N - 1);
    const float kx = dk * (float)signed_idx(mx, N);
    const float2 *__restrict__ ha = d.h0T + (size_t)mx * N;
    const float2 *__restrict__ hb = d.h0T + (size_t)mxn * N;
    // all loads of the thread first (one round trip), then the evolution
    float2 av[E], bv[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = t + k * T;
      av[k] = ha[e];
      bv[k] = hb[(N - e) & (N - 1)];
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = t + k * T;
      const float2 a = av[k], b = bv[k];
      float ky = dk * (float)signed_idx(e, N);
      // phase w t in revolutions, reduced to [-1/2, 1/2] for v_sin/v_cos
      const float w = sqrtf(g * sqrtf(fmaf(kx, kx, ky * ky)));
      float rev = w * tn * 0.159154943091895336f;
      rev -= rintf(rev);
      const float s = __builtin_amdgcn_sinf(rev), c = __builtin_amdgcn_cosf(rev);
      // a e^{-iwt} + conj(b) e^{+iwt}
      float re = fmaf(a.x + b.x, c, (a.y + b.y) * s);
      float im = fmaf(a.y - b.y, c, (b.x - a.x) * s);
      if (field != 0) {   // times i m
        float m = 0.f;
        if (mx != N / 2 && e != N / 2) {
          if (field == 1) m = kx;
          else if (field == 2) m = ky;
          else {
            const float kk2 = fmaf(kx, kx, ky * ky);
            m = kk2 > 0.f ? -(field == 3 ? kx : ky) * rsqrtf(kk2) : 0.f;
          }
        }
        const float r2 = -m * im;
        im = m * re;
        re = r2;
      }
      row[e] = make_float2(re, im);
    }
  } else {
    for (int e = t; e < N; e += T) row[e] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_row<N, T>(row, t, d.tw, d.fft_mfma16 != 0);
  if (active) {
    float2 *__restrict__ out = d.FT + (size_t)field * (N / 2 + 1) * N + (size_t)mx * N;
    for (int e = t; e < N; e += T) out[e] = row[e];
  }
}

template <int N> struct FftShapeB {
  // row pairs per block; 4096-point transforms take 64 KiB of rows so that
  // each half-plane row is read in runs of at least 32 bytes; 2048-point
  // ones take two row pairs (runs of 32 bytes, two blocks per CU: 12.0 us
  // per pass against 12.4 us with four pairs in 512-thread blocks)
  static constexpr int F0 = FftShape<N>::F < N / 2 ? FftShape<N>::F : N / 2;
  static constexpr int F = (N == 2048) ? 2 : (N >= 4096) ? 65536 / (8 * N) : F0;
  static constexpr int B = kThreads;   // threads per block
  static constexpr int T = B / F;
};

template <int N>
__global__ __launch_bounds__(FftShapeB<N>::B) void k_fft_b(Dev d) {
  constexpr int F = FftShapeB<N>::F, T = FftShapeB<N>::T, B = FftShapeB<N>::B;
  constexpr int C = 2 * F;                    // output rows per block
  __shared__ float2 buf[F * N];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int jy0 = blk * C;
  const float2 *__restrict__ FT = d.FT + (size_t)blockIdx.y * (N / 2 + 1) * N;
  // Load the half plane F[0..N/2][jy0 .. jy0+C) with consecutive threads on
  // consecutive column pairs of one row, and rebuild the full x-spectrum:
  // Z[mx] = F_a[mx] + i F_b[mx], Z[N-mx] = conj(F_a[mx]) + i conj(F_b[mx]).
  // all loads of the thread first (one round trip), then the repacking
  constexpr int Q = (N / 2 + 1) * F, K = (Q + B - 1) / B;
  float4 v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int q = (int)threadIdx.x + k * B;
    if (q < Q) {
      const int mx = q / F, f = q % F;
      v[k] = *reinterpret_cast<const float4 *>(FT + (size_t)mx * N + jy0 + 2 * f);
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int q = (int)threadIdx.x + k * B;
    if (q < Q) {
      const int mx = q / F, f = q % F;
      const float2 fa = make_float2(v[k].x, v[k].y), fb = make_float2(v[k].z, v[k].w);
      float2 *z = buf + f * N;
      z[mx] = make_float2(fa.x - fb.y, fa.y + fb.x);
      if (mx > 0 && mx < N / 2) z[N - mx] = make_float2(fa.x + fb.y, fb.x - fa.y);
    }
  }
  __syncthreads();
  const int f = threadIdx.x / T, t = threadIdx.x % T;
  float2 *row = buf + f * N;
  fft_row<N, T>(row, t, d.tw, d.fft_mfma16 != 0);
  float *__restrict__ ha = d.H + (size_t)blockIdx.y * N * N + (size_t)(jy0 + 2 * f) * N;
  float *__restrict__ hb = ha + N;
  for (int e = t; e < N; e += T) {
    float2 z = row[e];
    ha[e] = z.x;
    hb[e] = z.y;
  }
}

// ---------------------------------------------------------------- h0 (FP64)
__device__ double jonswap_d(double w, double alpha, double g, double wp, double gamma) {
  if (w <= 0.0) return 0.0;
  double sigma = (w <= wp) ? 0.07 : 0.09;
  double dd = w - wp;
  double r = exp(-(dd * dd) / (2.0 * sigma * sigma * wp * wp));
  double x = wp / w;
  double x4 = x * x * x * x;
  return alpha * g * g * pow(w, -5.0) * exp(-1.25 * x4) * pow(gamma, r);
}

__device__ double dir_d(double s, double theta) {
  double norm = tgamma(s + 1.0) / (2.0 * sqrt(M_PI) * tgamma(s + 0.5));
  double c = fabs(cos(0.5 * theta));
  return norm * pow(c, 2.0 * s);
}

__global__ void k_h0(Dev d, float2 *h0T, double alpha, double wp, double gamma, double s_const,
                     double wind_dir, int h0_mode) {
  const int N = d.N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int jy = (int)(idx / N), jx = (int)(idx % N);
  const int mx = signed_idx(jx, N), my = signed_idx(jy, N);
  float2 out = make_float2(0.f, 0.f);
  if (mx != 0 || my != 0) {
    const double dk = 2.0 * M_PI / d.L;
    const double kx = dk * (double)mx, ky = dk * (double)my;
    const double k = sqrt(kx * kx + ky * ky);
    const double w = sqrt(d.g * k);
    double th = atan2(ky, kx) - wind_dir;
    th = th - 2.0 * M_PI * floor((th + M_PI) / (2.0 * M_PI));
    double s = s_const;
    if (s < 0.0) s = 16.0 * pow(w / wp, (w <= wp) ? 5.0 : -2.5);
    const double Sk = jonswap_d(w, alpha, d.g, wp, gamma) * dir_d(s, th) * d.g / (2.0 * w * k);
    uint64_t c[4] = {(uint64_t)jy, (uint64_t)jx, 0, 0};
    philox4x64(c, d.seed, kStreamH0);
    const double ua = (double)(c[0] >> 11) * (1.0 / 9007199254740992.0) + (1.0 / 18014398509481984.0);
    const double ub = (double)(c[1] >> 11) * (1.0 / 9007199254740992.0) + (1.0 / 18014398509481984.0);
    double amp, rho;
    if (h0_mode == 1) {
      amp = dk * sqrt(0.5 * Sk);
      rho = 1.0;
    } else {
      amp = 0.5 * sqrt(Sk) * dk;
      rho = sqrt(-2.0 * log(ua));
    }
    out = make_float2((float)(amp * rho * cos(2.0 * M_PI * ub)), (float)(amp * rho * sin(2.0 * M_PI * ub)));
  }
  h0T[(size_t)jx * N + jy] = out;
}

__global__ void k_twiddle(float2 *tw, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double a = 2.0 * M_PI * (double)k / (double)N;
  tw[k] = make_float2((float)cos(a), (float)sin(a));
}

void launch_h0(const Dev &d, float2 *h0T, float2 *tw, double alpha, double wp, double gamma,
               double s_const, double wind_dir, int h0_mode, hipStream_t st) {
  const int64_t n2 = (int64_t)d.N * d.N;
  hipLaunchKernelGGL(k_h0, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, d, h0T, alpha, wp, gamma,
                     s_const, wind_dir, h0_mode);
  hipLaunchKernelGGL(k_twiddle, dim3((d.N + 255) / 256), dim3(256), 0, st, tw, d.N);
}

template <int N> static void fft_a_n(const Dev &d, hipStream_t st) {
  constexpr int F = FftShape<N>::F;
  const int rows = N / 2 + 1;
  hipLaunchKernelGGL(k_fft_a<N>, dim3((rows + F - 1) / F, d.nfields), dim3(kThreads), 0, st, d);
}
template <int N> static void fft_b_n(const Dev &d, hipStream_t st) {
  constexpr int F = FftShapeB<N>::F;
  hipLaunchKernelGGL(k_fft_b<N>, dim3(N / (2 * F), d.nfields), dim3(FftShapeB<N>::B), 0, st, d);
}

void launch_fft_a(const Dev &d, hipStream_t st) {
  switch (d.N) {
    case 16: fft_a_n<16>(d, st); break;
    case 32: fft_a_n<32>(d, st); break;
    case 64: fft_a_n<64>(d, st); break;
    case 128: fft_a_n<128>(d, st); break;
    case 256: fft_a_n<256>(d, st); break;
    case 512: fft_a_n<512>(d, st); break;
    case 1024: fft_a_n<1024>(d, st); break;
    case 2048: fft_a_n<2048>(d, st); break;
    case 4096: fft_a_n<4096>(d, st); break;
    default: break;
  }
}
void launch_fft_b(const Dev &d, hipStream_t st) {
  switch (d.N) {
    case 16: fft_b_n<16>(d, st); break;
    case 32: fft_b_n<32>(d, st); break;
    case 64: fft_b_n<64>(d, st); break;
    case 128: fft_b_n<128>(d, st); break;
    case 256: fft_b_n<256>(d, st); break;
    case 512: fft_b_n<512>(d, st); break;
    case 1024: fft_b_n<1024>(d, st); break;
    case 2048: fft_b_n<2048>(d, st); break;
    case 4096: fft_b_n<4096>(d, st); break;
    default: break;
  }
}

}  // namespace hwo

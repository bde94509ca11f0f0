// layers.hip -- the paper's own height synthesis (Sec 4.2), as an alternative
// to the exact-position splat: every particle point is accumulated into the
// layer texture of its bucket, each layer is smoothed by a pass along x and a
// pass along y with the raised cosine sampled at whole-cell offsets, and the
// layers are summed and blended with the background.
//
// Deposit.  A point (crest +A at the particle, trough -A at the particle minus
// round(r u 2^20)) is shared bilinearly by the four cell centres around it,
// which keeps the result within A dx^2 pi^2 / (8 r^2) of the exact kernel.  A
// layer covers the patch plus R = ceil(r / dx) - 1 cells on each side (the
// reach of the taps), so points farther out are dropped.  Texel indices come
// from integer positions and are exact; weights are FP32.  Deposits are
// float atomics into HBM (L2), one thread per particle, over the bin-sorted
// buffer so that neighbouring threads hit neighbouring texels.
//
// Pass along x: one block per layer row, the row and the taps staged in LDS,
// one output per thread and column.  Pass along y: one block per 64 x 64
// output tile; per bucket the (64 + 2R) x 64 strip of the x-filtered layer is
// staged in LDS and each thread sums 16 rows of one column; the sum over
// buckets stays in registers and is blended and stored once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hwo_dev.h"

namespace hwo {

namespace {

constexpr int kRowsPerThread = kTile * kTile / kThreads;   // 16

__global__ __launch_bounds__(kThreads) void k_layer_clear(float4 *__restrict__ p, int64_t n4) {
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kThreads) p[i] = z;
}

// Bilinear deposit of amplitude A at window-relative position (x, y) (units)
// into a layer of W x Hh texels whose texel t sits at cell t - R.
__device__ __forceinline__ void deposit_point(float *__restrict__ lay, int W, int Hh, int R, int dxu, float inv_dxu,
                                              int64_t x, int64_t y, float A) {
  // shifted so that the quotient is t0 + 1 >= 0 for every point that can
  // touch texel 0; anything else lies outside the layer
  const int64_t xo = x - dxu / 2 + (int64_t)(R + 1) * dxu;
  const int64_t yo = y - dxu / 2 + (int64_t)(R + 1) * dxu;
  if (xo < 0 || yo < 0 || xo >= (int64_t)(W + 1) * dxu || yo >= (int64_t)(Hh + 1) * dxu) return;
  const uint32_t qx = (uint32_t)xo / (uint32_t)dxu, qy = (uint32_t)yo / (uint32_t)dxu;
  const float tx = (float)((uint32_t)xo - qx * (uint32_t)dxu) * inv_dxu;
  const float ty = (float)((uint32_t)yo - qy * (uint32_t)dxu) * inv_dxu;
  const int i0 = (int)qx - 1, j0 = (int)qy - 1;
  const float a0 = A * (1.f - ty), a1 = A * ty;
  if (j0 >= 0) {
    float *row = lay + (size_t)j0 * W;
    if (i0 >= 0) atomicAdd(row + i0, a0 * (1.f - tx));
    if (i0 + 1 < W) atomicAdd(row + i0 + 1, a0 * tx);
  }
  if (j0 + 1 < Hh) {
    float *row = lay + (size_t)(j0 + 1) * W;
    if (i0 >= 0) atomicAdd(row + i0, a1 * (1.f - tx));
    if (i0 + 1 < W) atomicAdd(row + i0 + 1, a1 * tx);
  }
}

template <class Rec>
__global__ __launch_bounds__(kThreads) void k_deposit(Dev d, const Rec *__restrict__ direct, int ndirect) {
  const int64_t n = d.glob->n;
  const Rec *__restrict__ S = direct ? direct : (const Rec *)((n & 1) ? d.S1 : d.S0);
  const int count = direct ? ndirect : d.glob->n_live;
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < count; k += gridDim.x * kThreads) {
    const Part q = RecIO<Rec>::unpack(S[k], n);
    const int p = (int)m_patch(q.meta), b = (int)m_bucket(q.meta);
    const PatchDev &P = d.patches[p];
    const StepPatch &Wp = d.sp[p];
    const int2 v = d.V[b * kNCode + q.code];
    const int64_t px = (int64_t)q.ox + (((int64_t)q.age * v.x) >> 12);
    const int64_t py = (int64_t)q.oy + (((int64_t)q.age * v.y) >> 12);
    const int64_t x = px - (int64_t)Wp.wx * P.dxu, y = py - (int64_t)Wp.wy * P.dxu;
    const float A = particle_amp<Rec>(d, q);
    const int R = P.lay_R[b];
    const int W = P.nx + 2 * R, Hh = P.ny + 2 * R;
    float *lay = d.lay + P.lay_off[b];
    const float inv_dxu = 1.0f / (float)P.dxu;
    const int2 to = d.toff[b * kNCode + q.code];
    deposit_point(lay, W, Hh, R, P.dxu, inv_dxu, x, y, A);
    deposit_point(lay, W, Hh, R, P.dxu, inv_dxu, x - to.x, y - to.y, -A);
  }
}

// Layer (patch, bucket) holding global layer row r: last l with row_base[l] <= r.
__device__ __forceinline__ int layer_of_row(const Dev &d, int r) {
  int lo = 0, hi = d.np * d.nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.row_base[mid] <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kThreads) void k_filter_x(Dev d) {
  extern __shared__ float xs[];
  const int r = blockIdx.x;
  const int l = layer_of_row(d, r);
  const int p = l / d.nb, b = l - p * d.nb;
  const PatchDev &P = d.patches[p];
  const int j = r - d.row_base[l];
  const int R = P.lay_R[b], W = P.nx + 2 * R, nt = 2 * R + 1;
  float *s_row = xs;
  float *s_w = xs + W;
  const float *src = d.lay + P.lay_off[b] + (size_t)j * W;
  for (int i = threadIdx.x; i < W; i += kThreads) s_row[i] = src[i];
  for (int i = threadIdx.x; i < nt; i += kThreads) s_w[i] = d.taps[P.tap_off[b] + i];
  __syncthreads();
  float *dst = d.lt + P.lt_off[b] + (size_t)j * P.nx;
  for (int i = threadIdx.x; i < P.nx; i += kThreads) {
    // the taps are symmetric: sum_k row[i + R - k] w(k) = sum_t row[i + t] w_t
    float s = 0.f;
    for (int t = 0; t < nt; ++t) s = fmaf(s_row[i + t], s_w[t], s);
    dst[i] = s;
  }
}

__global__ __launch_bounds__(kThreads) void k_filter_y(Dev d, int t0, float *__restrict__ raw_out,
                                                       float *__restrict__ blend_out, int64_t out_off) {
  extern __shared__ float ys[];
  const int tile = t0 + blockIdx.x;
  const int p = patch_of_tile(d, tile);
  TileGeom T;
  tile_geom(d, tile, p, T);
  const PatchDev &P = d.patches[p];
  const StepPatch &Wp = d.sp[p];
  const int c = threadIdx.x & (kTile - 1);
  const int jr0 = (threadIdx.x / kTile) * kRowsPerThread;
  float acc[kRowsPerThread];
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) acc[u] = 0.f;
  for (int b = 0; b < d.nb; ++b) {
    const int R = P.lay_R[b], nt = 2 * R + 1;
    const int rows = T.th + 2 * R;
    float *s_t = ys;
    float *s_w = ys + (size_t)(kTile + 2 * R) * kTile;
    // rows j0 .. j0 + th + 2R - 1 of the x-filtered layer (patch rows j - R)
    const float *src = d.lt + P.lt_off[b] + (size_t)T.j0 * P.nx + T.i0;
    for (int e = threadIdx.x; e < rows * kTile; e += kThreads) {
      const int rr = e / kTile, cc = e - rr * kTile;
      s_t[e] = (cc < T.tw) ? src[(size_t)rr * P.nx + cc] : 0.f;
    }
    for (int i = threadIdx.x; i < nt; i += kThreads) s_w[i] = d.taps[P.tap_off[b] + i];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u) {
      const int jr = jr0 + u;
      if (jr < T.th) {
        float s = 0.f;
        for (int t = 0; t < nt; ++t) s = fmaf(s_t[(jr + t) * kTile + c], s_w[t], s);
        acc[u] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) {
    const int jr = jr0 + u;
    if (jr < T.th && c < T.tw) blend_store(d, P, Wp, T, c, jr, acc[u], raw_out, blend_out, out_off);
  }
}

}  // namespace

void launch_layer_clear(const Dev &d, hipStream_t st) {
  if (d.lay_n <= 0) return;
  const int64_t n4 = d.lay_n / 4;
  const int grid = (int)std::min<int64_t>((n4 + kThreads - 1) / kThreads, 8192);
  hipLaunchKernelGGL(k_layer_clear, dim3(grid), dim3(kThreads), 0, st, (float4 *)d.lay, n4);
}

void launch_deposit(const Dev &d, const void *recs, int n, hipStream_t st) {
  const int grid = recs ? std::max(1, std::min((n + kThreads - 1) / kThreads, 8192)) : std::max(1, std::min(d.cap / kThreads + 1, 4096));
  if (d.compact)
    hipLaunchKernelGGL(k_deposit<RecCompact>, dim3(grid), dim3(kThreads), 0, st, d, (const RecCompact *)recs, n);
  else
    hipLaunchKernelGGL(k_deposit<RecWide>, dim3(grid), dim3(kThreads), 0, st, d, (const RecWide *)recs, n);
}

void launch_filter_x(const Dev &d, hipStream_t st) {
  if (d.nlayer_rows <= 0) return;
  hipLaunchKernelGGL(k_filter_x, dim3(d.nlayer_rows), dim3(kThreads), d.xsmem, st, d);
}

hipError_t prepare_layers(const Dev &d) {
  // the y pass stages (64 + 2R) x 64 floats, which can exceed the default
  // 64 KiB dynamic LDS limit (gfx950 offers 160 KiB per workgroup)
  hipError_t e = hipFuncSetAttribute((const void *)k_filter_y, hipFuncAttributeMaxDynamicSharedMemorySize, d.ysmem);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_filter_x, hipFuncAttributeMaxDynamicSharedMemorySize, d.xsmem);
  return e;
}

void launch_filter_y(const Dev &d, int t0, int ntiles, float *raw, float *blend, int64_t out_off, hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_filter_y, dim3(ntiles), dim3(kThreads), d.ysmem, st, d, t0, raw, blend, out_off);
}

}  // namespace hwo

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
// reach of the taps); points farther out are dropped.  Texel indices come
// from integer positions and are exact; weights are FP32.
//
// Three launches, none with global atomics and no layer texture in HBM:
//   k_deposit_x  one block per 64 x 64 tile of a bucket's x-filtered layer:
//                the crests of the bins that can reach the tile's
//                64 x (64 + 2R) texels are deposited with LDS atomics, then
//                the pass along x runs from LDS and the tile is stored.
//   k_filter_y   one block per (output tile, bucket): the (64 + 2R) x 64 strip
//                of the x-filtered layer is staged in LDS, each thread sums
//                16 rows of one column, the bucket's plane is stored.
//   k_layer_sum  one thread per patch cell: the sum over the bucket planes,
//                blended with the background and stored with the raw map.
// k_normals (either synthesis, when enabled) derives unit normals from the
// blended maps by finite differences.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hwo_dev.h"

namespace hwo {

namespace {

constexpr int kRowsPerThread = kTile * kTile / kThreads;   // 16
constexpr int kBatch = 4;                                   // particles in flight per thread (deposit)
// A part costs its particles plus one x pass, so only tiles far above a
// typical load are cut (the wake rings of a source crowd a few tiles).
constexpr int kPartLoad = 4096;                             // particles per part of a heavy layer tile

// Bilinear deposit of amplitude A at window-relative position (x, y) (units)
// into the LDS window D of columns [tx0, tx0 + dw) and rows [ty0, ty0 + dh)
// of a layer whose texel t sits at cell t - R.
__device__ __forceinline__ void deposit_point(float *__restrict__ D, int pitch, int tx0, int ty0, int dw, int dh,
                                              int R, int dxu, float inv_dxu, int64_t x, int64_t y, float A) {
  // shifted so that the quotient is t0 + 1 >= 0 for every point that can
  // touch texel 0 of the layer
  const int64_t xo = x - dxu / 2 + (int64_t)(R + 1) * dxu;
  const int64_t yo = y - dxu / 2 + (int64_t)(R + 1) * dxu;
  if (xo < (int64_t)tx0 * dxu || yo < (int64_t)ty0 * dxu || xo >= (int64_t)(tx0 + dw + 1) * dxu ||
      yo >= (int64_t)(ty0 + dh + 1) * dxu)
    return;
  // 0 <= xo < (W + 1) dxu < 2^32 here
  const uint32_t qx = (uint32_t)xo / (uint32_t)dxu, qy = (uint32_t)yo / (uint32_t)dxu;
  const float tx = (float)((uint32_t)xo - qx * (uint32_t)dxu) * inv_dxu;
  const float ty = (float)((uint32_t)yo - qy * (uint32_t)dxu) * inv_dxu;
  const int i0 = (int)qx - 1 - tx0, j0 = (int)qy - 1 - ty0;   // in [-1, dw - 1] x [-1, dh - 1]
  const float a0 = A * (1.f - ty), a1 = A * ty;
  if (j0 >= 0) {
    float *row = D + j0 * pitch;
    if (i0 >= 0) atomicAdd(row + i0, a0 * (1.f - tx));
    if (i0 + 1 < dw) atomicAdd(row + i0 + 1, a0 * tx);
  }
  if (j0 + 1 < dh) {
    float *row = D + (j0 + 1) * pitch;
    if (i0 >= 0) atomicAdd(row + i0, a1 * (1.f - tx));
    if (i0 + 1 < dw) atomicAdd(row + i0 + 1, a1 * tx);
  }
}

// Layer (patch, bucket) holding x-filter tile k: last l with xt_base[l] <= k.
__device__ __forceinline__ int layer_of_xtile(const Dev &d, int k) {
  int lo = 0, hi = d.np * d.nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.xt_base[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class Rec>
__device__ __forceinline__ void deposit_rec(const Dev &d, const Rec &r, int64_t n, int b, const PatchDev &P,
                                            const StepPatch &Wp, float *D, int pitch, int tx0, int ty0, int dw,
                                            int dh, int R, float inv_dxu) {
  const Part q = RecIO<Rec>::unpack(r, n);
  const int2 v = velocity(d, b, q.code, m_kind(q.meta) == 0);
  const int64_t px = (int64_t)q.ox + (((int64_t)q.age * v.x) >> 12);
  const int64_t py = (int64_t)q.oy + (((int64_t)q.age * v.y) >> 12);
  const int64_t x = px - (int64_t)Wp.wx * P.dxu, y = py - (int64_t)Wp.wy * P.dxu;
  const float A = particle_amp<Rec>(d, q, n);
  const int2 to = d.toff[b * kNCode + q.code];
  deposit_point(D, pitch, tx0, ty0, dw, dh, R, P.dxu, inv_dxu, x, y, A);
  deposit_point(D, pitch, tx0, ty0, dw, dh, R, P.dxu, inv_dxu, x - to.x, y - to.y, -A);
}

// Register-blocked FIR over 16 consecutive outputs: out[u] = sum_k w[k] v[u + k]
// for u < 16, k < K16 (taps zero-padded to a multiple of 16).  v(i) returns
// the input at offset i (LDS); two windows of 16 inputs stay in registers, so
// each tap costs one broadcast LDS read for 16 multiply-adds.
template <class Load>
__device__ __forceinline__ void fir16(const float *__restrict__ s_w, int K16, Load v, float acc[16]) {
  float cur[16], nxt[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) cur[u] = v(u);
  for (int k0 = 0; k0 < K16; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) nxt[u] = v(16 + k0 + u);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const float wk = s_w[k0 + kk];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = fmaf(wk, (u + kk < 16) ? cur[u + kk] : nxt[u + kk - 16], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) cur[u] = nxt[u];
  }
}

template <class Rec>
__global__ __launch_bounds__(kThreads) void k_deposit_x(Dev d, const Rec *__restrict__ direct, int ndirect) {
  extern __shared__ float xs[];
  __shared__ int s_rlo[64], s_pre[65];
  __shared__ int s_total;
  // block = (x tile, part); a tile whose bins hold many particles is cut
  // into up to d.xparts parts of about kPartLoad particles, each writing a
  // partial tile that the y pass sums.  Part 0 of every tile comes first in
  // the grid, the blocks of further parts (most of which exit at once) last.
  const int part = (int)blockIdx.x / d.n_xtiles;
  const int k = (int)blockIdx.x - part * d.n_xtiles;
  const int l = layer_of_xtile(d, k);
  const int p = l / d.nb, b = l - p * d.nb;
  const PatchDev &P = d.patches[p];
  const StepPatch &Wp = d.sp[p];
  const int R = P.lay_R[b], nt = 2 * R + 1, K16 = (nt + 15) & ~15;
  const int W = P.nx + 2 * R, Hh = P.ny + 2 * R;
  const int ntc = (P.nx + kTile - 1) / kTile;
  const int kt = k - d.xt_base[l];
  const int tr = kt / ntc, tc = kt - tr * ntc;
  const int ty0 = tr * kTile, tx0 = tc * kTile;            // first texel row / column of D
  const int dh = min(kTile, Hh - ty0);                      // rows of this tile
  const int tw = min(kTile, P.nx - tx0);                    // output columns
  const int dw = min(kTile + 2 * R, W - tx0);               // texel columns of D
  const int pitch = kTile + 2 * R + 17;                     // odd: column reads across rows are conflict-free
  float *D = xs;
  float *s_w = xs + kTile * pitch;
  const int64_t n = d.glob->n;
  const float inv_dxu = 1.0f / (float)P.dxu;
  // crests whose crest or trough can land in D: window-relative x in
  // [xa - ru, xb + ru) with ru >= |trough offset|; bins are anchored at the
  // window origin minus the survival margin m
  const int64_t m = d.margin[b], binu = P.binu[b];
  const int64_t ru = (int64_t)(d.bucket_r[b] * 1048576.0f * 1.000001f) + 2;
  const int64_t xa = (int64_t)(tx0 - 1 - R) * P.dxu + P.dxu / 2, xb = (int64_t)(tx0 + dw - R) * P.dxu + P.dxu / 2;
  const int64_t ya = (int64_t)(ty0 - 1 - R) * P.dxu + P.dxu / 2, yb = (int64_t)(ty0 + dh - R) * P.dxu + P.dxu / 2;
  const int bx_lo = (int)max<int64_t>(0, floor_div(xa - ru + m, binu));
  const int bx_hi = (int)min<int64_t>(P.nbx[b] - 1, floor_div(xb + ru + m, binu));
  const int by_lo = (int)max<int64_t>(0, floor_div(ya - ru + m, binu));
  const int by_hi = (int)min<int64_t>(P.nby[b] - 1, floor_div(yb + ru + m, binu));
  // particles in the bin rectangle (one wavefront), hence the parts
  if (threadIdx.x < 64) {
    int tot = 0;
    if (!direct && bx_lo <= bx_hi)
      for (int by = by_lo + (int)threadIdx.x; by <= by_hi; by += 64) {
        const int rb = P.binbase[b] + by * P.nbx[b];
        tot += max(0, min(d.off[rb + bx_hi + 1], d.cap) - min(d.off[rb + bx_lo], d.cap));
      }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
    if (threadIdx.x == 0) s_total = tot;
  }
  __syncthreads();
  const int M = s_total;
  const int nparts = direct ? 1 : max(1, min(d.xparts, (M + kPartLoad - 1) / kPartLoad));
  if (part >= nparts) return;   // block-uniform
  if (part == 0 && threadIdx.x == 0) d.xt_nparts[k] = nparts;
  const int e_lo = (int)((int64_t)M * part / nparts), e_hi = (int)((int64_t)M * (part + 1) / nparts);
  for (int e = threadIdx.x; e < kTile * pitch; e += kThreads) D[e] = 0.f;
  for (int e = threadIdx.x; e < K16; e += kThreads) s_w[e] = e < nt ? d.taps[P.tap_off[b] + e] : 0.f;
  __syncthreads();
  if (direct) {
    for (int e = threadIdx.x; e < ndirect; e += kThreads) {
      const Part q = RecIO<Rec>::unpack(direct[e], n);
      if ((int)m_patch(q.meta) == p && (int)m_bucket(q.meta) == b)
        deposit_rec<Rec>(d, direct[e], n, b, P, Wp, D, pitch, tx0, ty0, dw, dh, R, inv_dxu);
    }
  } else {
    const Rec *__restrict__ S = (const Rec *)((n & 1) ? d.S1 : d.S0);
    // up to 64 bin rows at a time: row lengths, their prefix (one wavefront),
    // then every thread takes particles of the flattened list that fall in
    // this part, so that the record loads of a block are independent
    int g0 = 0;   // flattened index of the chunk's first particle
    for (int r0 = by_lo; r0 <= by_hi && bx_lo <= bx_hi && g0 < e_hi; r0 += 64) {   // block-uniform
      const int nr = min(64, by_hi - r0 + 1);
      if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int len = 0;
        if (lane < nr) {
          const int rb = P.binbase[b] + (r0 + lane) * P.nbx[b];
          const int lo = min(d.off[rb + bx_lo], d.cap), hi = min(d.off[rb + bx_hi + 1], d.cap);
          s_rlo[lane] = lo;
          len = max(0, hi - lo);
        }
        int inc = len;
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(inc, o);
          if (lane >= o) inc += y;
        }
        s_pre[lane] = inc - len;
        if (lane == 63) s_pre[64] = inc;
      }
      __syncthreads();
      const int total = s_pre[64];
      const int c_lo = max(0, e_lo - g0), c_hi = min(total, e_hi - g0);
      g0 += total;
      // kBatch particles per thread per round: their record loads, then their
      // table loads, are issued together before any deposit
      for (int e0 = c_lo; e0 < c_hi; e0 += kThreads * kBatch) {
        Rec rr[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          const int e = e0 + j * kThreads + (int)threadIdx.x;
          if (e < c_hi) {
            int lo = 0, hi = nr - 1;   // last row with prefix <= e
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
            }
            rr[j] = S[s_rlo[lo] + (e - s_pre[lo])];
          }
        }
        Part q[kBatch];
        int2 v[kBatch], to[kBatch];
        float A[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          if (e0 + j * kThreads + (int)threadIdx.x < c_hi) {
            q[j] = RecIO<Rec>::unpack(rr[j], n);
            v[j] = velocity(d, b, q[j].code, m_kind(q[j].meta) == 0);
            to[j] = d.toff[b * kNCode + q[j].code];
            A[j] = particle_amp<Rec>(d, q[j], n);
          }
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          if (e0 + j * kThreads + (int)threadIdx.x < c_hi) {
            const int64_t px = (int64_t)q[j].ox + (((int64_t)q[j].age * v[j].x) >> 12);
            const int64_t py = (int64_t)q[j].oy + (((int64_t)q[j].age * v[j].y) >> 12);
            const int64_t x = px - (int64_t)Wp.wx * P.dxu, y = py - (int64_t)Wp.wy * P.dxu;
            deposit_point(D, pitch, tx0, ty0, dw, dh, R, P.dxu, inv_dxu, x, y, A[j]);
            deposit_point(D, pitch, tx0, ty0, dw, dh, R, P.dxu, inv_dxu, x - to[j].x, y - to[j].y, -A[j]);
          }
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // pass along x: T[ty0 + row][tx0 + c] = sum_t D[row][c + t] w_t (the taps
  // are symmetric); each thread makes 16 consecutive columns of one row
  const int row = threadIdx.x & (kTile - 1);
  const int c0 = (threadIdx.x / kTile) * 16;
  if (row < dh && c0 < tw) {
    float acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.f;
    const float *src = D + row * pitch + c0;
    fir16(s_w, K16, [&](int i) { return src[i]; }, acc);
    float *dst = (nparts == 1) ? d.lt + P.lt_off[b] + (size_t)(ty0 + row) * P.nx + tx0 + c0
                               : d.xpartial + ((size_t)k * d.xparts + part) * (kTile * kTile) + row * kTile + c0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (c0 + u < tw) dst[u] = acc[u];
  }
}

__global__ __launch_bounds__(kThreads) void k_filter_y(Dev d, int t0) {
  extern __shared__ float ys[];
  const int tile = t0 + (int)blockIdx.x / d.nb;
  const int b = (int)blockIdx.x - (tile - t0) * d.nb;
  const int p = patch_of_tile(d, tile);
  TileGeom T;
  tile_geom(d, tile, p, T);
  const PatchDev &P = d.patches[p];
  const int c = threadIdx.x & (kTile - 1);
  const int jr0 = (threadIdx.x / kTile) * kRowsPerThread;
  const int R = P.lay_R[b], nt = 2 * R + 1, K16 = (nt + 15) & ~15;
  const int rows = T.th + 2 * R;
  const int srows = kTile + 2 * R + 17;   // rows read by the register-blocked pass, zero beyond `rows`
  float *s_t = ys;
  float *s_w = ys + srows * kTile;
  // rows j0 .. j0 + th + 2R - 1 of the x-filtered layer (patch rows j - R);
  // rows of a tile cut into parts are the sum of its partial tiles
  const float *src = d.lt + P.lt_off[b] + (size_t)T.j0 * P.nx + T.i0;
  const int xbase = d.xt_base[p * d.nb + b] + T.i0 / kTile;
  const int ntc = (P.nx + kTile - 1) / kTile;
  __shared__ int s_np[16];   // parts of the x tiles the strip crosses (the LDS budget keeps R <= 279: <= 10 tiles)
  const int xr0 = T.j0 / kTile;
  if (threadIdx.x < 16 && (T.j0 + rows - 1) / kTile >= xr0 + (int)threadIdx.x)
    s_np[threadIdx.x] = d.xt_nparts[xbase + (xr0 + (int)threadIdx.x) * ntc];
  __syncthreads();
  for (int e = threadIdx.x; e < srows * kTile; e += kThreads) {
    const int rr = e / kTile, cc = e - rr * kTile;
    float v = 0.f;
    if (rr < rows && cc < T.tw) {
      const int tr = T.j0 + rr;   // x-filtered layer row
      const int xt = xbase + (tr / kTile) * ntc;
      const int np = s_np[tr / kTile - xr0];
      if (np <= 1) {
        v = src[(size_t)rr * P.nx + cc];
      } else {
        const float *pp = d.xpartial + (size_t)xt * d.xparts * (kTile * kTile) + (tr % kTile) * kTile + cc;
        for (int q = 0; q < np; ++q) v += pp[(size_t)q * (kTile * kTile)];
      }
    }
    s_t[e] = v;
  }
  for (int i = threadIdx.x; i < K16; i += kThreads) s_w[i] = i < nt ? d.taps[P.tap_off[b] + i] : 0.f;
  __syncthreads();
  if (c >= T.tw || jr0 >= T.th) return;
  float acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.f;
  const float *col = s_t + jr0 * kTile + c;
  fir16(s_w, K16, [&](int i) { return col[i * kTile]; }, acc);
  float *dst = d.yplanes + (size_t)b * d.ncells + P.cell0 + (size_t)T.j0 * P.nx + T.i0 + c;
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u)
    if (jr0 + u < T.th) dst[(size_t)(jr0 + u) * P.nx] = acc[u];
}

__global__ __launch_bounds__(kThreads) void k_layer_sum(Dev d, int p0, int p1, float *__restrict__ raw_out,
                                                        float *__restrict__ blend_out, int64_t out_off) {
  const int64_t c0 = d.patches[p0].cell0;
  const int64_t c1 = d.patches[p1 - 1].cell0 + (int64_t)d.patches[p1 - 1].nx * d.patches[p1 - 1].ny;
  for (int64_t cell = c0 + (int64_t)blockIdx.x * kThreads + threadIdx.x; cell < c1;
       cell += (int64_t)gridDim.x * kThreads) {
    int lo = p0, hi = p1 - 1;   // last patch with cell0 <= cell
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (d.patches[mid].cell0 <= cell) lo = mid; else hi = mid - 1;
    }
    const PatchDev &P = d.patches[lo];
    float h = 0.f;
    for (int b = 0; b < d.nb; ++b) h += d.yplanes[(size_t)b * d.ncells + cell];
    const int64_t lc = cell - P.cell0;
    TileGeom T;
    T.p = lo;
    T.i0 = 0;
    T.j0 = 0;
    blend_store(d, P, d.sp[lo], T, (int)(lc % P.nx), (int)(lc / P.nx), h, raw_out, blend_out, out_off);
  }
}

// Normals of the blended maps by finite differences (Sec 4.2): central
// differences inside, one-sided at the first and last row and column, unit
// normal (-sx, -sy, 1) / sqrt(1 + sx^2 + sy^2); one thread per cell.
__global__ __launch_bounds__(kThreads) void k_normals(Dev d) {
  for (int64_t cell = (int64_t)blockIdx.x * kThreads + threadIdx.x; cell < d.ncells;
       cell += (int64_t)gridDim.x * kThreads) {
    int lo = 0, hi = d.np - 1;   // last patch with cell0 <= cell
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (d.patches[mid].cell0 <= cell) lo = mid; else hi = mid - 1;
    }
    const PatchDev &P = d.patches[lo];
    const int64_t lc = cell - P.cell0;
    const int i = (int)(lc % P.nx), j = (int)(lc / P.nx);
    const float *h = d.blend + P.cell0;
    const float inv_dx = (float)(1.0 / P.dx);
    float sx = 0.f, sy = 0.f;
    if (P.nx > 1) {
      const int a = i > 0 ? i - 1 : i, b = i < P.nx - 1 ? i + 1 : i;
      sx = (h[(size_t)j * P.nx + b] - h[(size_t)j * P.nx + a]) * inv_dx / (float)(b - a);
    }
    if (P.ny > 1) {
      const int a = j > 0 ? j - 1 : j, b = j < P.ny - 1 ? j + 1 : j;
      sy = (h[(size_t)b * P.nx + i] - h[(size_t)a * P.nx + i]) * inv_dx / (float)(b - a);
    }
    const float inv = 1.0f / sqrtf(1.f + sx * sx + sy * sy);
    d.nrm[cell] = -sx * inv;
    d.nrm[d.ncells + cell] = -sy * inv;
    d.nrm[2 * d.ncells + cell] = inv;
  }
}

}  // namespace

void launch_normals(const Dev &d, hipStream_t st) {
  if (!d.nrm || d.ncells <= 0) return;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((d.ncells + kThreads - 1) / kThreads, 16384));
  hipLaunchKernelGGL(k_normals, dim3(grid), dim3(kThreads), 0, st, d);
}

hipError_t prepare_layers(const Dev &d) {
  // both passes stage up to (64 + 2R) x 64 floats, which can exceed the
  // default 64 KiB dynamic LDS limit (gfx950 offers 160 KiB per workgroup)
  hipError_t e = hipFuncSetAttribute((const void *)k_filter_y, hipFuncAttributeMaxDynamicSharedMemorySize, d.lsmem);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_deposit_x<RecCompact>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            d.lsmem);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_deposit_x<RecWide>, hipFuncAttributeMaxDynamicSharedMemorySize, d.lsmem);
  return e;
}

void launch_deposit_x(const Dev &d, const void *recs, int n, hipStream_t st) {
  if (d.n_xtiles <= 0) return;
  const int grid = d.n_xtiles * d.xparts;
  if (d.compact)
    hipLaunchKernelGGL(k_deposit_x<RecCompact>, dim3(grid), dim3(kThreads), d.lsmem, st, d, (const RecCompact *)recs,
                       n);
  else
    hipLaunchKernelGGL(k_deposit_x<RecWide>, dim3(grid), dim3(kThreads), d.lsmem, st, d, (const RecWide *)recs, n);
}

void launch_filter_y(const Dev &d, int t0, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_filter_y, dim3(ntiles * d.nb), dim3(kThreads), d.lsmem, st, d, t0);
}

void launch_layer_sum(const Dev &d, int p0, int p1, int64_t cells, float *raw, float *blend, int64_t out_off,
                      hipStream_t st) {
  if (p1 <= p0 || cells <= 0) return;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((cells + kThreads - 1) / kThreads, 16384));
  hipLaunchKernelGGL(k_layer_sum, dim3(grid), dim3(kThreads), 0, st, d, p0, p1, raw, blend, out_off);
}

}  // namespace hwo

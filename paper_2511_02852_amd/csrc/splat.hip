// splat.hip -- per-bucket splat of wave-particle pairs and the blend epilogue.
//
// Each particle of bucket b is a crest +A at its position p and a trough -A
// one radius behind it, p - r_b u (the positive-negative pair of Fig 1);
// both use the separable raised cosine K(d) = w(d_x) w(d_y),
// w(d) = 1/2 (1 + cos(pi d / r_b)) for |d| < r_b (Sec 4.2: per-bucket layers
// smoothed by separable x and y passes; here evaluated at the exact
// particle position).  The bucket layers are summed into the patch height.
//
// One block owns one 64x64 output tile of one patch and keeps it in LDS for
// all buckets.  For each bucket it walks the particle bins whose crests can
// reach the tile (within 2 r_b), which are contiguous runs of the sorted
// particle buffer.  A group of G lanes (G ~ footprint width, a power of two)
// takes one particle: the lanes first write the row weights w(d_y) of the
// clipped footprint to a per-wave LDS scratch, then each lane owns columns
// and adds A w(d_x) w(d_y) into the tile with LDS atomics.  After the last
// bucket the tile is blended with the background,
//   h = s h_WP + (1 - s) bilinear(H),  s = smoothstep(edge distance / band),
// (Sec 3.1 local replacement, smooth distance weights of Sec 4.2) and both
// maps leave in one coalesced write.
#include "hwo_dev.h"

namespace hwo {

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class Rec>
__global__ __launch_bounds__(kThreads) void k_splat(Dev d, int t0, const Rec *__restrict__ direct, int ndirect,
                                                    float *__restrict__ raw_out, float *__restrict__ blend_out,
                                                    int64_t out_off) {
  __shared__ float acc[kTile][kTile + 1];
  __shared__ float scratch[kThreads / 64][64];
  __shared__ int s_p;
  const int tile = t0 + (int)blockIdx.x;
  if (threadIdx.x == 0) {
    int p = 0;
    while (p + 1 < d.np && d.patches[p + 1].tile0 <= tile) ++p;
    s_p = p;
  }
  for (int c = threadIdx.x; c < kTile * (kTile + 1); c += kThreads) (&acc[0][0])[c] = 0.f;
  __syncthreads();
  const int p = s_p;
  const PatchDev &P = d.patches[p];
  const StepPatch W = d.sp[p];
  const int64_t n = d.glob->n;
  const Rec *__restrict__ S = direct ? direct : (const Rec *)((n & 1) ? d.S1 : d.S0);
  const int lt = tile - P.tile0;
  const int i0 = (lt % P.ntx) * kTile, j0 = (lt / P.ntx) * kTile;
  const int tw = min(kTile, P.nx - i0), th = min(kTile, P.ny - j0);
  const int32_t dxu = P.dxu;
  const int64_t X0 = ((int64_t)W.wx + i0) * dxu + dxu / 2;
  const int64_t Y0 = ((int64_t)W.wy + j0) * dxu + dxu / 2;
  const float inv_dxu = 1.0f / (float)dxu;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nwaves = kThreads / 64;
  float *scr = scratch[wave];

  for (int b = 0; b < d.nb; ++b) {
    const float rc = d.bucket_r[b] / (float)P.dx;   // radius in cells
    int need = (int)floorf(2.f * rc) + 2;
    int lg = 0;
    while ((1 << lg) < need && lg < 6) ++lg;
    const int G = 1 << lg, ppw = 64 >> lg;
    const int grp = lane >> lg, gl = lane & (G - 1);
    const float kpi = 3.14159265358979f / rc;
    // bin rows / columns whose crests can reach the tile
    int nrange, by_lo = 0, bx_lo = 0, bx_hi = 0, row0 = 0;
    if (direct) {
      nrange = 1;
    } else {
      const int32_t m = d.margin[b];
      const int32_t binu = P.binu[b];
      const int64_t ax0 = (int64_t)i0 * dxu + dxu / 2;
      const int64_t ay0 = (int64_t)j0 * dxu + dxu / 2;
      bx_lo = (int)(ax0 / binu);
      bx_hi = min(P.nbx[b] - 1, (int)((ax0 + (int64_t)(tw - 1) * dxu + 2 * (int64_t)m) / binu));
      by_lo = (int)(ay0 / binu);
      const int by_hi = min(P.nby[b] - 1, (int)((ay0 + (int64_t)(th - 1) * dxu + 2 * (int64_t)m) / binu));
      nrange = (bx_lo <= bx_hi && by_lo <= by_hi) ? by_hi - by_lo + 1 : 0;
      row0 = P.binbase[b];
    }
    for (int rr = 0; rr < nrange; ++rr) {
      int lo, hi;
      if (direct) {
        lo = 0;
        hi = ndirect;
      } else {
        const int rb = row0 + (by_lo + rr) * P.nbx[b];
        lo = min(d.off[rb + bx_lo], d.cap);
        hi = min(d.off[rb + bx_hi + 1], d.cap);
      }
      for (int k0 = lo + wave * ppw; k0 < hi; k0 += nwaves * ppw) {
        const int k = k0 + grp;
        bool valid = k < hi;
        float cx = 0.f, cy = 0.f, A = 0.f;
        float2 u = make_float2(0.f, 0.f);
        if (valid) {
          const Part q = RecIO<Rec>::load(S, k, n);
          if ((int)m_bucket(q.meta) != b || (int)m_patch(q.meta) != p) {
            valid = false;
          } else {
            const int2 v = d.V[b * kNCode + q.code];
            const int64_t px = (int64_t)q.ox + (((int64_t)q.age * v.x) >> 12);
            const int64_t py = (int64_t)q.oy + (((int64_t)q.age * v.y) >> 12);
            cx = (float)(px - X0) * inv_dxu;
            cy = (float)(py - Y0) * inv_dxu;
            A = particle_amp<Rec>(d, q);
            u = d.UC[q.code];
          }
        }
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
          const float ccx = pass ? cx - rc * u.x : cx;
          const float ccy = pass ? cy - rc * u.y : cy;
          const float amp = pass ? -A : A;
          int nr = 0, nc = 0, ilo = 0, jlo = 0;
          if (valid) {
            ilo = max(0, (int)ceilf(ccx - rc));
            const int ihi = min(tw - 1, (int)floorf(ccx + rc));
            jlo = max(0, (int)ceilf(ccy - rc));
            const int jhi = min(th - 1, (int)floorf(ccy + rc));
            if (ihi >= ilo && jhi >= jlo) {
              nc = ihi - ilo + 1;
              nr = jhi - jlo + 1;
            }
          }
          for (int jj = gl; jj < nr; jj += G)
            scr[grp * G + jj] = 0.5f + 0.5f * cosf(kpi * ((float)(jlo + jj) - ccy));
          wave_fence();
          for (int ii = gl; ii < nc; ii += G) {
            const float wx = amp * (0.5f + 0.5f * cosf(kpi * ((float)(ilo + ii) - ccx)));
            float *col = &acc[jlo][ilo + ii];
            for (int jj = 0; jj < nr; ++jj) atomicAdd(col + jj * (kTile + 1), wx * scr[grp * G + jj]);
          }
          wave_fence();
        }
      }
    }
  }
  __syncthreads();

  // blend epilogue
  const float dx = (float)P.dx;
  const int N = d.N;
  for (int c = threadIdx.x; c < kTile * kTile; c += kThreads) {
    const int i = c % kTile, j = c / kTile;
    if (i >= tw || j >= th) continue;
    const float h = acc[j][i];
    const int ci = i0 + i, cj = j0 + j;
    const size_t o = (size_t)(P.cell0 - out_off) + (size_t)cj * P.nx + ci;
    raw_out[o] = h;
    if (blend_out) {
      const float dd = fminf(fminf((float)ci + 0.5f, (float)P.nx - (float)ci - 0.5f),
                             fminf((float)cj + 0.5f, (float)P.ny - (float)cj - 0.5f)) * dx;
      const float t = fminf(dd / P.band, 1.f);
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
  }
}

void launch_splat_tiles(const Dev &d, int t0, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return;
  if (d.compact)
    hipLaunchKernelGGL(k_splat<RecCompact>, dim3(ntiles), dim3(kThreads), 0, st, d, t0,
                       (const RecCompact *)nullptr, 0, d.raw, d.blend, (int64_t)0);
  else
    hipLaunchKernelGGL(k_splat<RecWide>, dim3(ntiles), dim3(kThreads), 0, st, d, t0, (const RecWide *)nullptr, 0,
                       d.raw, d.blend, (int64_t)0);
}

void launch_splat_direct(const Dev &d, int t0, int ntiles, const void *recs, int n, float *raw,
                         int64_t out_off, hipStream_t st) {
  if (ntiles <= 0) return;
  if (d.compact)
    hipLaunchKernelGGL(k_splat<RecCompact>, dim3(ntiles), dim3(kThreads), 0, st, d, t0,
                       (const RecCompact *)recs, n, raw, (float *)nullptr, out_off);
  else
    hipLaunchKernelGGL(k_splat<RecWide>, dim3(ntiles), dim3(kThreads), 0, st, d, t0, (const RecWide *)recs, n,
                       raw, (float *)nullptr, out_off);
}

}  // namespace hwo

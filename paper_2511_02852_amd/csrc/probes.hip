// probes.hip -- object-receives-water sampling (Sec 4.3): height and unit
// normal of the current frame at world points, for buoyancy probes.
//
// A probe inside the cell-centre hull of a patch (the first such patch)
// reads that patch's blended map, else the periodic background.  Height is
// bilinear; the slopes are central differences at the four surrounding grid
// points (one-sided at a patch's first and last row or column), interpolated
// the same way; the normal is (-sx, -sy, 1) normalised.  One thread per
// probe; patch positions are resolved in FP64 like the rest of the frame.
#include <hip/hip_runtime.h>

#include "hwo_dev.h"

namespace hwo {

namespace {

__device__ __forceinline__ void slopes_at(const float *h, int nx, int ny, bool periodic, int i, int j, float inv_dx,
                                          float &sx, float &sy) {
  if (periodic) {
    const int a = (i + nx - 1) % nx, b = (i + 1) % nx;
    sx = (h[(size_t)j * nx + b] - h[(size_t)j * nx + a]) * 0.5f * inv_dx;
    const int c = (j + ny - 1) % ny, e = (j + 1) % ny;
    sy = (h[(size_t)e * nx + i] - h[(size_t)c * nx + i]) * 0.5f * inv_dx;
    return;
  }
  sx = 0.f;
  sy = 0.f;
  if (nx > 1) {
    const int a = i > 0 ? i - 1 : i, b = i < nx - 1 ? i + 1 : i;
    sx = (h[(size_t)j * nx + b] - h[(size_t)j * nx + a]) * inv_dx / (float)(b - a);
  }
  if (ny > 1) {
    const int a = j > 0 ? j - 1 : j, b = j < ny - 1 ? j + 1 : j;
    sy = (h[(size_t)b * nx + i] - h[(size_t)a * nx + i]) * inv_dx / (float)(b - a);
  }
}

__global__ __launch_bounds__(kThreads) void k_probes(Dev d, const double2 *__restrict__ xy, int n,
                                                     float4 *__restrict__ out) {
  const int q = blockIdx.x * kThreads + threadIdx.x;
  if (q >= n) return;
  const double x = xy[q].x, y = xy[q].y;
  const float *h = d.H;
  int nx = d.N, ny = d.N, i0 = 0, j0 = 0;
  float fx = 0.f, fy = 0.f, inv_dx = (float)(1.0 / d.dxf);
  bool periodic = true;
  for (int p = 0; p < d.np; ++p) {
    const PatchDev &P = d.patches[p];
    const StepPatch &W = d.sp[p];
    const double u = (x - P.ax) * 1048576.0 / (double)P.dxu - (double)W.wx - 0.5;
    const double v = (y - P.ay) * 1048576.0 / (double)P.dxu - (double)W.wy - 0.5;
    if (u >= 0.0 && v >= 0.0 && u <= (double)(P.nx - 1) && v <= (double)(P.ny - 1)) {
      h = d.blend + P.cell0;
      nx = P.nx;
      ny = P.ny;
      inv_dx = (float)(1.0 / P.dx);
      periodic = false;
      i0 = min((int)floor(u), max(nx - 2, 0));
      j0 = min((int)floor(v), max(ny - 2, 0));
      fx = (float)(u - (double)i0);
      fy = (float)(v - (double)j0);
      break;
    }
  }
  if (periodic) {
    const double u = x / d.dxf, v = y / d.dxf;
    const double fu = floor(u), fv = floor(v);
    fx = (float)(u - fu);
    fy = (float)(v - fv);
    const int64_t N = d.N;
    i0 = (int)((((int64_t)fu % N) + N) % N);
    j0 = (int)((((int64_t)fv % N) + N) % N);
  }
  float hv = 0.f, sxv = 0.f, syv = 0.f;
#pragma unroll
  for (int dj = 0; dj < 2; ++dj)
#pragma unroll
    for (int di = 0; di < 2; ++di) {
      int i = i0 + di, j = j0 + dj;
      if (periodic) {
        i %= nx;
        j %= ny;
      } else {
        i = min(i, nx - 1);
        j = min(j, ny - 1);
      }
      const float w = (di ? fx : 1.f - fx) * (dj ? fy : 1.f - fy);
      float sx, sy;
      slopes_at(h, nx, ny, periodic, i, j, inv_dx, sx, sy);
      hv = fmaf(w, h[(size_t)j * nx + i], hv);
      sxv = fmaf(w, sx, sxv);
      syv = fmaf(w, sy, syv);
    }
  const float inv = 1.0f / sqrtf(1.f + sxv * sxv + syv * syv);
  out[q] = make_float4(hv, -sxv * inv, -syv * inv, inv);
}

}  // namespace

void launch_probes(const Dev &d, const void *xy, int n, void *out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_probes, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, d, (const double2 *)xy, n,
                     (float4 *)out);
}

}  // namespace hwo

// Overlap-weighted stitch of tile logits into a whole-slide plane, or the
// paper's majority vote of binary tile predictions.
//
// The paper merges overlapping tile predictions back into a slide-sized map
// per tissue type (Sections 2.2 and 2.3).  Here each pixel p takes the
// weighted mean of the logits of the kept tiles that cover it,
// Lambda(p) = N(p) / D(p), N = sum_t w_t(p) l_t(p - o_t), D = sum_t w_t(p),
// with the separable ramp w(i, j) = r(i) r(j), r(i) = min(i + 1, T - i); the
// mask is N(p) > 0.  The sum is a gather over the at most ceil(T/s)^2 tiles
// covering p, in (jy, jx) order: no atomics, deterministic.  N is summed in
// FP32 with Neumaier compensation; D is an exact integer.  Vote mode (the
// merge of Section 2.2, thresholds of Section 3.2): the mask is on where at
// least `vote` of the covering tiles predict the class (logit > 0); the
// optional logit plane receives the vote count.
#include "internal.h"

namespace omniseg {

__device__ __forceinline__ void stitch_pixel(const StitchArgs& a, int x, int y) {
  const int T = a.T, s = a.s;
  const int jy0 = (y < T) ? 0 : (y - T) / s + 1, jy1 = min(a.ny - 1, y / s);
  const int jx0 = (x < T) ? 0 : (x - T) / s + 1, jx1 = min(a.nx - 1, x / s);
  if (a.vote > 0) {
    // majority vote: count the covering tiles whose logit is positive
    int votes = 0, cover = 0;
    for (int jy = jy0; jy <= jy1; ++jy) {
      const int iy = y - jy * s;
      for (int jx = jx0; jx <= jx1; ++jx) {
        const int t = a.index[jy * a.nx + jx];
        if (t < 0) continue;
        const int ix = x - jx * s;
        votes += a.logits[(int64_t)t * a.tile_stride + a.slot_off + (int64_t)iy * T + ix] > 0.f ? 1 : 0;
        ++cover;
      }
    }
    bool m = cover > 0 && votes >= a.vote;
    if (a.fg) m = m && a.fg[(int64_t)(y >> a.fg_shift) * a.Wc + (x >> a.fg_shift)];
    a.mask[(int64_t)y * a.mask_pitch + x] = m ? 1 : 0;
    if (a.logit) a.logit[(int64_t)y * a.logit_pitch + x] = (float)votes;
    return;
  }
  float sum = 0.f, comp = 0.f;
  int den = 0;
  for (int jy = jy0; jy <= jy1; ++jy) {
    const int iy = y - jy * s;
    const int ry = min(iy + 1, T - iy);
    for (int jx = jx0; jx <= jx1; ++jx) {
      const int t = a.index[jy * a.nx + jx];
      if (t < 0) continue;
      const int ix = x - jx * s;
      const int w = ry * min(ix + 1, T - ix);
      const float v = (float)w * a.logits[(int64_t)t * a.tile_stride + a.slot_off + (int64_t)iy * T + ix];
      const float t2 = sum + v;
      comp += (fabsf(sum) >= fabsf(v)) ? ((sum - t2) + v) : ((v - t2) + sum);
      sum = t2;
      den += w;
    }
  }
  const float n = sum + comp;
  bool m = (den > 0) && (a.coverage || n > 0.f);
  if (a.fg) m = m && a.fg[(int64_t)(y >> a.fg_shift) * a.Wc + (x >> a.fg_shift)];
  a.mask[(int64_t)y * a.mask_pitch + x] = m ? 1 : 0;
  if (a.logit) a.logit[(int64_t)y * a.logit_pitch + x] = den > 0 ? n / (float)den : 0.f;
}

// One thread per pixel; rows beyond the grid's y extent are taken in strides.
__global__ __launch_bounds__(256) void k_stitch(StitchArgs a) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= a.Wk) return;
  for (int y = blockIdx.y; y < a.Hk; y += gridDim.y) stitch_pixel(a, x, y);
}

hipError_t launch_stitch(const StitchArgs& a, hipStream_t st) {
  if (a.Hk <= 0 || a.Wk <= 0) return hipSuccess;
  dim3 grid(ceil_div(a.Wk, 256), std::min(a.Hk, kMaxGridY));
  hipLaunchKernelGGL(k_stitch, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// index grid [ny][nx] = -1, then grid[jy][jx] = i for every listed tile i
__global__ void k_grid_fill(int32_t* grid, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) grid[i] = -1;
}
__global__ void k_grid_set(const int32_t* yx, int n_tiles, int ny, int nx, int32_t* grid) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n_tiles) {
    const int jy = yx[2 * i], jx = yx[2 * i + 1];
    if (jy >= 0 && jy < ny && jx >= 0 && jx < nx) grid[jy * nx + jx] = i;  // others are ignored
  }
}

hipError_t launch_grid_from_list(const int32_t* tile_yx, int n_tiles, int ny, int nx, int32_t* grid,
                                 hipStream_t st) {
  const int n = ny * nx;
  hipLaunchKernelGGL(k_grid_fill, dim3(ceil_div(n, 256)), dim3(256), 0, st, grid, n);
  if (n_tiles > 0)
    hipLaunchKernelGGL(k_grid_set, dim3(ceil_div(n_tiles, 256)), dim3(256), 0, st, tile_yx, n_tiles,
                       ny, nx, grid);
  return hipGetLastError();
}

}  // namespace omniseg

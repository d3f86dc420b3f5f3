// Slide-wise aggregation and mapping (Section 2.3; the per-class optimal
// magnifications are named in Section 1).
//
// Merge to 40x: each class's stitched result at its own scale k becomes one
// 40x mask.  NEAREST repeats the scale-k mask over 2^k x 2^k blocks.
// BILINEAR samples the scale-k logit plane at the 40x pixel centres
// (source coordinate max(0, (y + 0.5) / 2^k - 0.5), neighbours clamped to
// the plane) and thresholds the value at 0.  The interpolation weights are
// dyadic fractions, exact in FP32.
//
// Overlay: every class whose mask is on at a pixel blends its colour into
// the 40x RGB, in class order, out = (out (256 - a) + colour a + 128) >> 8
// per channel (a in [0, 256]; exact integers).  The optional 10x map is the
// rounded mean of each 4 x 4 block of the overlay that lies inside the
// slide, from the same thread that wrote the block.
#include <algorithm>

#include "internal.h"

namespace omniseg {

__device__ __forceinline__ uint8_t merge_pixel(const MergePlane& p, int y, int x) {
  const int k = p.k;
  if (p.bilinear) {
    const float inv = 1.0f / (float)(2 << k);  // 1 / 2^(k+1), exact
    const float sy = fmaxf(0.f, (float)(2 * y + 1 - (1 << k)) * inv);
    const float sx = fmaxf(0.f, (float)(2 * x + 1 - (1 << k)) * inv);
    const int y0 = (int)sy, x0 = (int)sx;
    const int y1 = min(y0 + 1, p.Hk - 1), x1 = min(x0 + 1, p.Wk - 1);
    const float ly = sy - (float)y0, lx = sx - (float)x0;
    const float* r0 = p.logit + (int64_t)y0 * p.pitch;
    const float* r1 = p.logit + (int64_t)y1 * p.pitch;
    const float top = (1.f - lx) * r0[x0] + lx * r0[x1];
    const float bot = (1.f - lx) * r1[x0] + lx * r1[x1];
    return ((1.f - ly) * top + ly * bot) > 0.f ? 1 : 0;
  }
  return p.mask[(int64_t)(y >> k) * p.pitch + (x >> k)] ? 1 : 0;
}

// Four consecutive pixels of one row, bilinear: the sixteen logit reads are
// issued before any is used (same arithmetic per pixel as merge_pixel).
__device__ __forceinline__ uint32_t merge4_bilinear(const MergePlane& p, int y, int x0) {
  const int k = p.k;
  const float inv = 1.0f / (float)(2 << k);
  const float sy = fmaxf(0.f, (float)(2 * y + 1 - (1 << k)) * inv);
  const int y0 = (int)sy;
  const int y1 = min(y0 + 1, p.Hk - 1);
  const float ly = sy - (float)y0;
  const float* r0 = p.logit + (int64_t)y0 * p.pitch;
  const float* r1 = p.logit + (int64_t)y1 * p.pitch;
  int c0[4], c1[4];
  float lx[4], v[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float sx = fmaxf(0.f, (float)(2 * (x0 + q) + 1 - (1 << k)) * inv);
    c0[q] = (int)sx;
    c1[q] = min(c0[q] + 1, p.Wk - 1);
    lx[q] = sx - (float)c0[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q][0] = r0[c0[q]];
    v[q][1] = r0[c1[q]];
    v[q][2] = r1[c0[q]];
    v[q][3] = r1[c1[q]];
  }
  uint32_t out = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float top = (1.f - lx[q]) * v[q][0] + lx[q] * v[q][1];
    const float bot = (1.f - lx[q]) * v[q][2] + lx[q] * v[q][3];
    out |= (((1.f - ly) * top + ly * bot) > 0.f ? 1u : 0u) << (8 * q);
  }
  return out;
}

// One thread per four consecutive 40x pixels: one 4-byte store when the
// plane's output rows allow it (vec4), else four byte stores.
__global__ __launch_bounds__(256) void k_merge_base(MergeArgs a) {
  const MergePlane& p = a.plane[blockIdx.z];
  const int x0 = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (x0 >= a.W) return;
  for (int y = blockIdx.y; y < a.H; y += gridDim.y) {
    uint8_t* o = p.out + (int64_t)y * p.out_pitch + x0;
    if (p.vec4 && x0 + 3 < a.W) {
      uint32_t v;
      if (p.bilinear) {
        v = merge4_bilinear(p, y, x0);
      } else {
        v = (uint32_t)merge_pixel(p, y, x0) | ((uint32_t)merge_pixel(p, y, x0 + 1) << 8) |
            ((uint32_t)merge_pixel(p, y, x0 + 2) << 16) | ((uint32_t)merge_pixel(p, y, x0 + 3) << 24);
      }
      *reinterpret_cast<uint32_t*>(o) = v;
    } else {
      for (int q = 0; q < 4 && x0 + q < a.W; ++q) o[q] = merge_pixel(p, y, x0 + q);
    }
  }
}

hipError_t launch_merge_base(const MergeArgs& a, int n_planes, hipStream_t st) {
  if (n_planes <= 0 || a.H <= 0 || a.W <= 0) return hipSuccess;
  const dim3 grid(ceil_div(a.W, 1024), std::min(a.H, kMaxGridY), n_planes);
  hipLaunchKernelGGL(k_merge_base, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// One thread per 4 x 4 block of the 40x slide.
__global__ __launch_bounds__(256) void k_overlay(OverlayArgs a) {
  const int bx = blockIdx.x * 256 + threadIdx.x;
  const int Wb = (a.W + 3) >> 2, Hb = (a.H + 3) >> 2;
  if (bx >= Wb) return;
  for (int by = blockIdx.y; by < Hb; by += gridDim.y) {
    int sum[3] = {0, 0, 0}, cnt = 0;
    const bool full = a.vec && 4 * bx + 3 < a.W;
    for (int i = 0; i < 4; ++i) {
      const int y = 4 * by + i;
      if (y >= a.H) break;
      const uint8_t* src = a.rgb + (int64_t)y * a.pitch;
      uint8_t* dst = a.out + (int64_t)y * a.out_pitch;
      if (full) {
        // the block's 4 pixels of this row: 12 bytes, three aligned words
        const uint32_t* s4 = reinterpret_cast<const uint32_t*>(src + 12 * bx);
        const uint32_t w3[3] = {s4[0], s4[1], s4[2]};
        int px[4][3];
#pragma unroll
        for (int b = 0; b < 12; ++b) px[b / 3][b % 3] = (int)((w3[b / 4] >> (8 * (b % 4))) & 0xFFu);
        for (int c = 0; c < a.n; ++c) {
          const OverlayClass& oc = a.cls[c];
          const uint8_t* mrow = oc.mask + (int64_t)(y >> oc.k) * oc.pitch;
          uint32_t on;
          if (oc.k == 0 && oc.vec4) {
            on = *reinterpret_cast<const uint32_t*>(mrow + 4 * bx);
          } else {
            on = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) on |= (uint32_t)mrow[(4 * bx + q) >> oc.k] << (8 * q);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (!((on >> (8 * q)) & 0xFFu)) continue;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
              px[q][ch] = (px[q][ch] * (256 - oc.alpha) + oc.rgb[ch] * oc.alpha + 128) >> 8;
          }
        }
        uint32_t o3[3] = {0u, 0u, 0u};
#pragma unroll
        for (int b = 0; b < 12; ++b) {
          o3[b / 4] |= (uint32_t)px[b / 3][b % 3] << (8 * (b % 4));
          sum[b % 3] += px[b / 3][b % 3];
        }
        uint32_t* d4 = reinterpret_cast<uint32_t*>(dst + 12 * bx);
        d4[0] = o3[0];
        d4[1] = o3[1];
        d4[2] = o3[2];
        cnt += 4;
        continue;
      }
      for (int j = 0; j < 4; ++j) {
        const int x = 4 * bx + j;
        if (x >= a.W) break;
        int px[3] = {src[3 * x], src[3 * x + 1], src[3 * x + 2]};
        for (int c = 0; c < a.n; ++c) {
          const OverlayClass& oc = a.cls[c];
          if (!oc.mask[(int64_t)(y >> oc.k) * oc.pitch + (x >> oc.k)]) continue;
          for (int ch = 0; ch < 3; ++ch) px[ch] = (px[ch] * (256 - oc.alpha) + oc.rgb[ch] * oc.alpha + 128) >> 8;
        }
        for (int ch = 0; ch < 3; ++ch) {
          dst[3 * x + ch] = (uint8_t)px[ch];
          sum[ch] += px[ch];
        }
        ++cnt;
      }
    }
    if (a.out10) {
      uint8_t* d = a.out10 + (int64_t)by * a.out10_pitch + 3 * bx;
      for (int ch = 0; ch < 3; ++ch) d[ch] = (uint8_t)((sum[ch] + cnt / 2) / cnt);
    }
  }
}

hipError_t launch_overlay(const OverlayArgs& a, hipStream_t st) {
  if (a.H <= 0 || a.W <= 0) return hipSuccess;
  const int Wb = (a.W + 3) >> 2, Hb = (a.H + 3) >> 2;
  const dim3 grid(ceil_div(Wb, 256), std::min(Hb, kMaxGridY));
  hipLaunchKernelGGL(k_overlay, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace omniseg

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

// The bilinear blend of one 40x pixel from its four neighbours; every path
// below goes through this one expression, so they agree bit for bit.
__device__ __forceinline__ uint32_t blend_positive(float v00, float v01, float v10, float v11, float lx,
                                                   float ly) {
  const float top = (1.f - lx) * v00 + lx * v01;
  const float bot = (1.f - lx) * v10 + lx * v11;
  return ((1.f - ly) * top + ly * bot) > 0.f ? 1u : 0u;
}

// Source coordinate of 40x index i at scale k: max(0, (i + 0.5) / 2^k - 0.5),
// computed as (2 i + 1 - 2^k) / 2^(k+1), exact in FP32 for i < 2^23.
__device__ __forceinline__ float source_coord(int i, int k) {
  const float inv = ldexpf(1.0f, -(k + 1));  // 1 / 2^(k+1), exact
  return fmaxf(0.f, (float)(2 * i + 1 - (1 << k)) * inv);
}

__device__ __forceinline__ uint8_t merge_pixel(const MergePlane& p, int y, int x) {
  const int k = p.k;
  if (p.bilinear) {
    const float sy = source_coord(y, k), sx = source_coord(x, k);
    const int y0 = (int)sy, x0 = (int)sx;
    const int y1 = min(y0 + 1, p.Hk - 1), x1 = min(x0 + 1, p.Wk - 1);
    const float* r0 = p.logit + (int64_t)y0 * p.pitch;
    const float* r1 = p.logit + (int64_t)y1 * p.pitch;
    return (uint8_t)blend_positive(r0[x0], r0[x1], r1[x0], r1[x1], sx - (float)x0, sy - (float)y0);
  }
  return p.mask[(int64_t)(y >> k) * p.pitch + (x >> k)] ? 1 : 0;
}

// Four consecutive pixels of one row, bilinear: the sixteen logit reads are
// issued before any is used.
__device__ __forceinline__ uint32_t merge4_bilinear(const MergePlane& p, int y, int x0) {
  const int k = p.k;
  const float sy = source_coord(y, k);
  const int y0 = (int)sy;
  const int y1 = min(y0 + 1, p.Hk - 1);
  const float ly = sy - (float)y0;
  const float* r0 = p.logit + (int64_t)y0 * p.pitch;
  const float* r1 = p.logit + (int64_t)y1 * p.pitch;
  int c0[4], c1[4];
  float lx[4], v[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float sx = source_coord(x0 + q, k);
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
  for (int q = 0; q < 4; ++q) out |= blend_positive(v[q][0], v[q][1], v[q][2], v[q][3], lx[q], ly) << (8 * q);
  return out;
}

// Sixteen consecutive pixels x0 .. x0 + 15 (x0 a multiple of 16) at scale
// K <= 3.  Their source columns form one run: for pixel q the left
// neighbour is column (x0 >> K) + floor((2 q + 1 - 2^K) / 2^(K+1)) and the
// right one the next column, so the run starts at (x0 >> K) - (K > 0) and
// holds 16 / 2^K + 1 + (K > 0) columns.  The caller guarantees that the run
// lies inside the plane and that no clamp applies (x0 >= 16 when K > 0), so
// each pixel reads exactly the columns merge_pixel reads.
template <int K>
struct Run16 {
  static constexpr int lo = K > 0 ? -1 : 0;
  static constexpr int n = (16 >> K) + 1 + (K > 0 ? 1 : 0);
  static constexpr int left(int q) {  // index of pixel q's left neighbour in the run
    const int num = 2 * q + 1 - (1 << K), den = 2 << K;
    return (num >= 0 ? num / den : -((-num + den - 1) / den)) - lo;
  }
};

// Loads the run's n columns of one row.  VEC: the row start is 16-byte
// aligned, so the middle 16 / 2^K columns (which start at x0 >> K, a
// multiple of 16 / 2^K) go as one to four vector loads.
template <int K, bool VEC>
__device__ __forceinline__ void load_run(const float* row, int base, float (&v)[Run16<K>::n]) {
  constexpr int mid = 16 >> K, lo = Run16<K>::lo;
  if constexpr (VEC) {
    if constexpr (lo < 0) v[0] = row[base - 1];
    const float* m = row + base;
    if constexpr (mid >= 4) {
#pragma unroll
      for (int j = 0; j < mid; j += 4) {
        const float4 f = *reinterpret_cast<const float4*>(m + j);
        v[j - lo] = f.x;
        v[j + 1 - lo] = f.y;
        v[j + 2 - lo] = f.z;
        v[j + 3 - lo] = f.w;
      }
    } else {
      const float2 f = *reinterpret_cast<const float2*>(m);
      v[-lo] = f.x;
      v[1 - lo] = f.y;
    }
    v[mid - lo] = row[base + mid];
  } else {
#pragma unroll
    for (int j = 0; j < Run16<K>::n; ++j) v[j] = row[base + lo + j];
  }
}

// One 16-byte store marked non-temporal: the 40x masks are written once and
// are larger than the caches, so they stream to HBM without displacing the
// logit rows still being read.
__device__ __forceinline__ void store16_stream(uint8_t* dst, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = {w0, w1, w2, w3};
  __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(dst));
}

// A band of rows [ylo, yhi) of sixteen pixels, bilinear.  Rows are taken
// in order, so the source row pair (y0, y1) either repeats (k > 0) or moves
// down by one, and then the old y1 row is the new y0 row: each source row of
// the band is loaded once.  The horizontal weights depend on the column only.
template <int K, bool VEC>
__device__ __forceinline__ void merge16_bilinear_band(const MergePlane& p, int ylo, int yhi, int x0) {
  using R = Run16<K>;
  const int base = x0 >> K;
  float lx[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const float sx = source_coord(x0 + q, K);
    lx[q] = sx - (float)(int)sx;
  }
  float a[R::n], b[R::n];
  int cy0 = -1, cy1 = -1;
  for (int y = ylo; y < yhi; ++y) {
    const float sy = source_coord(y, K);
    const int y0 = (int)sy;
    const int y1 = min(y0 + 1, p.Hk - 1);
    const float ly = sy - (float)y0;
    if (y0 != cy0) {
      if (y0 == cy1) {
#pragma unroll
        for (int j = 0; j < R::n; ++j) a[j] = b[j];
      } else {
        load_run<K, VEC>(p.logit + (int64_t)y0 * p.pitch, base, a);
      }
      load_run<K, VEC>(p.logit + (int64_t)y1 * p.pitch, base, b);
      cy0 = y0;
      cy1 = y1;
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = R::left(q);
      w[q >> 2] |= blend_positive(a[c], a[c + 1], b[c], b[c + 1], lx[q], ly) << (8 * (q & 3));
    }
    store16_stream(p.out + (int64_t)y * p.out_pitch + x0, w[0], w[1], w[2], w[3]);
  }
}

// The 16 / 2^K source bytes of one mask row at x0 >> K.  VEC: the row start
// is 16-byte aligned.
template <int K, bool VEC>
__device__ __forceinline__ void load_mask_run(const uint8_t* src, uint8_t (&s)[16 >> K]) {
  constexpr int n = 16 >> K;
  if constexpr (VEC && n == 16) {
    const uint4 f = *reinterpret_cast<const uint4*>(src);
    const uint32_t u[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
    for (int j = 0; j < 16; ++j) s[j] = (uint8_t)(u[j >> 2] >> (8 * (j & 3)));
  } else if constexpr (VEC && n == 8) {
    const uint2 f = *reinterpret_cast<const uint2*>(src);
    const uint32_t u[2] = {f.x, f.y};
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] = (uint8_t)(u[j >> 2] >> (8 * (j & 3)));
  } else if constexpr (VEC && n == 4) {
    const uint32_t u = *reinterpret_cast<const uint32_t*>(src);
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = (uint8_t)(u >> (8 * j));
  } else {
#pragma unroll
    for (int j = 0; j < n; ++j) s[j] = src[j];
  }
}

// A band of rows, nearest: each source byte repeated 2^K times across and
// its row 2^K times down (loaded once per source row).
template <int K, bool VEC>
__device__ __forceinline__ void merge16_nearest_band(const MergePlane& p, int ylo, int yhi, int x0) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  int cur = -1;
  for (int y = ylo; y < yhi; ++y) {
    if ((y >> K) != cur) {
      cur = y >> K;
      uint8_t s[16 >> K];
      load_mask_run<K, VEC>(p.mask + (int64_t)cur * p.pitch + (x0 >> K), s);
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = 0u;
#pragma unroll
      for (int q = 0; q < 16; ++q) w[q >> 2] |= (s[q >> K] ? 1u : 0u) << (8 * (q & 3));
    }
    store16_stream(p.out + (int64_t)y * p.out_pitch + x0, w[0], w[1], w[2], w[3]);
  }
}

// The run form for one plane at compile-time scale K (the band loop sits
// inside the scale switch, so each scale's column terms are hoisted out of
// its own loop only).
template <int K>
__device__ __forceinline__ void merge16_band(const MergePlane& p, int ylo, int yhi, int x0) {
  if (p.bilinear) {
    if (p.vec_src) merge16_bilinear_band<K, true>(p, ylo, yhi, x0);
    else merge16_bilinear_band<K, false>(p, ylo, yhi, x0);
  } else {
    if (p.vec_src) merge16_nearest_band<K, true>(p, ylo, yhi, x0);
    else merge16_nearest_band<K, false>(p, ylo, yhi, x0);
  }
}

// Whether the sixteen pixels from x0 take the run form: all inside the
// width, 16-byte output stores, and (bilinear) the source run inside the
// plane with no clamp at either end.
__device__ __forceinline__ bool run16_fits(const MergePlane& p, int W, int x0) {
  if (!p.vec16 || x0 + 15 >= W) return false;
  if (!p.bilinear) return true;
  const int base = x0 >> p.k;
  if (p.k > 0 && base < 1) return false;
  return base + (16 >> p.k) <= p.Wk - 1;
}

// One thread per sixteen consecutive 40x pixels in each row of a band of
// consecutive rows (blockIdx.y picks the band).  The run form stores the
// sixteen as one 16-byte word; elsewhere (the last pixels of a row, the
// first sixteen at k > 0, the right edge of the plane, unaligned outputs)
// they go four at a time: a 4-byte store when the output rows allow it
// (vec4), else byte stores.
__global__ __launch_bounds__(256) void k_merge_base(MergeArgs a) {
  const MergePlane& p = a.plane[blockIdx.z];
  const int x0 = (blockIdx.x * 256 + threadIdx.x) * 16;
  if (x0 >= a.W) return;
  const int rows = (a.H + gridDim.y - 1) / gridDim.y;
  const int ylo = blockIdx.y * rows, yhi = min(a.H, ylo + rows);
  if (run16_fits(p, a.W, x0)) {
    switch (p.k) {
      case 0: merge16_band<0>(p, ylo, yhi, x0); break;
      case 1: merge16_band<1>(p, ylo, yhi, x0); break;
      case 2: merge16_band<2>(p, ylo, yhi, x0); break;
      default: merge16_band<3>(p, ylo, yhi, x0); break;
    }
    return;
  }
  for (int y = ylo; y < yhi; ++y) {
    uint8_t* o = p.out + (int64_t)y * p.out_pitch + x0;
#pragma unroll 1
    for (int g = 0; g < 16; g += 4) {
      const int xg = x0 + g;
      if (xg >= a.W) break;
      if (p.vec4 && xg + 3 < a.W) {
        uint32_t v;
        if (p.bilinear) {
          v = merge4_bilinear(p, y, xg);
        } else {
          v = (uint32_t)merge_pixel(p, y, xg) | ((uint32_t)merge_pixel(p, y, xg + 1) << 8) |
              ((uint32_t)merge_pixel(p, y, xg + 2) << 16) | ((uint32_t)merge_pixel(p, y, xg + 3) << 24);
        }
        *reinterpret_cast<uint32_t*>(o + g) = v;
      } else {
        for (int q = 0; q < 4 && xg + q < a.W; ++q) o[g + q] = merge_pixel(p, y, xg + q);
      }
    }
  }
}

// Bands of at least eight consecutive rows (a bilinear band reuses its
// source rows), and at most about sixteen thousand workgroups in all.
constexpr int kMergeBlocks = 16384;
constexpr int kMergeMinRows = 8;

hipError_t launch_merge_base(const MergeArgs& a, int n_planes, hipStream_t st) {
  if (n_planes <= 0 || a.H <= 0 || a.W <= 0) return hipSuccess;
  const int gx = ceil_div(a.W, 4096);
  const int gy = std::max(1, std::min(ceil_div(a.H, kMergeMinRows), ceil_div(kMergeBlocks, gx * n_planes)));
  const dim3 grid(gx, gy, n_planes);
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

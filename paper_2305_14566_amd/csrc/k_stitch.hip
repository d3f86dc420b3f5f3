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

// Logit slot of list index t: t itself, or t % ring in a ring store.
__device__ __forceinline__ int64_t tile_slot(const StitchArgs& a, int t) {
  return a.ring > 0 ? (int64_t)(t % a.ring) : (int64_t)t;
}

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
        votes += a.logits[tile_slot(a, t) * a.tile_stride + a.slot_off + (int64_t)iy * T + ix] > 0.f ? 1 : 0;
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
      const float v = (float)w * a.logits[tile_slot(a, t) * a.tile_stride + a.slot_off + (int64_t)iy * T + ix];
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

// Four consecutive outputs of row y at x0 (x0 a multiple of 4), gated by the
// tissue mask.  Output rows need no alignment: with an odd pitch, say, every
// other row starts off a 4-byte boundary, and such a row is written byte by
// byte (a float logit plane: element by element off a 16-byte boundary).
// The test is per row, so it is uniform across a wave.
__device__ __forceinline__ void store4(const StitchArgs& a, int x0, int y, bool (&m)[4], const float (&out)[4]) {
  if (a.fg) {
    const uint8_t* fr = a.fg + (int64_t)(y >> a.fg_shift) * a.Wc;
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = m[q] && fr[(x0 + q) >> a.fg_shift];
  }
  uint8_t* mp = a.mask + (int64_t)y * a.mask_pitch + x0;
  if ((reinterpret_cast<uintptr_t>(mp) & 3) == 0) {
    *reinterpret_cast<uint32_t*>(mp) =
        (m[0] ? 1u : 0u) | (m[1] ? 1u << 8 : 0u) | (m[2] ? 1u << 16 : 0u) | (m[3] ? 1u << 24 : 0u);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) mp[q] = m[q] ? 1 : 0;
  }
  if (a.logit) {
    float* lp = a.logit + (int64_t)y * a.logit_pitch + x0;
    if ((reinterpret_cast<uintptr_t>(lp) & 15) == 0) {
      *reinterpret_cast<float4*>(lp) = make_float4(out[0], out[1], out[2], out[3]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) lp[q] = out[q];
    }
  }
}

// Four consecutive pixels x0 .. x0 + 3 (x0 a multiple of 4, all inside the
// row) when the stride and the tile size are multiples of 4: the four share
// their covering tiles, and each tile's four logits are one aligned 16-byte
// load.  Per pixel the arithmetic and its order are those of stitch_pixel.
__device__ __forceinline__ void stitch_span4(const StitchArgs& a, int x0, int y) {
  const int T = a.T, s = a.s;
  const int jy0 = (y < T) ? 0 : (y - T) / s + 1, jy1 = min(a.ny - 1, y / s);
  const int jx0 = (x0 < T) ? 0 : (x0 - T) / s + 1, jx1 = min(a.nx - 1, x0 / s);
  float out[4];
  bool m[4];
  if (a.vote > 0) {
    int votes[4] = {0, 0, 0, 0}, cover = 0;
    for (int jy = jy0; jy <= jy1; ++jy) {
      const int iy = y - jy * s;
      for (int jx = jx0; jx <= jx1; ++jx) {
        const int t = a.index[jy * a.nx + jx];
        if (t < 0) continue;
        const int ix = x0 - jx * s;
        const float4 l =
            *reinterpret_cast<const float4*>(a.logits + tile_slot(a, t) * a.tile_stride + a.slot_off + (int64_t)iy * T + ix);
        votes[0] += l.x > 0.f ? 1 : 0;
        votes[1] += l.y > 0.f ? 1 : 0;
        votes[2] += l.z > 0.f ? 1 : 0;
        votes[3] += l.w > 0.f ? 1 : 0;
        ++cover;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      m[q] = cover > 0 && votes[q] >= a.vote;
      out[q] = (float)votes[q];
    }
  } else {
    float sum[4] = {0.f, 0.f, 0.f, 0.f}, comp[4] = {0.f, 0.f, 0.f, 0.f};
    int den[4] = {0, 0, 0, 0};
    for (int jy = jy0; jy <= jy1; ++jy) {
      const int iy = y - jy * s;
      const int ry = min(iy + 1, T - iy);
      for (int jx = jx0; jx <= jx1; ++jx) {
        const int t = a.index[jy * a.nx + jx];
        if (t < 0) continue;
        const int ix = x0 - jx * s;
        const float4 l4 =
            *reinterpret_cast<const float4*>(a.logits + tile_slot(a, t) * a.tile_stride + a.slot_off + (int64_t)iy * T + ix);
        const float l[4] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int w = ry * min(ix + q + 1, T - ix - q);
          const float v = (float)w * l[q];
          const float t2 = sum[q] + v;
          comp[q] += (fabsf(sum[q]) >= fabsf(v)) ? ((sum[q] - t2) + v) : ((v - t2) + sum[q]);
          sum[q] = t2;
          den[q] += w;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float n = sum[q] + comp[q];
      m[q] = (den[q] > 0) && (a.coverage || n > 0.f);
      out[q] = den[q] > 0 ? n / (float)den[q] : 0.f;
    }
  }
  store4(a, x0, y, m, out);
}

// Buffer resource of `bytes` bytes at p (raw buffer loads, 32-bit offsets).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const float* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)bytes, 0x00020000);
}

// The covering tiles of four pixels x0 .. x0 + 3 in the rows of one tile-row
// band (at most 2 x 2 tiles): their slots' buffer resources and in-tile
// column.  A missing tile's resource has an empty range, so its reads
// return zeros without touching memory.
struct Cover2x2 {
  int jy0, jx0;
  bool have[2][2];
  __amdgpu_buffer_rsrc_t r[2][2];
  int ix[2];
};

__device__ __forceinline__ Cover2x2 cover_2x2(const StitchArgs& a, int x0, int y) {
  const int T = a.T, s = a.s;
  Cover2x2 c;
  c.jy0 = (y < T) ? 0 : (y - T) / s + 1;
  const int jy1 = min(a.ny - 1, y / s);
  c.jx0 = (x0 < T) ? 0 : (x0 - T) / s + 1;
  const int jx1 = min(a.nx - 1, x0 / s);
  int t[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const bool in = c.jy0 + u <= jy1 && c.jx0 + v <= jx1;
      const int ti = a.index[min(c.jy0 + u, jy1) * a.nx + min(c.jx0 + v, jx1)];
      t[u][v] = in ? ti : -1;
    }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int tt = t[u][v];
      c.have[u][v] = tt >= 0;
      c.r[u][v] = tile_rsrc(a.logits + tile_slot(a, max(tt, 0)) * a.tile_stride,
                            tt >= 0 ? (uint32_t)(a.tile_stride * 4) : 0u);
    }
#pragma unroll
  for (int v = 0; v < 2; ++v) c.ix[v] = x0 - (c.jx0 + v) * s;
  return c;
}

__device__ __forceinline__ void load_2x2(const StitchArgs& a, const Cover2x2& c, int y, float4 (&L)[2][2]) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int iy = y - (c.jy0 + u) * a.s;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const uint32_t off = (uint32_t)(a.slot_off + (int64_t)iy * a.T + c.ix[v]) * 4u;
      L[u][v] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(c.r[u][v], c.have[u][v] ? off : 0u,
                                                                                 0, 0));
    }
  }
}

// Mask (and logit or vote count) of pixels x0 .. x0 + 3 of row y from the
// logits of their covering tiles, in (jy, jx) order.
__device__ __forceinline__ void finish_2x2(const StitchArgs& a, const Cover2x2& c, int x0, int y,
                                           const float4 (&L)[2][2]) {
  const int T = a.T;
  float out[4];
  bool m[4];
  if (a.vote > 0) {
    int votes[4] = {0, 0, 0, 0}, cover = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (!c.have[u][v]) continue;
        const float4 l = L[u][v];
        votes[0] += l.x > 0.f ? 1 : 0;
        votes[1] += l.y > 0.f ? 1 : 0;
        votes[2] += l.z > 0.f ? 1 : 0;
        votes[3] += l.w > 0.f ? 1 : 0;
        ++cover;
      }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      m[q] = cover > 0 && votes[q] >= a.vote;
      out[q] = (float)votes[q];
    }
  } else {
    float sum[4] = {0.f, 0.f, 0.f, 0.f}, comp[4] = {0.f, 0.f, 0.f, 0.f};
    int den[4] = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int iy = y - (c.jy0 + u) * a.s;
      const int ry = min(iy + 1, T - iy);
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (!c.have[u][v]) continue;
        const int ix = c.ix[v];
        const float l[4] = {L[u][v].x, L[u][v].y, L[u][v].z, L[u][v].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int w = ry * min(ix + q + 1, T - ix - q);
          const float vv = (float)w * l[q];
          const float t2 = sum[q] + vv;
          comp[q] += (fabsf(sum[q]) >= fabsf(vv)) ? ((sum[q] - t2) + vv) : ((vv - t2) + sum[q]);
          sum[q] = t2;
          den[q] += w;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float n = sum[q] + comp[q];
      m[q] = (den[q] > 0) && (a.coverage || n > 0.f);
      out[q] = den[q] > 0 ? n / (float)den[q] : 0.f;
    }
  }
  store4(a, x0, y, m, out);
}

// stitch_span4 when T <= 2 s, so at most 2 x 2 tiles cover a pixel: the four
// index reads, then the four logit-vector reads, are issued together, and
// the covering tiles are then taken in the same (jy, jx) order with the same
// arithmetic.
__device__ __forceinline__ void stitch_span4_2x2(const StitchArgs& a, int x0, int y) {
  const Cover2x2 c = cover_2x2(a, x0, y);
  float4 L[2][2];
  load_2x2(a, c, y, L);
  finish_2x2(a, c, x0, y, L);
}

// Rows y0 .. y1 - 1 at columns x0 .. x0 + 3, rows that share their covering
// tiles (one tile-row band): the index reads are done once, and two rows'
// logit reads are in flight together.  Per pixel as stitch_span4_2x2.
__device__ __forceinline__ void stitch_rows4_2x2(const StitchArgs& a, int x0, int y0, int y1) {
  const Cover2x2 c = cover_2x2(a, x0, y0);
  int y = y0;
  for (; y + 1 < y1; y += 2) {
    float4 L0[2][2], L1[2][2];
    load_2x2(a, c, y, L0);
    load_2x2(a, c, y + 1, L1);
    finish_2x2(a, c, x0, y, L0);
    finish_2x2(a, c, x0, y + 1, L1);
  }
  if (y < y1) {
    float4 L0[2][2];
    load_2x2(a, c, y, L0);
    finish_2x2(a, c, x0, y, L0);
  }
}

// One thread per pixel; rows beyond the grid's y extent are taken in strides.
__global__ __launch_bounds__(256) void k_stitch(StitchArgs a) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= a.Wk) return;
  for (int y = blockIdx.y; y < a.Hk; y += gridDim.y) stitch_pixel(a, x, y);
}

// The first row after y at which the covering tiles of a row can change:
// the next multiple of s (the last covering tile row, y / s) or the next
// T + k s (the first, (y - T) / s + 1).
__device__ __forceinline__ int cover_change(int y, int T, int s) {
  const int a = (y / s + 1) * s;
  const int b = y < T ? T : T + ((y - T) / s + 1) * s;
  return min(a, b);
}

// One thread per four pixels (see stitch_span4) in each row of a band of
// consecutive rows (blockIdx.y picks the band); the row's ragged end goes
// pixel by pixel.  TWO: at most 2 x 2 covering tiles (T <= 2 s); the band is
// then cut where the covering tiles change, and each piece reads its tile
// indices once (stitch_rows4_2x2).
template <bool TWO>
__global__ __launch_bounds__(256) void k_stitch4(StitchArgs a) {
  const int x0 = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (x0 >= a.Wk) return;
  const int rows = (a.Hk + gridDim.y - 1) / gridDim.y;
  const int ylo = blockIdx.y * rows, yhi = min(a.Hk, ylo + rows);
  if (x0 + 3 < a.Wk) {
    if (TWO) {
      for (int y = ylo; y < yhi;) {
        const int ye = min(yhi, cover_change(y, a.T, a.s));
        stitch_rows4_2x2(a, x0, y, ye);
        y = ye;
      }
    } else {
      for (int y = ylo; y < yhi; ++y) stitch_span4(a, x0, y);
    }
  } else {
    for (int y = ylo; y < yhi; ++y)
      for (int x = x0; x < a.Wk; ++x) stitch_pixel(a, x, y);
  }
}

// Bands of up to eight rows, as long as the launch keeps at least about
// four thousand workgroups (a small plane goes row by row).
constexpr int kStitchMinBlocks = 4096;
constexpr int kStitchBandRows = 8;

hipError_t launch_stitch(const StitchArgs& a, hipStream_t st) {
  if (a.Hk <= 0 || a.Wk <= 0) return hipSuccess;
  // the four-pixel form needs shared covering tiles (s, T multiples of 4) and
  // aligned vector reads of the tile logits (output rows may have any
  // alignment, see store4)
  const bool span4 = a.s % 4 == 0 && a.T % 4 == 0 && a.tile_stride % 4 == 0 && a.slot_off % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(a.logits) % 16 == 0 &&
                     (!a.logit || reinterpret_cast<uintptr_t>(a.logit) % 4 == 0);
  if (span4) {
    const int gx = ceil_div(a.Wk, 1024);
    const int gy = std::min(a.Hk, std::max(ceil_div(a.Hk, kStitchBandRows), ceil_div(kStitchMinBlocks, gx)));
    dim3 grid(gx, gy);
    // a logit plane's float offsets inside a tile must fit the 32-bit byte
    // offsets of the buffer loads
    if (a.T <= 2 * a.s && a.tile_stride * 4 <= INT32_MAX)
      hipLaunchKernelGGL(k_stitch4<true>, grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(k_stitch4<false>, grid, dim3(256), 0, st, a);
  } else {
    dim3 grid(ceil_div(a.Wk, 256), std::min(a.Hk, kMaxGridY));
    hipLaunchKernelGGL(k_stitch, grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

// ---- streamed stitch --------------------------------------------------------

__global__ __launch_bounds__(256) void k_stream_units(StreamStitchArgs a) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u > a.n_units) return;
  StreamUnit out;
  if (u == a.n_units) {  // sentinel after the last unit: the item count
    out.batch = INT32_MAX;
    out.g = a.n_groups;
    out.y0 = out.y1 = 0;
    out.item_base = a.n_items;
    a.units[u] = out;
    return;
  }
  // the group of the unit: the last one whose first unit is <= u (every group
  // has at least one tile row, so the first units increase)
  int lo = 0, hi = a.n_groups - 1;
  while (lo < hi) {
    const int m = (lo + hi + 1) >> 1;
    if (a.groups[m].unit_base <= u) lo = m;
    else hi = m - 1;
  }
  const StreamGroup& G = a.groups[lo];
  const int j = u - G.unit_base;
  const int pos_end = a.pre[G.grid_base + (int64_t)(j + 1) * G.nx];
  out.batch = pos_end > 0 ? (pos_end - 1) / a.B : 0;
  out.g = lo;
  out.y0 = j * G.s;
  out.y1 = j == G.ny - 1 ? G.Hk : (j + 1) * G.s;
  // every row of the group before this unit's is a full row of s rows
  out.item_base = G.item_base + (int64_t)G.n_planes * G.nxc * j * ((G.s + kStitchRows - 1) / kStitchRows);
  a.units[u] = out;
}

// batch_first[b] = the first unit stitched after batch b or later: for each
// unit u, the batches after its predecessor's up to its own (the sentinel
// closes the table at n_units).
__global__ __launch_bounds__(256) void k_batch_first(StreamStitchArgs a) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u > a.n_units) return;
  const int b0 = u == 0 ? 0 : a.units[u - 1].batch + 1;
  const int b1 = min(a.units[u].batch, a.n_batches);
  for (int b = b0; b <= b1; ++b) a.batch_first[b] = u;
}

hipError_t launch_stream_units(const StreamStitchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_stream_units, dim3(ceil_div(a.n_units + 1, 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_batch_first, dim3(ceil_div(a.n_units + 1, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

static_assert(kStitchCols == 4 * 256, "one pass of four pixels per thread covers an item's columns");

// Every unit of batch a.batch: a fixed grid takes the units' items
// (one plane, kStitchRows rows, kStitchCols columns) in turn; per pixel the
// arithmetic and its order are those of the plane-wise stitch.
__global__ __launch_bounds__(256) void k_stitch_stream(StreamStitchArgs a) {
  __shared__ int s_u;
  const int u_lo = a.batch_first[a.batch], u_hi = a.batch_first[a.batch + 1];
  if (u_lo >= u_hi) return;
  const int64_t i_hi = a.units[u_hi].item_base;
  int cur = u_lo;
  for (int64_t it = a.units[u_lo].item_base + blockIdx.x; it < i_hi; it += gridDim.x) {
    __syncthreads();  // every thread has read s_u of the previous item
    if (threadIdx.x == 0) {
      // the item's unit: the last one in [cur, u_hi) whose first item is <= it
      int lo = cur, hi = u_hi - 1;
      while (lo < hi) {
        const int m = (lo + hi + 1) >> 1;
        if (a.units[m].item_base <= it) lo = m;
        else hi = m - 1;
      }
      s_u = lo;
    }
    __syncthreads();
    cur = s_u;
    const StreamUnit un = a.units[cur];
    const StreamGroup& G = a.groups[un.g];
    const int nblk = (un.y1 - un.y0 + kStitchRows - 1) / kStitchRows;
    const int local = (int)(it - un.item_base);
    const int per_plane = nblk * G.nxc;
    const StreamPlane& P = a.planes[G.plane_first + local / per_plane];
    const int rem = local % per_plane;
    const int xa = (rem % G.nxc) * kStitchCols, xb = min(G.Wk, xa + kStitchCols);
    StitchArgs sa;
    sa.logits = a.logits;
    sa.tile_stride = a.tile_stride;
    sa.slot_off = P.slot_off;
    sa.index = a.index + G.grid_base;
    sa.ny = G.ny;
    sa.nx = G.nx;
    sa.T = a.T;
    sa.s = G.s;
    sa.Hk = G.Hk;
    sa.Wk = G.Wk;
    sa.mask = P.mask;
    sa.mask_pitch = P.mask_pitch;
    sa.logit = P.logit;
    sa.logit_pitch = P.logit_pitch;
    sa.fg = G.fg;
    sa.fg_shift = G.fg_shift;
    sa.Hc = G.Hc;
    sa.Wc = G.Wc;
    sa.coverage = 0;
    sa.vote = G.vote;
    sa.ring = a.ring;
    const int r0 = un.y0 + (rem / G.nxc) * kStitchRows, r1 = min(un.y1, r0 + kStitchRows);
    // rows of one tile-row band share their covering tiles
    const bool band = P.mode == 2 && (r0 < a.T ? 0 : (r0 - a.T) / sa.s + 1) ==
                                         (r1 - 1 < a.T ? 0 : (r1 - 1 - a.T) / sa.s + 1) &&
                      min(sa.ny - 1, r0 / sa.s) == min(sa.ny - 1, (r1 - 1) / sa.s);
    if (band) {
      const int x0 = xa + threadIdx.x * 4;
      if (x0 + 3 < xb) {
        stitch_rows4_2x2(sa, x0, r0, r1);
      } else {
        for (int y = r0; y < r1; ++y)
          for (int x = x0; x < xb; ++x) stitch_pixel(sa, x, y);
      }
      continue;
    }
    for (int y = r0; y < r1; ++y) {
      if (P.mode == 0) {
        for (int x = xa + threadIdx.x; x < xb; x += 256) stitch_pixel(sa, x, y);
        continue;
      }
      // four pixels per thread: kStitchCols = 4 x 256 columns in one pass
      const int x0 = xa + threadIdx.x * 4;
      if (x0 + 3 < xb) {
        if (P.mode == 2) stitch_span4_2x2(sa, x0, y);
        else stitch_span4(sa, x0, y);
      } else {
        for (int x = x0; x < xb; ++x) stitch_pixel(sa, x, y);
      }
    }
  }
}

hipError_t launch_stitch_stream(const StreamStitchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_stitch_stream, dim3(2048), dim3(256), 0, st, a);
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

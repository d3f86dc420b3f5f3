// Slide preparation kernels: pad colour, box-sum pyramid, tissue map,
// per-tile tissue flags and the compaction into the ordered tile list.
//
// Pad colour: the rounded mean of the slide's top-left 2x2 block (paper
// Section 2.1, repeated in Section 3.2), round half up.  Pyramid: scale k
// holds the integer sums of 2^k x 2^k blocks of the padded 40x slide (the
// paper tiles 40x, 10x and 5x views of each region, Section 2.2); sums fit
// uint16 for k <= 3.  Tissue map: the coarsest scale's block mean is tissue
// when its gray value 0.299 R + 0.587 G + 0.114 B is below a threshold,
// tested exactly in integers (blank-region removal, Section 2.1).
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace omniseg {

__global__ void k_pad_colour(const uint8_t* __restrict__ rgb, int64_t pitch, int32_t* pad) {
  int c = threadIdx.x;
  if (c < 3) {
    int s = rgb[c] + rgb[3 + c] + rgb[pitch + c] + rgb[pitch + 3 + c];
    pad[c] = (s + 2) >> 2;
  } else if (c == 3) {
    pad[3] = 0;
  }
}

hipError_t launch_pad_colour(const uint8_t* rgb, int64_t pitch, int32_t* pad, hipStream_t st) {
  hipLaunchKernelGGL(k_pad_colour, dim3(1), dim3(64), 0, st, rgb, pitch, pad);
  return hipGetLastError();
}

// One thread per 2^kmax x 2^kmax block of the padded base.  Level k sums are
// formed from level k-1 sums (nested box sums are exact integer identities).
struct PyrArgs {
  const uint8_t* rgb;
  int64_t pitch;
  int H, W;
  const int32_t* pad;
  int kmax;
  uint16_t* lvl[4];  // index k (lvl[0] unused)
  int Ey[4], Ex[4];
  int nby, nbx;      // block grid
};

template <int KMAX>
__device__ __forceinline__ void pyramid_block(const PyrArgs& a, int bx, int by) {
  constexpr int F = 1 << KMAX;
  const int p0 = a.pad[0], p1 = a.pad[1], p2 = a.pad[2];
  // level-1 sums of this block: (F/2) x (F/2) x 3
  int s1[F / 2][F / 2][3];
#pragma unroll
  for (int i = 0; i < F / 2; ++i)
#pragma unroll
    for (int j = 0; j < F / 2; ++j) s1[i][j][0] = s1[i][j][1] = s1[i][j][2] = 0;
  const int y0 = by * F, x0 = bx * F;
#pragma unroll
  for (int r = 0; r < F; ++r) {
    const int y = y0 + r;
    const bool rin = y < a.H;
    const uint8_t* row = a.rgb + (int64_t)y * a.pitch;
#pragma unroll
    for (int c = 0; c < F; ++c) {
      const int x = x0 + c;
      int v0 = p0, v1 = p1, v2 = p2;
      if (rin && x < a.W) {
        v0 = row[3 * x];
        v1 = row[3 * x + 1];
        v2 = row[3 * x + 2];
      }
      s1[r >> 1][c >> 1][0] += v0;
      s1[r >> 1][c >> 1][1] += v1;
      s1[r >> 1][c >> 1][2] += v2;
    }
  }
  // write level 1, then fold into coarser levels in place
#pragma unroll
  for (int k = 1; k <= KMAX; ++k) {
    const int n = F >> k;  // pixels of level k per block side
    if (a.lvl[k]) {
      const int ly0 = by * n, lx0 = bx * n;
#pragma unroll
      for (int i = 0; i < F / 2; ++i) {
#pragma unroll
        for (int j = 0; j < F / 2; ++j) {
          const int yy = ly0 + i, xx = lx0 + j;
          if (i < n && j < n && yy < a.Ey[k] && xx < a.Ex[k]) {
            ushort4 v;
            v.x = (uint16_t)s1[i][j][0];
            v.y = (uint16_t)s1[i][j][1];
            v.z = (uint16_t)s1[i][j][2];
            v.w = 0;
            reinterpret_cast<ushort4*>(a.lvl[k])[(int64_t)yy * a.Ex[k] + xx] = v;
          }
        }
      }
    }
    if (k < KMAX) {
      // in-place 2x2 fold; row-major order never overwrites an unread input
#pragma unroll
      for (int i = 0; i < F / 4; ++i)
#pragma unroll
        for (int j = 0; j < F / 4; ++j)
#pragma unroll
          for (int ch = 0; ch < 3; ++ch)
            if (i < (n >> 1) && j < (n >> 1))
              s1[i][j][ch] = s1[2 * i][2 * j][ch] + s1[2 * i][2 * j + 1][ch] +
                             s1[2 * i + 1][2 * j][ch] + s1[2 * i + 1][2 * j + 1][ch];
    }
  }
}

// Block rows beyond the grid's y extent (65535 at most) are taken in strides.
template <int KMAX>
__global__ __launch_bounds__(256) void k_pyramid(PyrArgs a) {
  const int bx = blockIdx.x * blockDim.x + threadIdx.x;
  if (bx >= a.nbx) return;
  for (int by = blockIdx.y; by < a.nby; by += gridDim.y) pyramid_block<KMAX>(a, bx, by);
}

hipError_t launch_pyramid(const uint8_t* rgb, int64_t pitch, int H, int W, const int32_t* pad,
                          int kmax, uint16_t* const* lvl, const int* Ey, const int* Ex,
                          hipStream_t st) {
  if (kmax < 1) return hipSuccess;
  PyrArgs a{};
  a.rgb = rgb;
  a.pitch = pitch;
  a.H = H;
  a.W = W;
  a.pad = pad;
  a.kmax = kmax;
  int ny = 0, nx = 0;
  for (int k = 0; k < 4; ++k) {
    a.lvl[k] = (k >= 1 && k <= kmax) ? lvl[k] : nullptr;
    a.Ey[k] = Ey[k];
    a.Ex[k] = Ex[k];
    if (a.lvl[k]) {
      // blocks needed to cover the level-k extent
      int f = 1 << (kmax - k);
      ny = std::max(ny, ceil_div(Ey[k], f));
      nx = std::max(nx, ceil_div(Ex[k], f));
    }
  }
  a.nby = ny;
  a.nbx = nx;
  if (ny == 0) return hipSuccess;
  dim3 grid(ceil_div(nx, 256), std::min(ny, kMaxGridY));
  switch (kmax) {
    case 1: hipLaunchKernelGGL(k_pyramid<1>, grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_pyramid<2>, grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL(k_pyramid<3>, grid, dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

// Tissue map at scale kc for y < Hc, x < Wc.
__global__ void k_tissue(const uint8_t* __restrict__ rgb, int64_t pitch,
                         const uint16_t* __restrict__ sums, int ex, int kc, int Hc, int Wc,
                         int64_t limit, uint8_t* __restrict__ fg) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= Wc) return;
  for (int y = blockIdx.y; y < Hc; y += gridDim.y) {
    int64_t r, g, b;
    if (kc == 0) {
      const uint8_t* p = rgb + (int64_t)y * pitch + 3 * x;
      r = p[0];
      g = p[1];
      b = p[2];
    } else {
      ushort4 v = reinterpret_cast<const ushort4*>(sums)[(int64_t)y * ex + x];
      r = v.x;
      g = v.y;
      b = v.z;
    }
    int64_t gray = 299 * r + 587 * g + 114 * b;
    fg[(int64_t)y * Wc + x] = gray < limit ? 1 : 0;
  }
}

hipError_t launch_tissue(const uint8_t* rgb, int64_t pitch, int H, int W, const int32_t* pad,
                         const uint16_t* sums_kc, int ex_kc, int kc, int Hc, int Wc, int thr,
                         uint8_t* fg, hipStream_t st) {
  (void)H;
  (void)W;
  (void)pad;
  int64_t limit = (int64_t)thr * 1000 * ((int64_t)1 << (2 * kc));
  dim3 grid(ceil_div(Wc, 256), std::min(Hc, kMaxGridY));
  hipLaunchKernelGGL(k_tissue, grid, dim3(256), 0, st, rgb, pitch, sums_kc, ex_kc, kc, Hc, Wc,
                     limit, fg);
  return hipGetLastError();
}

// One workgroup per grid tile: keep it iff some tissue-map pixel overlaps its
// 40x footprint (coarse row r covers 40x rows [r 2^kc, (r+1) 2^kc), the tile
// covers [jy s 2^k, (jy s + T) 2^k)).
__global__ __launch_bounds__(256) void k_tile_flags(TileGroups g, const SlideDev* slides, int T,
                                                    int kc, int fg_filter, int32_t* flags) {
  const int t = blockIdx.x;
  int gi = 0;
  while (gi + 1 < g.n && g.base[gi + 1] <= t) ++gi;
  if (!fg_filter) {
    if (threadIdx.x == 0) flags[t] = 1;
    return;
  }
  const int local = t - g.base[gi];
  const int nx = g.nx[gi];
  const int s = g.s[gi];
  const int jy = local / nx, jx = local % nx;
  const int k = g.k[gi];
  const SlideDev& sd = slides[(int)g.slide[gi]];
  const int sh = kc - k;  // 2^kc / 2^k
  // rows r with r 2^kc < (jy s + T) 2^k and (r+1) 2^kc > jy s 2^k
  const int r0 = (jy * s) >> sh;
  const int r1 = min(sd.Hc, ((jy * s + T) + (1 << sh) - 1) >> sh);
  const int c0 = (jx * s) >> sh;
  const int c1 = min(sd.Wc, ((jx * s + T) + (1 << sh) - 1) >> sh);
  const int w = c1 - c0;
  int found = 0;
  if (w > 0 && r1 > r0) {
    const int n = (r1 - r0) * w;
    for (int i = threadIdx.x; i < n && !found; i += blockDim.x) {
      const int rr = r0 + i / w, cc = c0 + i % w;
      found |= sd.fg[(int64_t)rr * sd.Wc + cc];
    }
  }
  found = __syncthreads_or(found);
  if (threadIdx.x == 0) flags[t] = found ? 1 : 0;
}

hipError_t launch_tile_flags(const TileGroups& g, const SlideDev* slides_dev, int T, int kc,
                             int fg_filter, int32_t* flags, hipStream_t st) {
  int total = g.base[g.n];
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_flags, dim3(total), dim3(256), 0, st, g, slides_dev, T, kc, fg_filter, flags);
  return hipGetLastError();
}

// Single-workgroup ordered compaction: flags (0/1 per grid tile, canonical
// order) become list indices (-1 for dropped tiles); kept tiles are appended
// to the list as (slide, slot, jy, jx) in canonical order.  pre[t] (total + 1
// entries) is the number of kept tiles before grid tile t, so the kept tiles
// of grid tiles [a, b) are the list positions [pre[a], pre[b]).
__global__ __launch_bounds__(1024) void k_compact(int32_t* idx, int total, TileGroups g,
                                                  int4* list, int32_t* count, int32_t* pre) {
  __shared__ int wave_tot[16];
  __shared__ int run;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) run = 0;
  __syncthreads();
  int gi = 0;
  for (int t0 = 0; t0 < total; t0 += 1024) {
    const int t = t0 + threadIdx.x;
    const int f = (t < total) ? idx[t] : 0;
    const uint64_t bal = __ballot(f != 0);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wave] = __popcll(bal);
    __syncthreads();
    int off = run;
    for (int w = 0; w < wave; ++w) off += wave_tot[w];
    if (t < total) {
      pre[t] = off + before;
      if (f) {
        const int pos = off + before;
        while (gi + 1 < g.n && g.base[gi + 1] <= t) ++gi;
        const int local = t - g.base[gi];
        list[pos] = make_int4(g.slide[gi], g.slot[gi], local / g.nx[gi], local % g.nx[gi]);
        idx[t] = pos;
      } else {
        idx[t] = -1;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int s = 0;
      for (int w = 0; w < 16; ++w) s += wave_tot[w];
      run += s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *count = run;
    pre[total] = run;
  }
}

// launch_put: one workgroup per payload of kPutWords words.  The payload
// travels in the kernel arguments (so a captured graph holds the data, not a
// host pointer); 224 words keep the argument segment near 1 KB, well inside
// the 4 KB limit (a 3.5 KB payload crashed rocprofv3's counter collection
// on the host).
constexpr int kPutWords = 224;
struct PutPayload {
  uint32_t w[kPutWords];
};
__global__ __launch_bounds__(256) void k_put(uint32_t* dst, int n, PutPayload p) {
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = p.w[i];
}

hipError_t launch_put(void* dst, const void* src, int64_t bytes, hipStream_t st) {
  if (bytes % 4) return hipErrorInvalidValue;
  const int64_t n = bytes / 4;
  for (int64_t o = 0; o < n; o += kPutWords) {
    PutPayload p;
    const int m = (int)std::min<int64_t>(kPutWords, n - o);
    memcpy(p.w, static_cast<const uint32_t*>(src) + o, (size_t)m * 4);
    hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, st, static_cast<uint32_t*>(dst) + o, m, p);
  }
  return hipGetLastError();
}

hipError_t launch_compact(int32_t* flags_to_index, int total, const TileGroups& g, int32_t* list,
                          int32_t* count, int32_t* pre, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, flags_to_index, total, g,
                     reinterpret_cast<int4*>(list), count, pre);
  return hipGetLastError();
}

}  // namespace omniseg

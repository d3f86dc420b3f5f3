// Otsu tissue detection on the coarsest scale (Section 2.1 tissue detection
// and blank-region removal; Section 3.2 names Otsu, a median blur and the
// foreground contour that removes small noise).
//
//   1. gray:   g = round((299 R + 587 G + 114 B) / (1000 4^kc)) of the
//              coarse block sums, an exact integer in [0, 255];
//   2. median: m x m median of g with replicated borders (m odd; 1 = none);
//   3. Otsu:   the 256-bin histogram of the blurred map and the threshold t
//              that maximises the between-class variance n0 n1 (mu0 - mu1)^2
//              (first maximum), evaluated in FP64 in a fixed operation order;
//   4. tissue: blurred value <= t (tissue is the darker class);
//   5. noise:  8-connected components of the tissue pixels with fewer than
//              min_area pixels are dropped.
//
// Every step is integer work except the Otsu score, whose comparison is
// taken in FP64 with the operations and order stated in k_otsu; the result
// is deterministic.  All kernels are sized from the map and exit on every
// path; the union-find loops end because parent links only point to
// smaller indices.
#include <algorithm>

#include "internal.h"

namespace omniseg {

// ---- 1. gray ----------------------------------------------------------------

__global__ __launch_bounds__(256) void k_gray8(const uint8_t* __restrict__ rgb, int64_t pitch,
                                               const uint16_t* __restrict__ sums, int ex, int kc, int Hc,
                                               int Wc, uint8_t* __restrict__ gray) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= Wc) return;
  const int64_t den = 1000LL << (2 * kc);
  for (int y = blockIdx.y; y < Hc; y += gridDim.y) {
    int64_t r, g, b;
    if (kc == 0) {
      const uint8_t* p = rgb + (int64_t)y * pitch + 3 * x;
      r = p[0];
      g = p[1];
      b = p[2];
    } else {
      const ushort4 v = reinterpret_cast<const ushort4*>(sums)[(int64_t)y * ex + x];
      r = v.x;
      g = v.y;
      b = v.z;
    }
    gray[(int64_t)y * Wc + x] = (uint8_t)((299 * r + 587 * g + 114 * b + den / 2) / den);
  }
}

// ---- 2. median ----------------------------------------------------------------
// One lane per output column and run of `rows` output rows.  The lane keeps
// the histogram of its m x m window in LDS (256 16-bit counts packed in 128
// words, word w of lane l at [w][l], so each lane only ever touches its own
// bank) and slides it down one row at a time: m values leave, m enter.  The
// median and the count of values below it are updated incrementally.

constexpr int kMedianLanes = 64;

__global__ __launch_bounds__(kMedianLanes) void k_median(const uint8_t* __restrict__ in, int Hc, int Wc, int m,
                                                         int rows, uint8_t* __restrict__ out) {
  __shared__ uint32_t hist[128][kMedianLanes];
  const int lane = threadIdx.x;
  const int x = blockIdx.x * kMedianLanes + lane;
  const int y0 = blockIdx.y * rows;
  if (x >= Wc || y0 >= Hc) return;
  const int r = m / 2;
  const int k0 = (m * m - 1) / 2;  // rank of the median, 0-based
  for (int w = 0; w < 128; ++w) hist[w][lane] = 0u;
  auto add = [&](int v, int d) { hist[v >> 1][lane] += (uint32_t)d << (16 * (v & 1)); };
  auto count = [&](int v) { return (int)((hist[v >> 1][lane] >> (16 * (v & 1))) & 0xFFFFu); };
  auto at = [&](int y, int xx) {
    y = min(max(y, 0), Hc - 1);
    xx = min(max(xx, 0), Wc - 1);
    return (int)in[(int64_t)y * Wc + xx];
  };
  for (int i = -r; i <= r; ++i)
    for (int j = -r; j <= r; ++j) add(at(y0 + i, x + j), 1);
  int med = 0, lt = 0;
  while (lt + count(med) <= k0) {
    lt += count(med);
    ++med;
  }
  out[(int64_t)y0 * Wc + x] = (uint8_t)med;
  const int y1 = min(y0 + rows, Hc);
  for (int y = y0 + 1; y < y1; ++y) {
    for (int j = -r; j <= r; ++j) {
      const int vo = at(y - r - 1, x + j), vi = at(y + r, x + j);
      add(vo, -1);
      lt -= vo < med ? 1 : 0;
      add(vi, 1);
      lt += vi < med ? 1 : 0;
    }
    // the window holds m^2 > k0 values, so both loops stop inside [0, 255]
    while (lt > k0) {
      --med;
      lt -= count(med);
    }
    while (lt + count(med) <= k0) {
      lt += count(med);
      ++med;
    }
    out[(int64_t)y * Wc + x] = (uint8_t)med;
  }
}

// ---- 3. histogram and Otsu threshold ------------------------------------------

__global__ __launch_bounds__(256) void k_hist256(const uint8_t* __restrict__ g, int64_t n, uint32_t* hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += step) atomicAdd(&h[g[i]], 1u);
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// One block of 256 threads: thread t scores the split {<= t} / {> t}.
// Otsu's score of the split {<= t} / {> t} is n0 n1 (mu0 - mu1)^2 =
// (N s0 - n0 S)^2 / (n0 n1).  With fewer than 2^28 pixels |N s0 - n0 S| <
// 2^64 and n0 n1 < 2^56, so two scores compare exactly as 192-bit products
// A_a^2 D_b against A_b^2 D_a; no floating point is involved.
struct U192 {
  uint64_t w0, w1, w2;  // least significant first
};

__device__ __forceinline__ U192 mul_u128_u64(unsigned __int128 a, uint64_t b) {
  const unsigned __int128 p0 = (unsigned __int128)(uint64_t)a * b;
  const unsigned __int128 p1 = (unsigned __int128)(uint64_t)(a >> 64) * b + (p0 >> 64);
  return U192{(uint64_t)p0, (uint64_t)p1, (uint64_t)(p1 >> 64)};
}

// score(a2a, da) > score(a2b, db), scores a2 / d with d > 0
__device__ __forceinline__ bool score_greater(unsigned __int128 a2a, uint64_t da, unsigned __int128 a2b, uint64_t db) {
  const U192 x = mul_u128_u64(a2a, db), y = mul_u128_u64(a2b, da);
  if (x.w2 != y.w2) return x.w2 > y.w2;
  if (x.w1 != y.w1) return x.w1 > y.w1;
  return x.w0 > y.w0;
}

// stats[0] receives the threshold (the first t of the largest score), or -1
// when every pixel has one value.
__global__ __launch_bounds__(256) void k_otsu(const uint32_t* __restrict__ hist, int32_t* stats) {
  __shared__ int64_t cn[256], cs[256];
  __shared__ unsigned __int128 best_a2[256];
  __shared__ uint64_t best_d[256];  // 0: no split at this t
  __shared__ int best_t[256];
  const int t = threadIdx.x;
  cn[t] = hist[t];
  cs[t] = (int64_t)hist[t] * t;
  __syncthreads();
  // inclusive prefix sums (Hillis-Steele), exact in int64
  for (int d = 1; d < 256; d <<= 1) {
    const int64_t a = t >= d ? cn[t - d] : 0, b = t >= d ? cs[t - d] : 0;
    __syncthreads();
    cn[t] += a;
    cs[t] += b;
    __syncthreads();
  }
  const int64_t N = cn[255], S = cs[255], n0 = cn[t], s0 = cs[t], n1 = N - n0;
  unsigned __int128 a2 = 0;
  uint64_t dd = 0;
  if (n0 > 0 && n1 > 0) {
    const __int128 A = (__int128)N * s0 - (__int128)n0 * S;
    const unsigned __int128 absA = (unsigned __int128)(A < 0 ? -A : A);
    a2 = absA * absA;
    dd = (uint64_t)n0 * (uint64_t)n1;
  }
  best_a2[t] = a2;
  best_d[t] = dd;
  best_t[t] = t;
  __syncthreads();
  // argmax, first index on ties; t without a split loses to any split
  for (int d = 128; d > 0; d >>= 1) {
    if (t < d) {
      const uint64_t od = best_d[t + d], cd = best_d[t];
      bool take = false;
      if (od != 0) {
        if (cd == 0) {
          take = true;
        } else {
          const bool gt = score_greater(best_a2[t + d], od, best_a2[t], cd);
          const bool lt = score_greater(best_a2[t], cd, best_a2[t + d], od);
          take = gt || (!lt && best_t[t + d] < best_t[t]);
        }
      }
      if (take) {
        best_a2[t] = best_a2[t + d];
        best_d[t] = od;
        best_t[t] = best_t[t + d];
      }
    }
    __syncthreads();
  }
  if (t == 0) stats[0] = best_d[0] == 0 ? -1 : best_t[0];
}

// ---- 4-5. tissue pixels and connected components ------------------------------

__device__ __forceinline__ int ld_parent(const int32_t* p, int i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// parent links point to smaller indices, so the walk ends at a root
__device__ __forceinline__ int find_root(const int32_t* parent, int x) {
  int p = ld_parent(parent, x);
  while (p != x) {
    x = p;
    p = ld_parent(parent, x);
  }
  return x;
}

// The same walk with path halving: each visited node is relinked to its
// grandparent.  A non-root never becomes a root again and the stored value
// is an ancestor of the node (smaller than it), so concurrent walks, links
// and relinks keep every parent pointer valid.
__device__ __forceinline__ int find_root_halving(int32_t* parent, int x) {
  while (true) {
    const int p = ld_parent(parent, x);
    if (p == x) return x;
    const int gp = ld_parent(parent, p);
    if (gp == p) return p;
    __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}

__global__ __launch_bounds__(256) void k_tissue_label(const uint8_t* __restrict__ g, const int32_t* stats,
                                                      int64_t n, int32_t* __restrict__ label) {
  const int t = stats[0];
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += step)
    label[i] = (int)g[i] <= t ? (int32_t)i : -1;
}

// Union of each tissue pixel with its tissue neighbours above and to the
// left (8-connectivity: up-left, up, up-right, left).  A link always hangs
// the larger root under the smaller one, so the final root of a component
// is its smallest pixel index whatever the order of the unions.  A failed
// CAS means the root gained a parent meanwhile, which happens at most once
// per root, so the retry loop ends; the bound below is never reached.
__global__ __launch_bounds__(256) void k_tissue_union(int32_t* label, int Hc, int Wc, int32_t* stats) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= Wc) return;
  for (int y = blockIdx.y; y < Hc; y += gridDim.y) {
    const int p = y * Wc + x;
    if (ld_parent(label, p) < 0) continue;
    const int nb[4][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}};
    for (int k = 0; k < 4; ++k) {
      const int yy = y + nb[k][0], xx = x + nb[k][1];
      if (yy < 0 || xx < 0 || xx >= Wc) continue;
      const int q = yy * Wc + xx;
      if (ld_parent(label, q) < 0) continue;
      int a = p, b = q;
      bool done = false;
      for (int it = 0; it < (1 << 24) && !done; ++it) {
        a = find_root_halving(label, a);
        b = find_root_halving(label, b);
        if (a == b) {
          done = true;
        } else {
          if (a < b) {
            const int c = a;
            a = b;
            b = c;
          }
          done = atomicCAS(label + a, a, b) == a;
        }
      }
      if (!done) atomicOr(stats + 3, 1);  // reported as an error by the host
    }
  }
}

// Every tissue pixel's label becomes its root (the forest no longer
// changes; a concurrent walk sees either the old parent or the root, both
// ancestors), and the root counts the pixel.
__global__ __launch_bounds__(256) void k_tissue_flatten(int32_t* label, int64_t n, int32_t* area,
                                                        int32_t* stats) {
  const int64_t step = (int64_t)gridDim.x * 256;
  const int64_t span = (n + step - 1) / step * step;  // whole waves iterate together
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < span; i += step) {
    int root = -1;
    if (i < n && ld_parent(label, (int)i) >= 0) {
      root = find_root_halving(label, (int)i);
      __hip_atomic_store(label + i, root, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (root == (int)i) atomicAdd(stats + 1, 1);
    }
    // One atomic for the lanes that share the first tissue lane's root (a
    // run of one component, the common case); the other lanes add alone.
    // Every lane of the wave reaches the ballots.
    const uint64_t tissue = __ballot(root >= 0);
    if (tissue == 0) continue;
    const int leader = __ffsll((unsigned long long)tissue) - 1;
    const int lroot = __shfl(root, leader);
    const uint64_t same = __ballot(root >= 0 && root == lroot);
    if (root >= 0 && root != lroot) atomicAdd(area + root, 1);
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(area + lroot, (int)__popcll(same));
  }
}

__global__ __launch_bounds__(256) void k_tissue_filter(const int32_t* __restrict__ label,
                                                       const int32_t* __restrict__ area, int64_t n, int min_area,
                                                       uint8_t* __restrict__ fg, int32_t* stats) {
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += step) {
    const int root = label[i];
    uint8_t keep = 0;
    if (root >= 0) {
      keep = area[root] >= min_area ? 1 : 0;
      if (keep && root == (int)i) atomicAdd(stats + 2, 1);
    }
    fg[i] = keep;
  }
}

hipError_t launch_tissue_otsu(const TissueOtsuArgs& a, hipStream_t st) {
  const int64_t n = (int64_t)a.Hc * a.Wc;
  if (n <= 0) return hipSuccess;
  const unsigned flat = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16);
  const dim3 rows(ceil_div(a.Wc, 256), std::min(a.Hc, kMaxGridY));
  hipLaunchKernelGGL(k_gray8, rows, dim3(256), 0, st, a.rgb, a.pitch, a.sums, a.ex, a.kc, a.Hc, a.Wc,
                     a.median > 1 ? a.tmp : a.gray);
  if (a.median > 1) {
    const int run = std::max(32, ceil_div(a.Hc, kMaxGridY));
    const dim3 grid(ceil_div(a.Wc, kMedianLanes), ceil_div(a.Hc, run));
    hipLaunchKernelGGL(k_median, grid, dim3(kMedianLanes), 0, st, a.tmp, a.Hc, a.Wc, a.median, run, a.gray);
  }
  hipError_t e = launch_zero(a.hist, 256 * 4, st);
  if (e == hipSuccess) e = launch_zero(a.stats, 16, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hist256, dim3(flat), dim3(256), 0, st, a.gray, n, a.hist);
  hipLaunchKernelGGL(k_otsu, dim3(1), dim3(256), 0, st, a.hist, a.stats);
  hipLaunchKernelGGL(k_tissue_label, dim3(flat), dim3(256), 0, st, a.gray, a.stats, n, a.label);
  hipLaunchKernelGGL(k_tissue_union, rows, dim3(256), 0, st, a.label, a.Hc, a.Wc, a.stats);
  e = launch_zero(a.area, n * 4, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tissue_flatten, dim3(flat), dim3(256), 0, st, a.label, n, a.area, a.stats);
  hipLaunchKernelGGL(k_tissue_filter, dim3(flat), dim3(256), 0, st, a.label, a.area, n, a.min_area, a.fg,
                     a.stats);
  return hipGetLastError();
}

}  // namespace omniseg

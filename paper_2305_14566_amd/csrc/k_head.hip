// Global average pool of the bottleneck, the controller and the dynamic head.
//
// The controller maps [g; onehot_C(class); onehot_S(scale)] to the P
// parameters of a per-(tile, class) head, theta = W_c v + b_c, where g is the
// bottleneck's pixel mean.  With one-hot inputs this is W_c[:, :G] g plus two
// columns of W_c plus b_c.  The head is three 1x1 convs on the 8-channel
// feature F: h1 = ReLU(W1 F + b1), h2 = ReLU(W2 h1 + b2), z = W3 h2 + b3, with
// theta split as W1 (8x8), W2 (8x8), W3 (o x 8), b1, b2, b3.  The class logit
// is z_0 for one output and z_1 - z_0 for two.  F = ReLU(W_p D_0 + b_p) when
// the decoder's last level has C_0 != 8 channels, else D_0 itself.  All head
// arithmetic is FP32 (with BF16 D_0 and C_0 <= 64 the precls product runs on
// MFMA with each weight split into three exact BF16 terms, see
// precls_bf16_mfma).  The precls weights and a tile's generated head
// parameters are the same for every thread of a workgroup, so the head reads
// them as scalar (constant-cache) loads and uses them as FMA operands.
#include "internal.h"

#include <type_traits>

namespace omniseg {

__device__ __forceinline__ float ld1(const float* p) { return *p; }
__device__ __forceinline__ float ld1(const uint16_t* p) { return __uint_as_float((uint32_t)(*p) << 16); }
// FP8: the E4M3 code's value (the caller applies the channel scale)
__device__ __forceinline__ float ld1(const uint8_t* p) { return __builtin_amdgcn_cvt_f32_fp8((int)*p, 0); }

// 16 bytes of a pixel row -> floats (4 FP32, 8 BF16 or 16 E4M3 code values)
__device__ __forceinline__ void decode16(uint4 u, float* v /*[4]*/, float) {
  v[0] = __uint_as_float(u.x);
  v[1] = __uint_as_float(u.y);
  v[2] = __uint_as_float(u.z);
  v[3] = __uint_as_float(u.w);
}
__device__ __forceinline__ void decode16(uint4 u, float* v /*[8]*/, uint16_t) {
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __uint_as_float(w[i] << 16);
    v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}
__device__ __forceinline__ void decode16(uint4 u, float* v /*[16]*/, uint8_t) {
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[4 * i] = __builtin_amdgcn_cvt_f32_fp8((int)w[i], 0);
    v[4 * i + 1] = __builtin_amdgcn_cvt_f32_fp8((int)w[i], 1);
    v[4 * i + 2] = __builtin_amdgcn_cvt_f32_fp8((int)w[i], 2);
    v[4 * i + 3] = __builtin_amdgcn_cvt_f32_fp8((int)w[i], 3);
  }
}
template <typename T, int N>
__device__ __forceinline__ void decode16(uint4 u, float (&v)[N]) {
  decode16(u, &v[0], T());
}

// Bottleneck mean per channel.  One workgroup per (tile, 64-channel block):
// lane l of wave w sums channel l over pixels w, w + 4, ... and the four
// partial sums are added in LDS.  scale: FP8 channel scales (null for FP32 /
// BF16).
template <typename T>
__global__ __launch_bounds__(256) void k_gap(const T* __restrict__ e, int hw, int c_p, int c,
                                             const int32_t* count, int chunk_base, float* g,
                                             const float* __restrict__ scale) {
  const int nblk = (c + 63) / 64;
  const int b = blockIdx.x / nblk, cb = blockIdx.x % nblk;
  if (chunk_base + b >= *count) return;
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ch = cb * 64 + lane;
  float s = 0.f;
  if (ch < c) {
    // four independent partial sums per lane keep four loads in flight
    const T* base = e + (int64_t)b * hw * c_p + ch;
    float s4[4] = {0.f, 0.f, 0.f, 0.f};
    int p = wave;
    for (; p + 12 < hw; p += 16)
#pragma unroll
      for (int u = 0; u < 4; ++u) s4[u] += ld1(base + (int64_t)(p + 4 * u) * c_p);
    for (; p < hw; p += 4) s4[0] += ld1(base + (int64_t)p * c_p);
    s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  }
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && ch < c) {
    float t = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    if constexpr (std::is_same<T, uint8_t>::value) t *= scale[ch];
    g[(int64_t)b * c_p + ch] = t / (float)hw;
  }
}

hipError_t launch_gap(int precision, const void* e, int batch, int hw, int c_p, int c,
                      const int32_t* count, int chunk_base, float* g, hipStream_t st, const float* scale) {
  const dim3 grid(batch * ((c + 63) / 64));
  if (precision == OMNISEG_FP8) {
    if (!scale) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gap<uint8_t>, grid, dim3(256), 0, st, (const uint8_t*)e, hw, c_p, c, count, chunk_base, g,
                       scale);
  } else if (precision == OMNISEG_BF16) {
    hipLaunchKernelGGL(k_gap<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)e, hw, c_p, c, count, chunk_base,
                       g, nullptr);
  } else {
    hipLaunchKernelGGL(k_gap<float>, grid, dim3(256), 0, st, (const float*)e, hw, c_p, c, count, chunk_base, g,
                       nullptr);
  }
  return hipGetLastError();
}

constexpr int kCtrlRows = 16;  // output rows of one controller workgroup (four per wave)

// theta[b][slot][p]; one workgroup per tile and group of kCtrlRows rows.  W_c rows are row_len =
// G + n_classes + n_scales long.  The GAP part u[p] = W_c[p, :G] g is the same
// for every class at the tile's scale, so it is formed once per tile and
// shared by the tile's slots (same addition order as per slot).
__global__ __launch_bounds__(256) void k_controller(const float* __restrict__ g, int g_stride, int G,
                                                     const float* __restrict__ wc,
                                                     const float* __restrict__ bc, int P, int row_len,
                                                     int n_classes, SlotTable slots, int max_slots,
                                                     const int32_t* list, const int32_t* count,
                                                     int chunk_base, float* theta) {
  const int b = blockIdx.x;
  if (chunk_base + b >= *count) return;
  const int si = list[4 * (chunk_base + b) + 1];
  const int ns = slots.n_slots[si];
  __shared__ float sg[4096];
  const float* gb = g + (int64_t)b * g_stride;
  for (int i = threadIdx.x; i < G; i += blockDim.x) sg[i] = gb[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // one wave per output row p (blockIdx.y selects a group of kCtrlRows rows):
  // coalesced reads of W_c's row, wave reduction
  const int p_end = min(P, (int)(blockIdx.y + 1) * kCtrlRows);
  for (int p = blockIdx.y * kCtrlRows + wave; p < p_end; p += 4) {
    const float* w = wc + (int64_t)p * row_len;
    float s = 0.f;
    // sixteen loads in flight, then the FMAs in the same order as one at a time
    int i = lane;
    for (; i + 15 * 64 < G; i += 16 * 64) {
      float wv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) wv[u] = w[i + u * 64];
#pragma unroll
      for (int u = 0; u < 16; ++u) s = fmaf(wv[u], sg[i + u * 64], s);
    }
    for (; i < G; i += 64) s = fmaf(w[i], sg[i], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane < ns) {
      const int cls = slots.cls[si][lane];
      theta[((int64_t)b * max_slots + lane) * P + p] = s + w[G + cls] + w[G + n_classes + si] + bc[p];
    }
  }
}

hipError_t launch_controller(const float* g, int batch, int G, const float* wc, const float* bc,
                             int P, int n_classes, int n_scales, const SlotTable& slots,
                             int max_slots, const int32_t* list, const int32_t* count,
                             int chunk_base, float* theta, hipStream_t st) {
  if (G > 4096) return hipErrorInvalidValue;
  const int g_stride = pad_ch(G);
  hipLaunchKernelGGL(k_controller, dim3(batch, ceil_div(P, kCtrlRows)), dim3(256), 0, st, g, g_stride, G, wc,
                     bc, P, G + n_classes + n_scales, n_classes, slots, max_slots, list, count,
                     chunk_base, theta);
  return hipGetLastError();
}

// BF16 precls F = ReLU(W_p D_0 + b_p) on MFMA (C_0 padded to 32 or 64), in
// the two half chains of precls_half, so that it equals the fused conv
// epilogue's bit for bit.  Wave w takes the block's pixels 64 w .. 64 w + 63
// in four 16-pixel groups; a group's results go through LDS to the pixels'
// own threads.
__device__ __forceinline__ void precls_bf16_mfma(const uint16_t* __restrict__ blk, int c0, int c0_p,
                                                 const float* __restrict__ wp, const float* bp, float (&F)[8]) {
  __shared__ pf32x4 sF[256 * 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int nk = c0_p / 32;
  uint4 A[2][3];
  precls_weights(wp, c0, 0, lane, A[0]);
  precls_weights(wp, c0, 1, lane, A[1]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint16_t* p = blk + (int64_t)(wave * 64 + r * 16 + l16) * c0_p + 4 * g;
    pf32x4 P[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h < nk) {
        const uint2 lo = *reinterpret_cast<const uint2*>(p + 32 * h);
        const uint2 hi = *reinterpret_cast<const uint2*>(p + 32 * h + 16);
        P[h] = precls_half(A[h], make_uint4(lo.x, lo.y, hi.x, hi.y));
      } else {
        P[h] = pf32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
    if (g < 2) sF[(wave * 64 + r * 16 + l16) * 2 + g] = P[0] + P[1];
  }
  const pf32x4 f0 = sF[threadIdx.x * 2], f1 = sF[threadIdx.x * 2 + 1];
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    F[o] = fmaxf(f0[o] + bp[o], 0.f);
    F[o + 4] = fmaxf(f1[o] + bp[o + 4], 0.f);
  }
}

// One thread per pixel of one tile; all the tile's slots in one pass.
constexpr int kHeadChunk = 128;  // bytes of D_0 per pixel staged at a time

template <typename T, int O>
__global__ __launch_bounds__(256) void k_head(const T* __restrict__ d0, int T2, int c0, int c0_p,
                                              const float* __restrict__ wp,
                                              const float* __restrict__ bp,
                                              const float* __restrict__ theta, int P,
                                              SlotTable slots, int max_slots,
                                              const int32_t* list, const int32_t* count,
                                              int chunk_base, int out_base, float* __restrict__ out,
                                              const float* __restrict__ dscale, const float* __restrict__ fpre) {
  const int per_tile = T2 / 256;
  const int b = blockIdx.x / per_tile;
  const int pix = (blockIdx.x % per_tile) * 256 + threadIdx.x;
  if (chunk_base + b >= *count) return;
  const int si = list[4 * (chunk_base + b) + 1];
  const int ns = slots.n_slots[si];
  const bool pre = (c0 != 8);
  // The precls weights and the tile's generated head parameters are the
  // same for every thread of the block: they are read as constant memory
  // with uniform indices (scalar loads into SGPRs, used directly as FMA
  // operands), not staged through LDS.
  typedef const __attribute__((address_space(4))) float cfloat;
  cfloat* wpc = (cfloat*)wp;
  cfloat* bpc = (cfloat*)bp;
  // D_0 of this pixel in 16-byte vectors (channels padded to 32, so whole
  // vectors stay inside the pixel's row)
  const T* px = d0 + ((int64_t)b * T2 + pix) * c0_p;
  constexpr int V = 16 / sizeof(T);
  float F[8];
  bool done = false;
  if (fpre) {
    // F from the decoder's last conv
    const float4* f = reinterpret_cast<const float4*>(fpre + ((int64_t)b * T2 + pix) * 8);
    const float4 f0 = f[0], f1 = f[1];
    F[0] = f0.x;
    F[1] = f0.y;
    F[2] = f0.z;
    F[3] = f0.w;
    F[4] = f1.x;
    F[5] = f1.y;
    F[6] = f1.z;
    F[7] = f1.w;
    done = true;
  }
  if constexpr (std::is_same<T, uint16_t>::value) {
    if (!done && pre && c0_p <= 64) {
      precls_bf16_mfma(d0 + ((int64_t)b * T2 + (blockIdx.x % per_tile) * 256) * c0_p, c0, c0_p, wp, bp, F);
      done = true;
    }
  }
  if (done) {
  } else if (pre && sizeof(T) < 4) {
#pragma unroll
    for (int o = 0; o < 8; ++o) F[o] = bpc[o];
    // Whole 16-byte vectors first, the next one loaded while this one's FMAs
    // run (an unguarded body keeps the loop one basic block), then the
    // c0 % V channels of a partial vector; channels are summed in order.
    const int c0f = c0 - c0 % V;
    uint4 cur = *reinterpret_cast<const uint4*>(px);
    for (int c0v = 0; c0v < c0f; c0v += V) {
      const uint4 nxt = *reinterpret_cast<const uint4*>(px + min(c0v + V, c0_p - V));
      float v[V];
      decode16<T>(cur, v);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int c = c0v + k;
        float x = v[k];
        if constexpr (std::is_same<T, uint8_t>::value) x *= dscale[c];
#pragma unroll
        for (int o = 0; o < 8; ++o) F[o] = fmaf(wpc[o * c0 + c], x, F[o]);
      }
      cur = nxt;
    }
    if (c0f < c0) {
      float v[V];
      decode16<T>(cur, v);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int c = c0f + k;
        if (c < c0) {
          float x = v[k];
          if constexpr (std::is_same<T, uint8_t>::value) x *= dscale[c];
#pragma unroll
          for (int o = 0; o < 8; ++o) F[o] = fmaf(wpc[o * c0 + c], x, F[o]);
        }
      }
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) F[o] = fmaxf(F[o], 0.f);
  } else if (pre) {
    // FP32: the block's 256 pixels are contiguous in D_0.  Their channels
    // are staged through LDS in chunks of kHeadChunk bytes per pixel with
    // coalesced 16-byte loads (consecutive lanes, consecutive vectors), one
    // LDS row per pixel padded by 16 bytes; each thread then reads its own
    // row.  Read straight from memory, a pixel's 256 bytes per thread cost a
    // new cache line per lane and load; the 64- and 128-byte rows of FP8 and
    // BF16 are read directly.
    constexpr int RV = kHeadChunk / 16;  // 16-byte vectors per pixel and chunk
    __shared__ uint4 sD[256 * (RV + 1)];
    const T* blk = d0 + ((int64_t)b * T2 + (blockIdx.x % per_tile) * 256) * c0_p;
    const int pv = c0_p * (int)sizeof(T) / 16;  // vectors per pixel
#pragma unroll
    for (int o = 0; o < 8; ++o) F[o] = bpc[o];
    for (int v0 = 0; v0 < pv; v0 += RV) {
      const int nv = min(RV, pv - v0);
      __syncthreads();  // the previous chunk's rows have been read
      for (int i = threadIdx.x; i < 256 * nv; i += 256) {
        const int p = i / nv, v = i % nv;
        sD[p * (RV + 1) + v] = reinterpret_cast<const uint4*>(blk + (int64_t)p * c0_p)[v0 + v];
      }
      __syncthreads();
      for (int v = 0; v < nv; ++v) {
        float x16[V];
        decode16<T>(sD[threadIdx.x * (RV + 1) + v], x16);
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const int c = (v0 + v) * V + k;
          if (c < c0) {
            float x = x16[k];
            if constexpr (std::is_same<T, uint8_t>::value) x *= dscale[c];
#pragma unroll
            for (int o = 0; o < 8; ++o) F[o] = fmaf(wpc[o * c0 + c], x, F[o]);
          }
        }
      }
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) F[o] = fmaxf(F[o], 0.f);
  } else {
#pragma unroll
    for (int o0 = 0; o0 < 8; o0 += V) {
      float v[V];
      decode16<T>(*reinterpret_cast<const uint4*>(px + o0), v);
#pragma unroll
      for (int k = 0; k < V && o0 + k < 8; ++k) {
        F[o0 + k] = v[k];
        if constexpr (std::is_same<T, uint8_t>::value) F[o0 + k] *= dscale[o0 + k];
      }
    }
  }
  for (int j = 0; j < ns; ++j) {
    cfloat* th = (cfloat*)(theta + ((int64_t)b * max_slots + j) * P);
    cfloat* W1 = th;
    cfloat* W2 = th + 64;
    cfloat* W3 = th + 128;
    cfloat* b1 = th + 128 + 8 * O;
    cfloat* b2 = b1 + 8;
    cfloat* b3 = b2 + 8;
    float h1[8], h2[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      float s = b1[o];
#pragma unroll
      for (int i = 0; i < 8; ++i) s = fmaf(W1[o * 8 + i], F[i], s);
      h1[o] = fmaxf(s, 0.f);
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      float s = b2[o];
#pragma unroll
      for (int i = 0; i < 8; ++i) s = fmaf(W2[o * 8 + i], h1[i], s);
      h2[o] = fmaxf(s, 0.f);
    }
    float z[O];
#pragma unroll
    for (int o = 0; o < O; ++o) {
      float s = b3[o];
#pragma unroll
      for (int i = 0; i < 8; ++i) s = fmaf(W3[o * 8 + i], h2[i], s);
      z[o] = s;
    }
    const float l = (O == 1) ? z[0] : z[O - 1] - z[0];
    out[((int64_t)(out_base + b) * max_slots + j) * T2 + pix] = l;
  }
}

hipError_t launch_head(int precision, const void* d0, int batch, int T, int c0, int c0_p,
                       const float* wp, const float* bp, const float* theta, int P, int o,
                       const SlotTable& slots, int max_slots, const int32_t* list,
                       const int32_t* count, int chunk_base, int out_base, float* tile_logits,
                       hipStream_t st, const float* d0_scale, const float* fpre) {
  const int T2 = T * T;
  if (T2 % 256 || c0 > 256 || max_slots > OMNISEG_MAX_CLASSES) return hipErrorInvalidValue;
  if ((precision == OMNISEG_FP8) != (d0_scale != nullptr)) return hipErrorInvalidValue;
  dim3 grid(batch * (T2 / 256));
#define OMNISEG_HEAD(TY, O)                                                                                      \
  hipLaunchKernelGGL((k_head<TY, O>), grid, dim3(256), 0, st, (const TY*)d0, T2, c0, c0_p, wp, bp, theta, P, \
                     slots, max_slots, list, count, chunk_base, out_base, tile_logits, d0_scale, fpre)
  if (precision == OMNISEG_FP8) {
    if (o == 1) OMNISEG_HEAD(uint8_t, 1); else OMNISEG_HEAD(uint8_t, 2);
  } else if (precision == OMNISEG_BF16) {
    if (o == 1) OMNISEG_HEAD(uint16_t, 1); else OMNISEG_HEAD(uint16_t, 2);
  } else {
    if (o == 1) OMNISEG_HEAD(float, 1); else OMNISEG_HEAD(float, 2);
  }
#undef OMNISEG_HEAD
  return hipGetLastError();
}

}  // namespace omniseg

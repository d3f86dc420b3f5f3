// Weight packing: canonical FP32 conv weights W[cout][cin][3][3] -> the
// layout the conv kernels stage into LDS, [cin_p / KC][9][cout_p][KC] in the
// backbone's storage type, with zero rows and columns for padded channels.
// For the decoder's first conv the input channels are split into the
// upsampled part (cu real, cu_p padded) and the skip part, each padded on its
// own, matching the concatenated activation layout.
#include <algorithm>

#include "internal.h"

namespace omniseg {

__device__ __forceinline__ uint16_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T>
__device__ __forceinline__ T cvt(float v);
template <>
__device__ __forceinline__ float cvt<float>(float v) { return v; }
template <>
__device__ __forceinline__ uint16_t cvt<uint16_t>(float v) { return f2bf_rne(v); }

// The data gradient of Y = conv(X, W) is a 3x3 conv of dY with
// W'[c][o][i][j] = W[o][c][2 - i][2 - j]; its input channels are the forward
// outputs (plain padding) and its outputs the forward inputs (concat padding).
template <typename T, int KC>
__global__ void k_pack_conv_t(const float* __restrict__ canon, char* packed, PackConv p) {
  const int64_t total = (int64_t)p.cout_p * 9 * p.cin_p;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  // i enumerates [chunk of o][tap'][c'][kk]
  const int kk = (int)(i % KC);
  int64_t r = i / KC;
  const int cp = (int)(r % p.cin_p);
  r /= p.cin_p;
  const int tap = (int)(r % 9);
  const int chunk = (int)(r / 9);
  const int o = chunk * KC + kk;
  int c = -1;
  if (cp < p.cu_p) {
    if (cp < p.cu) c = cp;
  } else {
    const int ce = p.cin - p.cu;
    if (cp - p.cu_p < ce) c = p.cu + (cp - p.cu_p);
  }
  float v = 0.f;
  if (o < p.cout && c >= 0) v = canon[p.src + ((int64_t)o * p.cin + c) * 9 + (8 - tap)];
  reinterpret_cast<T*>(packed + p.dst)[i] = cvt<T>(v);
}

template <typename T, int KC>
__global__ void k_pack_conv(const float* __restrict__ canon, char* packed, PackConv p) {
  const int64_t total = (int64_t)p.cin_p * 9 * p.cout_p;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < total) {
    // i enumerates [chunk][tap][n][kk]
    const int kk = (int)(i % KC);
    int64_t r = i / KC;
    const int n = (int)(r % p.cout_p);
    r /= p.cout_p;
    const int tap = (int)(r % 9);
    const int chunk = (int)(r / 9);
    const int cp = chunk * KC + kk;  // padded input channel
    int c = -1;                      // real input channel
    if (cp < p.cu_p) {
      if (cp < p.cu) c = cp;
    } else {
      const int ce = p.cin - p.cu;
      if (cp - p.cu_p < ce) c = p.cu + (cp - p.cu_p);
    }
    float v = 0.f;
    if (n < p.cout && c >= 0) v = canon[p.src + ((int64_t)n * p.cin + c) * 9 + tap];
    reinterpret_cast<T*>(packed + p.dst)[i] = cvt<T>(v);
  }
  if (i < p.cout_p && p.dst_b >= 0) {
    reinterpret_cast<float*>(packed + p.dst_b)[i] = (i < p.cout) ? canon[p.src_b + i] : 0.f;
  }
}

hipError_t launch_pack_conv(int precision, const float* canon, void* packed, const PackConv& p,
                            hipStream_t st) {
  const int64_t total = std::max<int64_t>((int64_t)p.cin_p * 9 * p.cout_p, p.cout_p);
  dim3 grid((unsigned)((total + 255) / 256));
  if (p.transpose) {
    if (precision == OMNISEG_BF16)
      hipLaunchKernelGGL((k_pack_conv_t<uint16_t, 32>), grid, dim3(256), 0, st, canon, (char*)packed, p);
    else
      hipLaunchKernelGGL((k_pack_conv_t<float, 16>), grid, dim3(256), 0, st, canon, (char*)packed, p);
    return hipGetLastError();
  }
  if (precision == OMNISEG_BF16)
    hipLaunchKernelGGL((k_pack_conv<uint16_t, 32>), grid, dim3(256), 0, st, canon, (char*)packed, p);
  else
    hipLaunchKernelGGL((k_pack_conv<float, 16>), grid, dim3(256), 0, st, canon, (char*)packed, p);
  return hipGetLastError();
}

// ---- FP8 -------------------------------------------------------------------

// Exponent e of the power-of-two scale 2^e = 2^ceil(log2(amax / 448)) for
// amax > 0, without a rounded division: amax = m 2^x with m in [0.5, 1) and
// 448 = 0.875 2^9, so amax <= 448 2^e first holds at e = x - 9 when
// m <= 0.875 and at e = x - 8 otherwise.
__device__ __forceinline__ int fp8_scale_exp(float amax) {
  int x;
  const float m = frexpf(amax, &x);
  return m <= 0.875f ? x - 9 : x - 8;
}

__device__ __forceinline__ uint8_t fp8_code(float v) {
  const float c = fminf(fmaxf(v, -kFp8Max), kFp8Max);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(c, 0.f, 0, false) & 0xff);
}

// One workgroup per padded output channel o.  Pass 1: amax over the real
// input channels and taps of W[o][c][t] s_in(c); pass 2: codes of
// W[o][c][t] s_in(c) / w_o into [chunk][tap][cout_p][64] (zeros for padded
// channels), w_o = 2^e into wscale[o], the bias into dst_b.
__global__ __launch_bounds__(256) void k_pack_conv_fp8(const float* __restrict__ canon, char* packed, PackConv p,
                                                       const float* __restrict__ s_in_u,
                                                       const float* __restrict__ s_in_e, float* wscale) {
  const int o = blockIdx.x;
  const int nch = (p.cin_p + kFp8Chunk - 1) / kFp8Chunk;
  const int kin = nch * kFp8Chunk;
  auto scale_of = [&](int cp) { return cp < p.cu_p ? s_in_u[cp] : s_in_e[cp - p.cu_p]; };
  auto real_of = [&](int cp) {  // real input channel of padded channel cp, or -1
    if (cp < p.cu_p) return cp < p.cu ? cp : -1;
    const int ce = p.cin - p.cu;
    return (cp - p.cu_p < ce && cp < p.cin_p) ? p.cu + (cp - p.cu_p) : -1;
  };
  __shared__ float red[256];
  float m = 0.f;
  if (o < p.cout) {
    for (int i = threadIdx.x; i < kin * 9; i += 256) {
      const int cp = i / 9, tap = i % 9;
      const int c = real_of(cp);
      if (c >= 0) m = fmaxf(m, fabsf(canon[p.src + ((int64_t)o * p.cin + c) * 9 + tap] * scale_of(cp)));
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  const float amax = red[0];
  const int e = amax > 0.f ? fp8_scale_exp(amax) : 0;
  const float inv_w = ldexpf(1.f, -e);
  uint8_t* dst = reinterpret_cast<uint8_t*>(packed + p.dst);
  for (int i = threadIdx.x; i < kin * 9; i += 256) {
    const int tap = i / kin, cp = i % kin;
    const int c = o < p.cout ? real_of(cp) : -1;
    const float v = c >= 0 ? canon[p.src + ((int64_t)o * p.cin + c) * 9 + tap] * scale_of(cp) * inv_w : 0.f;
    dst[(((int64_t)(cp / kFp8Chunk) * 9 + tap) * p.cout_p + o) * kFp8Chunk + cp % kFp8Chunk] = fp8_code(v);
  }
  if (threadIdx.x == 0) {
    wscale[o] = ldexpf(1.f, e);
    if (p.dst_b >= 0) reinterpret_cast<float*>(packed + p.dst_b)[o] = o < p.cout ? canon[p.src_b + o] : 0.f;
  }
}

hipError_t launch_pack_conv_fp8(const float* canon, void* packed, const PackConv& p, const float* s_in_u,
                                const float* s_in_e, float* wscale, hipStream_t st) {
  if (p.transpose || !s_in_u || (p.cu_p < p.cin_p && !s_in_e)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_conv_fp8, dim3(p.cout_p), dim3(256), 0, st, canon, (char*)packed, p, s_in_u, s_in_e,
                     wscale);
  return hipGetLastError();
}

// Per-channel maximum of a non-negative FP32 tensor [npix][c_p] into amax
// (atomic max on the bit patterns: non-negative floats order like their
// unsigned bits; -0 and NaN never enter).
__global__ __launch_bounds__(256) void k_amax_channels(const float* __restrict__ x, int64_t npix, int c_p,
                                                       float* amax) {
  const int64_t p0 = (int64_t)blockIdx.x * 256;
  const int64_t p1 = p0 + 256 < npix ? p0 + 256 : npix;
  for (int c = threadIdx.x; c < c_p; c += 256) {
    float m = 0.f;
    for (int64_t p = p0; p < p1; ++p) {
      const float v = x[p * c_p + c];
      m = v > m ? v : m;
    }
    atomicMax(reinterpret_cast<unsigned int*>(amax) + c, __float_as_uint(m));
  }
}

hipError_t launch_amax_channels(const float* x, int64_t npix, int c_p, float* amax, hipStream_t st) {
  if (npix <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_amax_channels, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, x, npix, c_p, amax);
  return hipGetLastError();
}

__global__ void k_fp8_conv_scales(const float* in_scale, int cin, int cu, int cu_p, int cin_p,
                                  const float* out_scale, int cout, int cout_p, float* s_in_pad, float* oinv) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < cin_p) {
    int c = -1;
    if (i < cu_p) {
      if (i < cu) c = i;
    } else if (i - cu_p < cin - cu) {
      c = cu + (i - cu_p);
    }
    s_in_pad[i] = c >= 0 ? in_scale[c] : 1.f;
  }
  if (i < cout_p) oinv[i] = i < cout ? 1.f / out_scale[i] : 1.f;
}

hipError_t launch_fp8_conv_scales(const float* in_scale, int cin, int cu, int cu_p, int cin_p,
                                  const float* out_scale, int cout, int cout_p, float* s_in_pad, float* oinv,
                                  hipStream_t st) {
  const int n = cin_p > cout_p ? cin_p : cout_p;
  hipLaunchKernelGGL(k_fp8_conv_scales, dim3((n + 255) / 256), dim3(256), 0, st, in_scale, cin, cu, cu_p, cin_p,
                     out_scale, cout, cout_p, s_in_pad, oinv);
  return hipGetLastError();
}

__global__ void k_fp8_scales(const float* amax, int64_t n, float* scale, float* inv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float a = amax[i];
  const int e = a > 0.f ? fp8_scale_exp(a) : 0;
  scale[i] = ldexpf(1.f, e);
  inv[i] = ldexpf(1.f, -e);
}

hipError_t launch_fp8_scales(const float* amax, int64_t n, float* scale, float* inv, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fp8_scales, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, amax, n, scale, inv);
  return hipGetLastError();
}

__global__ void k_copy_f32(const float* src, float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace omniseg

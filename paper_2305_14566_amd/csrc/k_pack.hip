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

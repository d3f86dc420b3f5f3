// Backward pass of the slide-wise path: stitch, dynamic head, controller,
// bottleneck mean, and the U-Net's weight and data gradients.
//
// Every reduction is deterministic: partial sums go to per-block slots and
// are summed in a fixed order by a second kernel (no floating-point atomics).
// Weight gradients are written straight into the canonical FP32 order.
#include "internal.h"

namespace omniseg {

typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ float ldf(const float* p) { return *p; }
__device__ __forceinline__ float ldf(const uint16_t* p) { return __uint_as_float((uint32_t)(*p) << 16); }
__device__ __forceinline__ void stf(float* p, float v) { *p = v; }
__device__ __forceinline__ void stf(uint16_t* p, float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  *p = (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t bf16_bits(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
// Eight consecutive values (p 16-byte aligned for BF16, 32-byte for FP32).
__device__ __forceinline__ void ld8(const float* p, float (&v)[8]) {
  const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ __forceinline__ void ld8(const uint16_t* p, float (&v)[8]) {
  const uint4 q = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = __uint_as_float(w[k] << 16);
    v[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
  }
}
__device__ __forceinline__ void st8(float* p, const float (&v)[8]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4*>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
}
__device__ __forceinline__ void st8(uint16_t* p, const float (&v)[8]) {
  *reinterpret_cast<uint4*>(p) = make_uint4(bf16_bits(v[0]) | (bf16_bits(v[1]) << 16), bf16_bits(v[2]) | (bf16_bits(v[3]) << 16),
                                            bf16_bits(v[4]) | (bf16_bits(v[5]) << 16), bf16_bits(v[6]) | (bf16_bits(v[7]) << 16));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ---------------------------------------------------------------------------
// network input of each batch tile, FP32 NHWC with 32 channels (3 real)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_input_x(FirstConvArgs a, float* __restrict__ x) {
  const int T2 = a.T * a.T;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)a.batch * T2) return;
  const int b = (int)(i / T2), q = (int)(i % T2);
  const int4 t = reinterpret_cast<const int4*>(a.list)[a.chunk_base + b];
  const SlideDev& sd = a.slides[t.x];
  const int k = a.scale_k[t.y];
  const int Y = t.z * a.scale_s[t.y] + q / a.T, X = t.w * a.scale_s[t.y] + q % a.T;
  const float scale = 1.0f / (255.0f * (float)(1 << (2 * k)));
  float v0, v1, v2;
  if (k == 0) {
    int r, g, bb;
    if (Y < sd.H && X < sd.W) {
      const uint8_t* p = sd.rgb + (int64_t)Y * sd.pitch + 3 * X;
      r = p[0];
      g = p[1];
      bb = p[2];
    } else {
      r = sd.pad[0];
      g = sd.pad[1];
      bb = sd.pad[2];
    }
    v0 = r * scale;
    v1 = g * scale;
    v2 = bb * scale;
  } else {
    const ushort4 s4 = reinterpret_cast<const ushort4*>(sd.pyr[t.y])[(int64_t)Y * sd.pyr_ex[t.y] + X];
    v0 = s4.x * scale;
    v1 = s4.y * scale;
    v2 = s4.z * scale;
  }
  float4* o = reinterpret_cast<float4*>(x + i * 32);
  o[0] = make_float4(v0, v1, v2, 0.f);
#pragma unroll
  for (int j = 1; j < 8; ++j) o[j] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_input_x(const FirstConvArgs& a, float* x, hipStream_t st) {
  const int64_t n = (int64_t)a.batch * a.T * a.T;
  hipLaunchKernelGGL(k_input_x, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, x);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stitch backward: dl_t(q) = dLambda(o_t + q) w(q) / D(o_t + q)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stitch_bwd(StitchBwdArgs a) {
  const int T = a.T, s = a.s, T2 = T * T;
  const int per = T2 / 256;
  const int blk = blockIdx.x;
  const int t = blk / (a.max_slots * per);
  const int j = (blk / per) % a.max_slots;
  const int q = (blk % per) * 256 + threadIdx.x;
  const int4 tl = reinterpret_cast<const int4*>(a.list)[t];
  const int si = tl.y;
  if (j >= a.n_slots[si]) return;
  const int qy = q / T, qx = q % T;
  const int y = tl.z * s + qy, x = tl.w * s + qx;
  float out = 0.f;
  if (y < a.Hk[si] && x < a.Wk[si]) {
    const int ny = a.ny[si], nx = a.nx[si];
    const int32_t* grid = a.grid[si];
    const int jy0 = (y < T) ? 0 : (y - T) / s + 1, jy1 = min(ny - 1, y / s);
    const int jx0 = (x < T) ? 0 : (x - T) / s + 1, jx1 = min(nx - 1, x / s);
    int den = 0;
    for (int jy = jy0; jy <= jy1; ++jy) {
      const int iy = y - jy * s;
      const int ry = min(iy + 1, T - iy);
      for (int jx = jx0; jx <= jx1; ++jx) {
        if (grid[jy * nx + jx] < 0) continue;
        const int ix = x - jx * s;
        den += ry * min(ix + 1, T - ix);
      }
    }
    const int w = min(qy + 1, T - qy) * min(qx + 1, T - qx);
    const float g = a.dlam[a.plane_off[si][j] + (int64_t)y * a.Wk[si] + x];
    out = g * (float)w / (float)den;
  }
  a.dl[((int64_t)t * a.max_slots + j) * T2 + q] = out;
}

hipError_t launch_stitch_bwd(const StitchBwdArgs& a, hipStream_t st) {
  const int per = a.T * a.T / 256;
  hipLaunchKernelGGL(k_stitch_bwd, dim3(a.n_tiles * a.max_slots * per), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dynamic head + precls backward, one thread per pixel; per-block partial
// sums of the parameter gradients (theta per slot, W_p and b_p)
// ---------------------------------------------------------------------------
template <typename T, int O>
__global__ __launch_bounds__(256) void k_head_bwd(HeadBwdArgs a) {
  constexpr int P = 144 + 9 * O;
  __shared__ float sth[OMNISEG_MAX_CLASSES * P];
  __shared__ float swp[8 * 128 + 8];
  __shared__ float red[4][8 * 128 + 8];
  const int T2 = a.T * a.T;
  const int per = T2 / 256;
  const int b = blockIdx.x / per, pblk = blockIdx.x % per;
  const int pix = pblk * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int si = a.list[4 * b + 1];
  const int ns = a.n_slots[si];
  const int c0 = a.c0;
  for (int i = threadIdx.x; i < ns * P; i += 256) sth[i] = a.theta[(int64_t)b * a.max_slots * P + i];
  const bool pre = (c0 != 8);
  if (pre) {
    for (int i = threadIdx.x; i < 8 * c0; i += 256) swp[i] = a.wp[i];
    if (threadIdx.x < 8) swp[8 * c0 + threadIdx.x] = a.bp[threadIdx.x];
  }
  __syncthreads();
  const T* px = (const T*)a.d0 + ((int64_t)b * T2 + pix) * a.c0_p;
  float F[8], Fpre[8];
  if (pre) {
#pragma unroll
    for (int o = 0; o < 8; ++o) Fpre[o] = swp[8 * c0 + o];
    int c = 0;
    for (; c + 8 <= c0; c += 8) {  // eight channels per load, the same FMA order
      float v[8];
      ld8(px + c, v);
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int o = 0; o < 8; ++o) Fpre[o] = fmaf(swp[o * c0 + c + q], v[q], Fpre[o]);
    }
    for (; c < c0; ++c) {
      const float v = ldf(px + c);
#pragma unroll
      for (int o = 0; o < 8; ++o) Fpre[o] = fmaf(swp[o * c0 + c], v, Fpre[o]);
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) F[o] = fmaxf(Fpre[o], 0.f);
  } else {
#pragma unroll
    for (int o = 0; o < 8; ++o) F[o] = Fpre[o] = ldf(px + o);
  }
  float dF[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) dF[o] = 0.f;
  for (int j = 0; j < ns; ++j) {
    const float* th = &sth[j * P];
    const float* W1 = th;
    const float* W2 = th + 64;
    const float* W3 = th + 128;
    const float* b1 = th + 128 + 8 * O;
    const float* b2 = b1 + 8;
    float h1p[8], h1[8], h2p[8], h2[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      float s = b1[o];
#pragma unroll
      for (int i = 0; i < 8; ++i) s = fmaf(W1[o * 8 + i], F[i], s);
      h1p[o] = s;
      h1[o] = fmaxf(s, 0.f);
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      float s = b2[o];
#pragma unroll
      for (int i = 0; i < 8; ++i) s = fmaf(W2[o * 8 + i], h1[i], s);
      h2p[o] = s;
      h2[o] = fmaxf(s, 0.f);
    }
    const float dl = a.dl[((int64_t)b * a.max_slots + j) * T2 + pix];
    float dz[O];
    if (O == 1) {
      dz[0] = dl;
    } else {
      dz[0] = -dl;
      dz[O - 1] = dl;
    }
    float dh2[8], dh1[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < O; ++o) s = fmaf(W3[o * 8 + i], dz[o], s);
      dh2[i] = h2p[i] > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < 8; ++o) s = fmaf(W2[o * 8 + i], dh2[o], s);
      dh1[i] = h1p[i] > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < 8; ++o) s = fmaf(W1[o * 8 + i], dh1[o], s);
      dF[i] += s;
    }
    // per-pixel parameter gradient, reduced over the block: W1, W2, W3, b1,
    // b2, b3.  Each group of 64 parameters is reduce-scattered over the wave
    // (at mask m = 32 .. 1 a lane keeps the half of its values its lane bit m
    // selects and adds the partner's copy), so lane l ends with the wave sum
    // of parameter 64 g + l: the same pairs added in the same order as a
    // full xor-shuffle sum, with 63 shuffles per 64 parameters instead of 384.
    float* dst = a.dtheta_part + (((int64_t)b * a.max_slots + j) * per + pblk) * P;
#pragma unroll
    for (int g = 0; g < (P + 63) / 64; ++g) {
      float vals[64];
#pragma unroll
      for (int q = 0; q < 64; ++q) {
        const int p = 64 * g + q;
        float v = 0.f;
        if (p < 64) v = dh1[p / 8] * F[p % 8];
        else if (p < 128) v = dh2[(p - 64) / 8] * h1[(p - 64) % 8];
        else if (p < 128 + 8 * O) v = dz[(p - 128) / 8] * h2[(p - 128) % 8];
        else if (p < 136 + 8 * O) v = dh1[p - 128 - 8 * O];
        else if (p < 144 + 8 * O) v = dh2[p - 136 - 8 * O];
        else if (p < P) v = dz[p - 144 - 8 * O];
        vals[q] = v;
      }
#pragma unroll
      for (int m = 32, n = 32; m >= 1; m >>= 1, n >>= 1) {
        const bool up = (lane & m) != 0;
#pragma unroll
        for (int q = 0; q < n; ++q) {
          const float lo = vals[q], hi = vals[q + n];
          const float send = up ? lo : hi, keep = up ? hi : lo;
          vals[q] = keep + __shfl_xor(send, m);
        }
      }
      if (64 * g + lane < P) red[wave][64 * g + lane] = vals[0];
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += 256) dst[p] = (red[0][p] + red[1][p]) + (red[2][p] + red[3][p]);
    __syncthreads();
  }
  // precls backward
  T* dd0 = (T*)a.dd0 + ((int64_t)b * T2 + pix) * a.c0_p;
  if (pre) {
    float dpre[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) dpre[o] = Fpre[o] > 0.f ? dF[o] : 0.f;
    for (int c8 = 0; c8 < a.c0_p; c8 += 8) {  // c0_p is a multiple of 32
      float d[8], sv[8];
      if (a.mask_d0) ld8(px + c8, d);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = c8 + q;
        float s = 0.f;
        if (c < c0) {
#pragma unroll
          for (int o = 0; o < 8; ++o) s = fmaf(swp[o * c0 + c], dpre[o], s);
          if (a.mask_d0 && !(d[q] > 0.f)) s = 0.f;
        }
        sv[q] = s;
      }
      st8(dd0 + c8, sv);
    }
    const int NP = 8 * c0 + 8;
    float* dst = a.dwp_part + ((int64_t)b * per + pblk) * NP;
    if (c0 % 8 == 0) {
      // 64 parameters at a time, 8 output channels x 8 input channels, wave
      // sums by the butterfly reduce-scatter of the theta gradient (the same
      // sums as wave_sum); lane l ends with parameter (l / 8, cc + l % 8)
      for (int cc = 0; cc < c0; cc += 8) {
        float x[8];
        ld8(px + cc, x);
        float vals[64];
#pragma unroll
        for (int q = 0; q < 64; ++q) vals[q] = dpre[q >> 3] * x[q & 7];
#pragma unroll
        for (int m = 32, n = 32; m >= 1; m >>= 1, n >>= 1) {
          const bool up = (lane & m) != 0;
#pragma unroll
          for (int q = 0; q < n; ++q) {
            const float lo = vals[q], hi = vals[q + n];
            const float send = up ? lo : hi, keep = up ? hi : lo;
            vals[q] = keep + __shfl_xor(send, m);
          }
        }
        red[wave][(lane >> 3) * c0 + cc + (lane & 7)] = vals[0];
      }
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const float v = wave_sum(dpre[o]);
        if (lane == 0) red[wave][8 * c0 + o] = v;
      }
    } else {
      for (int p = 0; p < NP; ++p) {
        float v = (p < 8 * c0) ? dpre[p / c0] * ldf(px + p % c0) : dpre[p - 8 * c0];
        v = wave_sum(v);
        if (lane == 0) red[wave][p] = v;
      }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < NP; p += 256) dst[p] = (red[0][p] + red[1][p]) + (red[2][p] + red[3][p]);
  } else {
    for (int c = 0; c < a.c0_p; ++c) stf(dd0 + c, c < 8 && !(a.mask_d0 && !(F[c] > 0.f)) ? dF[c] : 0.f);
  }
}

hipError_t launch_head_bwd(int precision, const HeadBwdArgs& a, hipStream_t st) {
  const int per = a.T * a.T / 256;
  dim3 grid(a.n_tiles * per);
  if (a.c0 > 128) return hipErrorInvalidValue;
  if (precision == OMNISEG_BF16) {
    if (a.o == 1) hipLaunchKernelGGL((k_head_bwd<uint16_t, 1>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_head_bwd<uint16_t, 2>), grid, dim3(256), 0, st, a);
  } else {
    if (a.o == 1) hipLaunchKernelGGL((k_head_bwd<float, 1>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_head_bwd<float, 2>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

// out[r][kb][i] = sum of in[r][k][i] over the rows k of block kb (kc rows
// each): a workgroup takes 64 columns i of one row r and one block of kc
// rows k, wave w the rows k = w mod 4 in increasing order, then the four
// partial sums in a fixed order (deterministic).
constexpr int kSumRows = 256;
__global__ __launch_bounds__(256) void k_sum_mid(const float* __restrict__ in, int R, int K, int I, int kc,
                                                 float* __restrict__ out) {
  __shared__ float red[4][64];
  const int nib = (I + 63) / 64, nkb = (K + kc - 1) / kc;
  int blk = blockIdx.x;
  const int kb = blk % nkb;
  blk /= nkb;
  const int ib = blk % nib, r = blk / nib;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = ib * 64 + lane;
  const int k0 = kb * kc, k1 = min(K, k0 + kc);
  float s = 0.f;
  if (i < I) {
    const float* src = in + (int64_t)r * K * I + i;
#pragma unroll 8
    for (int k = k0 + w; k < k1; k += 4) s += src[(int64_t)k * I];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < I) out[((int64_t)r * nkb + kb) * I + i] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// out[r][i] = sum_k in[r][k][i] for k = 0..K-1 (fixed order).  K > 256 goes
// through `part` (R * ceil(K / 256) * I floats): block sums, then their sum.
hipError_t launch_sum_mid(const float* in, int R, int K, int I, float* out, float* part, hipStream_t st) {
  if ((int64_t)R * I == 0) return hipSuccess;
  if (K > kSumRows * kSumRows || (K > kSumRows && !part)) return hipErrorInvalidValue;
  const int nib = (I + 63) / 64;
  if (K <= kSumRows) {
    hipLaunchKernelGGL(k_sum_mid, dim3((unsigned)((int64_t)R * nib)), dim3(256), 0, st, in, R, K, I, K, out);
    return hipGetLastError();
  }
  const int nkb = (K + kSumRows - 1) / kSumRows;
  hipLaunchKernelGGL(k_sum_mid, dim3((unsigned)((int64_t)R * nib * nkb)), dim3(256), 0, st, in, R, K, I, kSumRows,
                     part);
  hipLaunchKernelGGL(k_sum_mid, dim3((unsigned)((int64_t)R * nib)), dim3(256), 0, st, (const float*)part, R, nkb, I,
                     nkb, out);
  return hipGetLastError();
}

int64_t sum_mid_part_floats(int R, int K, int I) {
  return K > kSumRows ? (int64_t)R * ((K + kSumRows - 1) / kSumRows) * I : 0;
}

// ---------------------------------------------------------------------------
// controller backward
// ---------------------------------------------------------------------------
// dW_c[p][i] (row_len columns) and db_c[p], summed over (tile, slot) in order
__global__ void k_ctrl_wgrad(CtrlBwdArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int cols = a.row_len + 1;
  if (idx >= (int64_t)a.P * cols) return;
  const int p = (int)(idx / cols), i = (int)(idx % cols);
  float s = 0.f;
  for (int t = 0; t < a.n_tiles; ++t) {
    const int si = a.list[4 * t + 1];
    for (int j = 0; j < a.n_slots[si]; ++j) {
      const float d = a.dtheta[((int64_t)t * a.max_slots + j) * a.P + p];
      float v;
      if (i < a.G) v = a.g[(int64_t)t * a.g_stride + i];
      else if (i < a.G + a.n_classes) v = (a.cls[si][j] == i - a.G) ? 1.f : 0.f;
      else if (i < a.row_len) v = (si == i - a.G - a.n_classes) ? 1.f : 0.f;
      else v = 1.f;  // bias
      s = fmaf(d, v, s);
    }
  }
  if (i < a.row_len) a.dwc[(int64_t)p * a.row_len + i] = s;
  else a.dbc[p] = s;
}

// dg[t][i] = sum_j sum_p W_c[p][i] dtheta[t][j][p]
__global__ void k_ctrl_dg(CtrlBwdArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.n_tiles * a.G) return;
  const int t = (int)(idx / a.G), i = (int)(idx % a.G);
  const int si = a.list[4 * t + 1];
  float s = 0.f;
  for (int j = 0; j < a.n_slots[si]; ++j)
    for (int p = 0; p < a.P; ++p)
      s = fmaf(a.wc[(int64_t)p * a.row_len + i], a.dtheta[((int64_t)t * a.max_slots + j) * a.P + p], s);
  a.dg[(int64_t)t * a.g_stride + i] = s;
}

hipError_t launch_ctrl_bwd(const CtrlBwdArgs& a, hipStream_t st) {
  const int64_t n1 = (int64_t)a.P * (a.row_len + 1);
  hipLaunchKernelGGL(k_ctrl_wgrad, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, a);
  const int64_t n2 = (int64_t)a.n_tiles * a.G;
  hipLaunchKernelGGL(k_ctrl_dg, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise gradient routing
// ---------------------------------------------------------------------------
// bottleneck mean backward: dE[t][pix][c] = dg[t][c] / hw (c < G), 0 on padding
template <typename T>
__global__ void k_gap_bwd(const float* dg, int g_stride, int G, int hw, int c_p, int64_t n, T* dE) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % c_p);
  const int64_t t = i / ((int64_t)hw * c_p);
  stf(dE + i, c < G ? dg[t * g_stride + c] / (float)hw : 0.f);
}

hipError_t launch_gap_bwd(int precision, const float* dg, int g_stride, int G, int hw, int c_p, int n_tiles,
                          void* dE, hipStream_t st) {
  const int64_t n = (int64_t)n_tiles * hw * c_p;
  dim3 grid((unsigned)((n + 255) / 256));
  if (precision == OMNISEG_BF16)
    hipLaunchKernelGGL(k_gap_bwd<uint16_t>, grid, dim3(256), 0, st, dg, g_stride, G, hw, c_p, n, (uint16_t*)dE);
  else
    hipLaunchKernelGGL(k_gap_bwd<float>, grid, dim3(256), 0, st, dg, g_stride, G, hw, c_p, n, (float*)dE);
  return hipGetLastError();
}

// out = (y > 0) ? dy : 0, elementwise
template <typename T>
__global__ void k_relu_mask(const T* dy, const T* y, int64_t n, T* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) stf(out + i, ldf(y + i) > 0.f ? ldf(dy + i) : 0.f);
}

hipError_t launch_relu_mask(int precision, const void* dy, const void* y, int64_t n, void* out, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256));
  if (precision == OMNISEG_BF16)
    hipLaunchKernelGGL(k_relu_mask<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)dy, (const uint16_t*)y, n,
                       (uint16_t*)out);
  else
    hipLaunchKernelGGL(k_relu_mask<float>, grid, dim3(256), 0, st, (const float*)dy, (const float*)y, n, (float*)out);
  return hipGetLastError();
}

// Split the data gradient of the decoder's concat input dZ [pix][cu_p + ce_p]:
// skip part added into dE [pix][ce_p]; upsampled part summed over each 2x2
// block into dD [pix/4][cu_p] (set, or added when `accumulate`).  With
// `ymask` (the coarse decoder output the upsampled part came from, a ReLU
// output) the stored dD is zero where ymask <= 0: the gradient through that
// ReLU, as a separate mask pass would give it.
template <typename T>
__global__ void k_concat_bwd(const T* dZ, int n_tiles, int H, int W, int cu_p, int ce_p, T* dE, T* dD,
                             int accumulate, const T* ymask) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int cz = cu_p + ce_p;
  const int64_t n_skip = (int64_t)n_tiles * H * W * ce_p;
  const int64_t n_up = (int64_t)n_tiles * (H / 2) * (W / 2) * cu_p;
  if (i < n_skip) {
    const int c = (int)(i % ce_p);
    const int64_t px = i / ce_p;
    stf(dE + i, ldf(dE + i) + ldf(dZ + px * cz + cu_p + c));
  } else if (i < n_skip + n_up) {
    const int64_t k = i - n_skip;
    const int c = (int)(k % cu_p);
    int64_t r = k / cu_p;
    const int X = (int)(r % (W / 2));
    r /= (W / 2);
    const int Y = (int)(r % (H / 2));
    const int64_t t = r / (H / 2);
    const T* z = dZ + ((t * H + 2 * Y) * W + 2 * X) * cz + c;
    float s = (ldf(z) + ldf(z + cz)) + (ldf(z + (int64_t)W * cz) + ldf(z + (int64_t)W * cz + cz));
    if (accumulate) s += ldf(dD + k);
    if (ymask && !(ldf(ymask + k) > 0.f)) s = 0.f;
    stf(dD + k, s);
  }
}

hipError_t launch_concat_bwd(int precision, const void* dZ, int n_tiles, int H, int W, int cu_p, int ce_p,
                             void* dE, void* dD, int accumulate, const void* ymask, hipStream_t st) {
  const int64_t n = (int64_t)n_tiles * H * W * ce_p + (int64_t)n_tiles * (H / 2) * (W / 2) * cu_p;
  dim3 grid((unsigned)((n + 255) / 256));
  if (precision == OMNISEG_BF16)
    hipLaunchKernelGGL(k_concat_bwd<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)dZ, n_tiles, H, W, cu_p,
                       ce_p, (uint16_t*)dE, (uint16_t*)dD, accumulate, (const uint16_t*)ymask);
  else
    hipLaunchKernelGGL(k_concat_bwd<float>, grid, dim3(256), 0, st, (const float*)dZ, n_tiles, H, W, cu_p, ce_p,
                       (float*)dE, (float*)dD, accumulate, (const float*)ymask);
  return hipGetLastError();
}

// 2x2 max-pool backward: each window's gradient goes to its first maximum
// (row-major); added into dE of the finer level.  With `relu` (E a ReLU
// output, and this the last contribution to dE) all four entries of the
// window are also stored as zero where E <= 0: the gradient through that
// ReLU, as a separate mask pass over dE would give it.
template <typename T>
__global__ void k_maxpool_bwd(const T* E, const T* dX, int n_tiles, int H, int W, int c_p, T* dE, int relu) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;  // coarse element
  const int Hh = H / 2, Wh = W / 2;
  if (i >= (int64_t)n_tiles * Hh * Wh * c_p) return;
  const int c = (int)(i % c_p);
  int64_t r = i / c_p;
  const int X = (int)(r % Wh);
  r /= Wh;
  const int Y = (int)(r % Hh);
  const int64_t t = r / Hh;
  int64_t off[4];
  off[0] = ((t * H + 2 * Y) * W + 2 * X) * c_p + c;
  off[1] = off[0] + c_p;
  off[2] = off[0] + (int64_t)W * c_p;
  off[3] = off[2] + c_p;
  int best = 0;
  float bv = ldf(E + off[0]);
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const float v = ldf(E + off[k]);
    if (v > bv) {
      bv = v;
      best = k;
    }
  }
  const float g = ldf(dX + i);
  if (relu) {
    float e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = ldf(E + off[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k == best) stf(dE + off[k], ldf(dE + off[k]) + g);  // rounded as without the mask
      if (!(e[k] > 0.f)) stf(dE + off[k], 0.f);
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k == best) stf(dE + off[k], ldf(dE + off[k]) + g);
}

hipError_t launch_maxpool_bwd(int precision, const void* E, const void* dX, int n_tiles, int H, int W, int c_p,
                              void* dE, hipStream_t st, int relu) {
  const int64_t n = (int64_t)n_tiles * (H / 2) * (W / 2) * c_p;
  dim3 grid((unsigned)((n + 255) / 256));
  if (precision == OMNISEG_BF16)
    hipLaunchKernelGGL(k_maxpool_bwd<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)E, (const uint16_t*)dX,
                       n_tiles, H, W, c_p, (uint16_t*)dE, relu);
  else
    hipLaunchKernelGGL(k_maxpool_bwd<float>, grid, dim3(256), 0, st, (const float*)E, (const float*)dX, n_tiles,
                       H, W, c_p, (float*)dE, relu);
  return hipGetLastError();
}

// grid-stride: buffers of more than 2^32 words take fewer blocks than words / 256
__global__ void k_fill_zero(uint32_t* p, int64_t n) {
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += step) p[i] = 0u;
}

__global__ void k_set_i32(int32_t* p, int32_t v) {
  if (threadIdx.x == 0) *p = v;
}

hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st) {
  const int64_t n = bytes / 4;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// weight gradient of a 3x3 conv on FP32 MFMA:
// dW[o][tap][c] = sum over pixels of dY[pix][o] * X[pix + tap offset][c].
// M = o (64 per block), N = c (32 per block), K = pixels of a BY x BX block;
// the block's share of the pixel blocks is split-K slot `split`, whose
// partial goes to part[split][o][tap][c].
// ---------------------------------------------------------------------------
template <typename TX, int LOADER>
__device__ __forceinline__ float4 wg_load_x(const WgradArgs& a, int b, int y, int x, int c) {
  const TX* X0 = (const TX*)a.x0;
  if (LOADER == LOAD_PLAIN) {
    const TX* p = X0 + (((int64_t)b * a.H + y) * a.W + x) * a.cin_p + c;
    return make_float4(ldf(p), ldf(p + 1), ldf(p + 2), ldf(p + 3));
  } else if (LOADER == LOAD_POOL) {
    const int W2 = 2 * a.W;
    const TX* p = X0 + (((int64_t)b * 2 * a.H + 2 * y) * W2 + 2 * x) * a.cin_p + c;
    float4 r;
    float* rr = &r.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float v0 = ldf(p + k), v1 = ldf(p + a.cin_p + k);
      const float v2 = ldf(p + (int64_t)W2 * a.cin_p + k), v3 = ldf(p + (int64_t)W2 * a.cin_p + a.cin_p + k);
      rr[k] = fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
    }
    return r;
  } else {
    if (c < a.cu_p) {
      const TX* p = X0 + (((int64_t)b * (a.H >> 1) + (y >> 1)) * (a.W >> 1) + (x >> 1)) * a.cu_p + c;
      return make_float4(ldf(p), ldf(p + 1), ldf(p + 2), ldf(p + 3));
    }
    const int ce_p = a.cin_p - a.cu_p;
    const TX* p = (const TX*)a.x1 + (((int64_t)b * a.H + y) * a.W + x) * ce_p + (c - a.cu_p);
    return make_float4(ldf(p), ldf(p + 1), ldf(p + 2), ldf(p + 3));
  }
}

template <typename TX, typename TG, int BX, int BO, int LOADER>
__global__ __launch_bounds__(256) void k_wgrad3x3(WgradArgs a) {
  constexpr int BY = 8, BM = BY * BX, PX = BX + 2, NPIX = (BY + 2) * PX;
  constexpr int BC = 32;
  constexpr int FO = BO / 32;                  // 16-row fragments per wave along o
  constexpr int GROW = BO + 1, XROW = BC + 1;  // odd row lengths spread LDS banks
  __shared__ float sG[BM * GROW];
  __shared__ float sX[NPIX * XROW];
  const int n_ob = a.cout_p / BO, n_cb = a.cin_p / BC;
  int rest = blockIdx.x;
  const int ob = rest % n_ob;
  rest /= n_ob;
  const int cb = rest % n_cb;
  const int split = rest / n_cb;
  const int o0 = ob * BO, c0 = cb * BC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // wave tile: BO/2 o x 16 c
  const int l16 = lane & 15, kq = lane >> 4;
  const int tiles_y = a.H / BY, tiles_x = a.W / BX;
  const int n_chunks = a.n_tiles * tiles_y * tiles_x;
  f32x4 acc[9][FO];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int f = 0; f < FO; ++f) acc[t][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ch = split; ch < n_chunks; ch += a.splits) {
    const int b = ch / (tiles_y * tiles_x);
    const int sy = (ch / tiles_x) % tiles_y, sx = ch % tiles_x;
    const int y0 = sy * BY, x0 = sx * BX;
    const TG* G = (const TG*)a.dy;
    for (int i = tid; i < BM * BO; i += 256) {
      const int m = i / BO, o = i % BO;
      const int y = y0 + m / BX, x = x0 + m % BX;
      sG[m * GROW + o] = ldf(G + (((int64_t)b * a.H + y) * a.W + x) * a.cout_p + o0 + o);
    }
    for (int i = tid; i < NPIX * (BC / 4); i += 256) {
      const int p = i / (BC / 4), v = (i % (BC / 4)) * 4;
      const int y = y0 + p / PX - 1, x = x0 + p % PX - 1;
      float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
      if (y >= 0 && y < a.H && x >= 0 && x < a.W) val = wg_load_x<TX, LOADER>(a, b, y, x, c0 + v);
      float* d = &sX[p * XROW + v];
      d[0] = val.x;
      d[1] = val.y;
      d[2] = val.z;
      d[3] = val.w;
    }
    __syncthreads();
    for (int k0 = 0; k0 < BM; k0 += 4) {
      const int m = k0 + kq;  // this lane's pixel (MFMA K index)
      const int py = m / BX, pxx = m % BX;
      float ga[FO];
#pragma unroll
      for (int f = 0; f < FO; ++f) ga[f] = sG[m * GROW + wm * (BO / 2) + f * 16 + l16];
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const float xv = sX[((py + tap / 3) * PX + pxx + tap % 3) * XROW + wn * 16 + l16];
#pragma unroll
        for (int f = 0; f < FO; ++f)
          acc[tap][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[f], xv, acc[tap][f], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* part = a.part + (int64_t)split * a.cout_p * 9 * a.cin_p;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int f = 0; f < FO; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + wm * (BO / 2) + f * 16 + kq * 4 + r;
        const int c = c0 + wn * 16 + l16;
        part[((int64_t)o * 9 + tap) * a.cin_p + c] = acc[tap][f][r];
      }
}

// ---------------------------------------------------------------------------
// The same weight gradient for BF16 inputs and output gradients on BF16 MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the products are exact in
// FP32 and the pixel sums run in FP32, as in the FP32-MFMA kernel.  K (the
// MFMA reduction) is the pixel, so both operands are staged transposed in
// LDS: dY as [o][pixel], and the input halo as [dx][c][halo row][x], one
// copy per horizontal tap offset dx, so that every operand read is one
// aligned 16-byte vector of 8 consecutive pixels.  A block owns BO output
// and 32 input channels; its four waves split them 2 x 2; one chunk is an
// 8-row x BX-column pixel block (K steps of 32 pixels).
// ---------------------------------------------------------------------------
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

template <int LOADER>
__device__ __forceinline__ uint4 wg_load_x_bf16(const WgradArgs& a, int b, int y, int x, int c) {
  const uint16_t* X0 = (const uint16_t*)a.x0;
  if (LOADER == LOAD_PLAIN) {
    return *reinterpret_cast<const uint4*>(X0 + (((int64_t)b * a.H + y) * a.W + x) * a.cin_p + c);
  } else if (LOADER == LOAD_POOL) {
    const int W2 = 2 * a.W;
    const uint16_t* p = X0 + (((int64_t)b * 2 * a.H + 2 * y) * W2 + 2 * x) * a.cin_p + c;
    uint4 q[4];
    q[0] = *reinterpret_cast<const uint4*>(p);
    q[1] = *reinterpret_cast<const uint4*>(p + a.cin_p);
    q[2] = *reinterpret_cast<const uint4*>(p + (int64_t)W2 * a.cin_p);
    q[3] = *reinterpret_cast<const uint4*>(p + (int64_t)W2 * a.cin_p + a.cin_p);
    uint4 r;
    uint16_t* rr = reinterpret_cast<uint16_t*>(&r);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float m = ldf(reinterpret_cast<const uint16_t*>(&q[0]) + k);
#pragma unroll
      for (int j = 1; j < 4; ++j) m = fmaxf(m, ldf(reinterpret_cast<const uint16_t*>(&q[j]) + k));
      rr[k] = (uint16_t)(__float_as_uint(m) >> 16);  // the maximum is one of the BF16 inputs: exact
    }
    return r;
  } else {
    if (c < a.cu_p) {
      const uint16_t* p = X0 + (((int64_t)b * (a.H >> 1) + (y >> 1)) * (a.W >> 1) + (x >> 1)) * a.cu_p + c;
      return *reinterpret_cast<const uint4*>(p);
    }
    const int ce_p = a.cin_p - a.cu_p;
    const uint16_t* p = (const uint16_t*)a.x1 + (((int64_t)b * a.H + y) * a.W + x) * ce_p + (c - a.cu_p);
    return *reinterpret_cast<const uint4*>(p);
  }
}

// Element-wise maximum of two words of two BF16 values each, as values (the
// result is one of the inputs, so exact), in the order of the pooling loader.
__device__ __forceinline__ uint32_t bf16_max2(uint32_t a, uint32_t b) {
  const uint32_t lo = __float_as_uint(fmaxf(__uint_as_float(a << 16), __uint_as_float(b << 16))) >> 16;
  const uint32_t hi = __float_as_uint(fmaxf(__uint_as_float(a & 0xffff0000u), __uint_as_float(b & 0xffff0000u)));
  return (hi & 0xffff0000u) | lo;
}

// 16-bit element j (0..7) of a 16-byte vector
__device__ __forceinline__ uint32_t elem16(const uint4& v, int j) {
  const uint32_t w = j < 2 ? v.x : j < 4 ? v.y : j < 6 ? v.z : v.w;
  return (j & 1) ? (w >> 16) : (w & 0xffffu);
}

template <int BX, int BO, int LOADER>
__global__ __launch_bounds__(256) void k_wgrad3x3_bf16(WgradArgs a) {
  constexpr int BY = 8, BM = BY * BX;  // pixels per chunk
  constexpr int BC = 32;
  constexpr int FO = BO / 32;          // 16-row fragments per wave along o
  constexpr int GP = BM + 8;           // sGt row (elements): 16 more bytes rotate the banks by 4 per row
  constexpr int HR = BY + 2, HX = BX + 2;
  constexpr int XP = BX + 8;           // sXt row (elements), 16-byte rows
  constexpr int CP = HR * XP + 8;      // sXt channel plane (elements): rotates the banks between channels
  // staging tasks: dY as quads of pixels x 8 channels, the halo as groups of
  // four pixels of one row x 8 channels; at most one of each per thread
  constexpr int NQ = (BM / 4) * (BO / 8);
  constexpr int NG = (HX + 3) / 4;
  constexpr int NXT = HR * NG * (BC / 8);
  constexpr int LPV = (LOADER == LOAD_POOL) ? 4 : 1;
  static_assert(NQ <= 256 && NXT <= 256, "one staging task of each kind per thread");
  static_assert((GP * 2) % 8 == 0 && (XP * 2) % 8 == 0 && (CP * 2) % 8 == 0, "aligned packed stores");
  __shared__ __align__(16) uint16_t sGt[BO * GP];
  __shared__ __align__(16) uint16_t sXt[3 * BC * CP];
  const int n_ob = a.cout_p / BO, n_cb = a.cin_p / BC;
  int rest = blockIdx.x;
  const int ob = rest % n_ob;
  rest /= n_ob;
  const int cb = rest % n_cb;
  const int split = rest / n_cb;
  const int o0 = ob * BO, c0 = cb * BC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // wave tile: BO/2 o x 16 c
  const int l16 = lane & 15, kg = lane >> 4;
  const int tiles_y = a.H / BY, tiles_x = a.W / BX;
  const int n_chunks = a.n_tiles * tiles_y * tiles_x;
  f32x4 acc[9][FO];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int f = 0; f < FO; ++f) acc[t][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* G = (const uint16_t*)a.dy;
  // this thread's staging tasks
  const int q_m = (tid / (BO / 8)) * 4, q_og = (tid % (BO / 8)) * 8;  // dY: pixels q_m..q_m+3, channels q_og..+7
  const bool q_on = tid < NQ;
  const int x_cv = (tid % (BC / 8)) * 8, x_g = (tid / (BC / 8)) % NG, x_hr = tid / ((BC / 8) * NG);
  const bool x_on = tid < NXT;
  const int x_hx0 = x_g * 4;
  uint4 gq[4];
  uint4 xr[4][LPV];

  auto fetch = [&](int ch) {
    const int b = ch / (tiles_y * tiles_x);
    const int sy = (ch / tiles_x) % tiles_y, sx = ch % tiles_x;
    const int y0 = sy * BY, x0 = sx * BX;
    if (q_on) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int m = q_m + k;
        const int y = y0 + m / BX, x = x0 + m % BX;
        gq[k] = *reinterpret_cast<const uint4*>(G + (((int64_t)b * a.H + y) * a.W + x) * a.cout_p + o0 + q_og);
      }
    }
    if (x_on) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int y = y0 + x_hr - 1, x = x0 + x_hx0 + k - 1;
        const bool in = x_hx0 + k < HX && y >= 0 && y < a.H && x >= 0 && x < a.W;
#pragma unroll
        for (int l = 0; l < LPV; ++l) xr[k][l] = make_uint4(0u, 0u, 0u, 0u);
        if (in) {
          if (LOADER == LOAD_POOL) {
            const uint16_t* p = (const uint16_t*)a.x0 + (((int64_t)b * 2 * a.H + 2 * y) * (2 * a.W) + 2 * x) * a.cin_p + c0 + x_cv;
            xr[k][0] = *reinterpret_cast<const uint4*>(p);
            xr[k][LPV > 1 ? 1 : 0] = *reinterpret_cast<const uint4*>(p + a.cin_p);
            xr[k][LPV > 2 ? 2 : 0] = *reinterpret_cast<const uint4*>(p + (int64_t)2 * a.W * a.cin_p);
            xr[k][LPV > 3 ? 3 : 0] = *reinterpret_cast<const uint4*>(p + (int64_t)2 * a.W * a.cin_p + a.cin_p);
          } else {
            xr[k][0] = wg_load_x_bf16<LOADER>(a, b, y, x, c0 + x_cv);
          }
        }
      }
    }
  };
  auto commit = [&]() {
    if (q_on) {
      // sGt[o][pixel]: four pixels of channel q_og + j in one 8-byte store
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint2 v = make_uint2(elem16(gq[0], j) | (elem16(gq[1], j) << 16), elem16(gq[2], j) | (elem16(gq[3], j) << 16));
        *reinterpret_cast<uint2*>(&sGt[(q_og + j) * GP + q_m]) = v;
      }
    }
    if (x_on) {
      uint4 xv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xv[k] = xr[k][0];
        if (LOADER == LOAD_POOL) {
          // 2x2 max, element by element, in the pooling loader's order
#pragma unroll
          for (int l = 1; l < LPV; ++l) {
            const uint4 o = xr[k][l < LPV ? l : 0];
            xv[k] = make_uint4(bf16_max2(xv[k].x, o.x), bf16_max2(xv[k].y, o.y), bf16_max2(xv[k].z, o.z),
                               bf16_max2(xv[k].w, o.w));
          }
        }
      }
      // sXt[dx][c][row][x] = X(row - 1, x + dx - 1): pixel hx0 + k of the halo
      // lands at x = hx0 + k - dx of copy dx
      const int h0 = x_hx0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        uint32_t e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = elem16(xv[k], j);
        uint16_t* r0 = &sXt[(0 * BC + x_cv + j) * CP + x_hr * XP];
        uint16_t* r1 = &sXt[(1 * BC + x_cv + j) * CP + x_hr * XP];
        uint16_t* r2 = &sXt[(2 * BC + x_cv + j) * CP + x_hr * XP];
        if (h0 + 3 < BX) *reinterpret_cast<uint2*>(r0 + h0) = make_uint2(e[0] | (e[1] << 16), e[2] | (e[3] << 16));
        if (h0 >= 1 && h0 - 1 < BX) r1[h0 - 1] = (uint16_t)e[0];
        if (h0 + 1 < BX) *reinterpret_cast<uint32_t*>(r1 + h0) = e[1] | (e[2] << 16);
        if (h0 + 2 < BX) r1[h0 + 2] = (uint16_t)e[3];
        if (h0 >= 2 && h0 - 1 < BX) *reinterpret_cast<uint32_t*>(r2 + h0 - 2) = e[0] | (e[1] << 16);
        if (h0 + 1 < BX) *reinterpret_cast<uint32_t*>(r2 + h0) = e[2] | (e[3] << 16);
      }
    }
  };

  if (split < n_chunks) fetch(split);
  for (int ch = split; ch < n_chunks; ch += a.splits) {
    commit();
    __syncthreads();
    if (ch + a.splits < n_chunks) fetch(ch + a.splits);  // in flight during the MFMAs
#pragma unroll
    for (int ks = 0; ks < BM / 32; ++ks) {
      const int pix0 = ks * 32 + kg * 8;  // this lane's 8 pixels (MFMA K index)
      const int row = pix0 / BX, xo = pix0 % BX;
      uint4 ga[FO];
#pragma unroll
      for (int f = 0; f < FO; ++f)
        ga[f] = *reinterpret_cast<const uint4*>(&sGt[(wm * (BO / 2) + f * 16 + l16) * GP + pix0]);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
        const uint4 xb = *reinterpret_cast<const uint4*>(&sXt[(dx * BC + wn * 16 + l16) * CP + (row + dy) * XP + xo]);
#pragma unroll
        for (int f = 0; f < FO; ++f)
          acc[tap][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ga[f]),
                                                                __builtin_bit_cast(bf16x8, xb), acc[tap][f], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* part = a.part + (int64_t)split * a.cout_p * 9 * a.cin_p;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int f = 0; f < FO; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + wm * (BO / 2) + f * 16 + kg * 4 + r;
        const int c = c0 + wn * 16 + l16;
        part[((int64_t)o * 9 + tap) * a.cin_p + c] = acc[tap][f][r];
      }
}

// canonical[(o cin + c) 9 + tap] = sum_s part[s][o][tap][cp(c)]: a workgroup
// takes 64 consecutive part entries (so the reads are coalesced), wave w the
// splits s = w mod 4 in order, then the four partial sums in a fixed order;
// padded input channels are dropped.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* part, int splits, int cout, int cin, int cu,
                                                      int cu_p, int cout_p, int cin_p, float* dst) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;  // (o, tap, cp) in [cout][9][cin_p]
  const int64_t n = (int64_t)cout * 9 * cin_p;
  const int64_t stride = (int64_t)cout_p * 9 * cin_p;
  float s = 0.f;
  if (j < n) {
#pragma unroll 8
    for (int k = w; k < splits; k += 4) s += part[k * stride + j];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < n) {
    const int cp = (int)(j % cin_p), tap = (int)((j / cin_p) % 9), o = (int)(j / (9LL * cin_p));
    // the upsampled channels first, then the skip channels, padding dropped
    const int c = cp < cu ? cp : (cp >= cu_p && cp - cu_p < cin - cu) ? cu + (cp - cu_p) : -1;
    if (c >= 0) dst[((int64_t)o * cin + c) * 9 + tap] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  }
}

int wgrad_bo(int cout_p) { return cout_p % 64 == 0 ? 64 : 32; }

// Weight gradient of the first conv (3 input channels, stored padded to
// x_cp): dW[o][c][ky][kx] = sum over pixels of dY[p][o] X[p + (ky - 1,
// kx - 1)][c], zero outside the tile.  The general kernel would run it as
// 32 input channels.  Here split `blockIdx.x` takes an equal range of the
// batch's tile rows and blockIdx.y a block of 64 output channels.  A row is
// taken in segments of 64 pixels: the segment's dY (64 pixels x 64
// channels, as FP32) and the three X rows around it (66 pixels x 3
// channels, zero outside the tile) are staged in LDS, then thread (ky, o)
// of wave ky runs along the segment with a three-pixel window of X row ky,
// nine FMAs per pixel, in pixel order.  part[split][o][tap][c] (c padded to
// 4) is reduced over the splits in order by k_wgrad_reduce.
constexpr int kFirstSeg = 64;

template <typename TG>
__global__ __launch_bounds__(256) void k_wgrad_first(const float* __restrict__ x, int x_cp, const TG* __restrict__ dy,
                                                     int cout_p, int T, int64_t rows, float* part) {
  constexpr int S = kFirstSeg, VEC = 16 / (int)sizeof(TG), NV = 64 / VEC;
  __shared__ float sG[S][64];
  __shared__ float sX[3][S + 2][3];
  const int tid = threadIdx.x, lane = tid & 63, ky = tid >> 6;
  const int ob = blockIdx.y * 64, o = ob + lane;
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(rows, r0 + per);
  float acc[3][3];
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[kx][c] = 0.f;
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t b = r / T;
    const int y = (int)(r % T);
    for (int x0 = 0; x0 < T; x0 += S) {
      const int len = min(S, T - x0);
      __syncthreads();  // the previous segment has been read
      for (int v = tid; v < S * NV; v += 256) {
        const int px = v / NV, j = v % NV;
        float g[VEC];
        if (px < len && ob + j * VEC < cout_p) {
          const uint4 u = *reinterpret_cast<const uint4*>(dy + ((b * T + y) * T + x0 + px) * cout_p + ob + j * VEC);
          if constexpr (VEC == 8) {
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              g[2 * k] = __uint_as_float(w[k] << 16);
              g[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
            }
          } else {
            g[0] = __uint_as_float(u.x);
            g[1] = __uint_as_float(u.y);
            g[2] = __uint_as_float(u.z);
            g[3] = __uint_as_float(u.w);
          }
        } else {
#pragma unroll
          for (int k = 0; k < VEC; ++k) g[k] = 0.f;
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k) sG[px][j * VEC + k] = g[k];
      }
      for (int v = tid; v < 3 * (S + 2) * 3; v += 256) {
        const int rr = v / ((S + 2) * 3), i = (v / 3) % (S + 2), c = v % 3;
        const int yy = y + rr - 1, xx = x0 + i - 1;
        float val = 0.f;
        if (yy >= 0 && yy < T && xx >= 0 && xx < T) val = x[((b * T + yy) * T + xx) * x_cp + c];
        sX[rr][i][c] = val;
      }
      __syncthreads();
      if (ky < 3) {
        float w0[3], w1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w0[c] = sX[ky][0][c];
          w1[c] = sX[ky][1][c];
        }
#pragma unroll 8
        for (int i = 0; i < len; ++i) {
          const float g = sG[i][lane];
          float w2[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            w2[c] = sX[ky][i + 2][c];
            acc[0][c] = fmaf(g, w0[c], acc[0][c]);
            acc[1][c] = fmaf(g, w1[c], acc[1][c]);
            acc[2][c] = fmaf(g, w2[c], acc[2][c]);
            w0[c] = w1[c];
            w1[c] = w2[c];
          }
        }
      }
    }
  }
  if (ky < 3 && o < cout_p) {
    float* dst = part + ((int64_t)blockIdx.x * cout_p + o) * 9 * 4;
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      const int tap = ky * 3 + kx;
#pragma unroll
      for (int c = 0; c < 3; ++c) dst[tap * 4 + c] = acc[kx][c];
      dst[tap * 4 + 3] = 0.f;
    }
  }
}

hipError_t launch_wgrad_first(int precision_g, const float* x, int x_cp, const void* dy, int n, int T, int cout,
                              int cout_p, float* part, int splits, float* dst, hipStream_t st) {
  if (splits < 1 || x_cp < 3 || cout_p % 8) return hipErrorInvalidValue;
  const int64_t rows = (int64_t)n * T;
  const dim3 grid(splits, ceil_div(cout_p, 64));
  if (precision_g == OMNISEG_BF16)
    hipLaunchKernelGGL(k_wgrad_first<uint16_t>, grid, dim3(256), 0, st, x, x_cp, (const uint16_t*)dy, cout_p, T, rows,
                       part);
  else
    hipLaunchKernelGGL(k_wgrad_first<float>, grid, dim3(256), 0, st, x, x_cp, (const float*)dy, cout_p, T, rows, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t m = (int64_t)cout * 9 * 4;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((m + 63) / 64)), dim3(256), 0, st, part, splits, cout, 3, 3, 4,
                     cout_p, 4, dst);
  return hipGetLastError();
}

hipError_t launch_wgrad(int precision_x, int precision_g, int loader, const WgradArgs& a, int cout, int cin,
                        int cu, float* dst, hipStream_t st) {
  if (a.cout_p % 32 || a.cin_p % 32) return hipErrorInvalidValue;
  const int bo = wgrad_bo(a.cout_p);
  const int blocks = (a.cout_p / bo) * (a.cin_p / 32) * a.splits;
  const bool bx16 = (a.W % 16 == 0);
#define OMNISEG_WG(TX, TG, BXV, LD)                                                                   \
  do {                                                                                              \
    if (bo == 64) hipLaunchKernelGGL((k_wgrad3x3<TX, TG, BXV, 64, LD>), dim3(blocks), dim3(256), 0, st, a); \
    else hipLaunchKernelGGL((k_wgrad3x3<TX, TG, BXV, 32, LD>), dim3(blocks), dim3(256), 0, st, a);          \
  } while (0)
#define OMNISEG_WG_LD(TX, TG, BXV)                                \
  do {                                                            \
    if (loader == LOAD_PLAIN) OMNISEG_WG(TX, TG, BXV, LOAD_PLAIN); \
    else if (loader == LOAD_POOL) OMNISEG_WG(TX, TG, BXV, LOAD_POOL); \
    else OMNISEG_WG(TX, TG, BXV, LOAD_UPCAT);                     \
  } while (0)
#define OMNISEG_WG_BX(TX, TG)             \
  do {                                    \
    if (bx16) OMNISEG_WG_LD(TX, TG, 16);  \
    else OMNISEG_WG_LD(TX, TG, 8);        \
  } while (0)
  const bool xb = precision_x == OMNISEG_BF16, gb = precision_g == OMNISEG_BF16;
#define OMNISEG_WGB(BXV, LD)                                                                                     \
  do {                                                                                                         \
    if (bo == 64) hipLaunchKernelGGL((k_wgrad3x3_bf16<BXV, 64, LD>), dim3(blocks), dim3(256), 0, st, a);        \
    else hipLaunchKernelGGL((k_wgrad3x3_bf16<BXV, 32, LD>), dim3(blocks), dim3(256), 0, st, a);                 \
  } while (0)
#define OMNISEG_WGB_LD(BXV)                                 \
  do {                                                      \
    if (loader == LOAD_PLAIN) OMNISEG_WGB(BXV, LOAD_PLAIN); \
    else if (loader == LOAD_POOL) OMNISEG_WGB(BXV, LOAD_POOL); \
    else OMNISEG_WGB(BXV, LOAD_UPCAT);                      \
  } while (0)
  if (xb && gb) {
    if (bx16) OMNISEG_WGB_LD(16);
    else OMNISEG_WGB_LD(8);
  }
#undef OMNISEG_WGB_LD
#undef OMNISEG_WGB
  else if (!xb && gb) OMNISEG_WG_BX(float, uint16_t);
  else if (xb && !gb) OMNISEG_WG_BX(uint16_t, float);
  else OMNISEG_WG_BX(float, float);
#undef OMNISEG_WG_BX
#undef OMNISEG_WG_LD
#undef OMNISEG_WG
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)cout * 9 * a.cin_p;  // part entries of the real output channels
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st, a.part, a.splits, cout,
                     cin, cu, a.cu_p, a.cout_p, a.cin_p, dst);
  return hipGetLastError();
}

// bias gradient: per-channel sum of dY over all pixels.  Split `split` of
// `splits` takes an equal pixel range; its threads read 16-byte vectors (V
// channels of one pixel): VL vector lanes cover a channel block of the
// pixel and the PL = 256 / VL pixel lanes of the workgroup take every PL-th
// pixel, four pixels in flight per thread.  The pixel lanes' sums are then
// added in LDS in lane order into part[split][c]; a second kernel adds the
// splits in order (deterministic).
template <typename T>
__global__ __launch_bounds__(256) void k_colsum(const T* dy, int64_t npix, int c_p, int splits, float* part) {
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ float red[256 * V];
  const int nvec = c_p / V;                 // vectors per pixel
  const int VL = nvec < 32 ? nvec : 32;     // vector lanes of a workgroup
  const int PL = 256 / VL;                  // pixel lanes
  const int t = threadIdx.x, vl = t % VL, pl = t / VL;
  const int split = blockIdx.y;
  const int c = (blockIdx.x * VL + vl) * V;
  const int64_t per = (npix + splits - 1) / splits;
  const int64_t p0 = split * per, p1 = min(npix, p0 + per);
  float acc[4][V];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int j = 0; j < V; ++j) acc[u][j] = 0.f;
  const bool live = pl < PL && c < c_p;
  if (live) {
    int64_t p = p0 + pl;
    for (; p + 3 * PL < p1; p += 4 * PL) {
      uint4 q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = *reinterpret_cast<const uint4*>(dy + (p + u * PL) * c_p + c);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < V; ++j) acc[u][j] += ldf(reinterpret_cast<const T*>(&q[u]) + j);
    }
    for (; p < p1; p += PL) {
      const uint4 q = *reinterpret_cast<const uint4*>(dy + p * c_p + c);
#pragma unroll
      for (int j = 0; j < V; ++j) acc[0][j] += ldf(reinterpret_cast<const T*>(&q) + j);
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) red[t * V + j] = (acc[0][j] + acc[1][j]) + (acc[2][j] + acc[3][j]);
  __syncthreads();
  if (pl == 0 && c < c_p) {
    float sv[V];
#pragma unroll
    for (int j = 0; j < V; ++j) sv[j] = red[vl * V + j];
    for (int q = 1; q < PL; ++q)
#pragma unroll
      for (int j = 0; j < V; ++j) sv[j] += red[(q * VL + vl) * V + j];
#pragma unroll
    for (int j = 0; j < V; ++j) part[(int64_t)split * c_p + c + j] = sv[j];
  }
}

// dst[c] = sum_s part[s][c]: 64 channels per workgroup, wave w the splits
// s = w mod 4 in order, then the four partial sums in a fixed order.
__global__ __launch_bounds__(256) void k_colsum_reduce(const float* part, int splits, int c_p, int cout, float* dst) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (c < cout) {
#pragma unroll 8
    for (int k = w; k < splits; k += 4) s += part[(int64_t)k * c_p + c];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && c < cout) dst[c] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

int bias_grad_splits(int64_t npix) { return (int)std::max<int64_t>(1, std::min<int64_t>(kBiasGradSplits, npix / 1024)); }

hipError_t launch_bias_grad(int precision, const void* dy, int64_t npix, int c_p, int cout, float* part,
                            int splits, float* dst, hipStream_t st) {
  if (c_p % 8 || (precision != OMNISEG_BF16 && c_p % 4)) return hipErrorInvalidValue;
  const int V = precision == OMNISEG_BF16 ? 8 : 4;
  const int VL = std::min(c_p / V, 32);
  dim3 grid(ceil_div(c_p / V, VL), splits);
  if (precision == OMNISEG_BF16)
    hipLaunchKernelGGL(k_colsum<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)dy, npix, c_p, splits, part);
  else
    hipLaunchKernelGGL(k_colsum<float>, grid, dim3(256), 0, st, (const float*)dy, npix, c_p, splits, part);
  hipLaunchKernelGGL(k_colsum_reduce, dim3((cout + 63) / 64), dim3(256), 0, st, part, splits, c_p, cout, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BCE-with-logits loss over the valid entries, mean over their count; FP64
// partial sums with a fixed-order final reduction
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bce_partial(const float* lg, const float* y, const uint8_t* valid,
                                                     int64_t n, double* part_sum, int* part_cnt) {
  __shared__ double rs[256];
  __shared__ int rc[256];
  double s = 0.0;
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (valid[i]) {
      const double L = lg[i], t = y[i];
      s += fmax(L, 0.0) - t * L + log1p(exp(-fabs(L)));
      ++c;
    }
  }
  rs[threadIdx.x] = s;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rc[threadIdx.x] += rc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_sum[blockIdx.x] = rs[0];
    part_cnt[blockIdx.x] = rc[0];
  }
}

__global__ void k_bce_final(const double* part_sum, const int* part_cnt, int nb, double* loss, int* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    long long c = 0;
    for (int i = 0; i < nb; ++i) {
      s += part_sum[i];
      c += part_cnt[i];
    }
    *loss = c > 0 ? s / (double)c : 0.0;
    *count = (int)c;
  }
}

__global__ void k_bce_grad(const float* lg, const float* y, const uint8_t* valid, int64_t n, const int* count,
                           float* grad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = *count;
  float g = 0.f;
  if (valid[i] && c > 0) {
    const float L = lg[i];
    const float sig = 1.f / (1.f + expf(-L));
    g = (sig - y[i]) / (float)c;
  }
  grad[i] = g;
}

hipError_t launch_bce(const float* lg, const float* y, const uint8_t* valid, int64_t n, double* part_sum,
                      int* part_cnt, int nb, double* loss, int* count, float* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_bce_partial, dim3(nb), dim3(256), 0, st, lg, y, valid, n, part_sum, part_cnt);
  hipLaunchKernelGGL(k_bce_final, dim3(1), dim3(64), 0, st, part_sum, part_cnt, nb, loss, count);
  if (grad)
    hipLaunchKernelGGL(k_bce_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lg, y, valid, n, count,
                       grad);
  return hipGetLastError();
}

}  // namespace omniseg

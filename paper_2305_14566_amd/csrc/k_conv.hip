// 3x3 convolutions of the residual U-Net backbone on gfx950.
//
// Each conv is an implicit GEMM: M = output pixels of a batch of tiles,
// N = output channels, K = 9 taps x input channels.  Activations are NHWC
// with channels padded to a multiple of 32, so one K-chunk of a pixel is a
// contiguous 16-byte vector.  A workgroup owns a BY x BX pixel block of one
// tile and BN output channels; per input-channel chunk it stages the
// (BY+2) x (BX+2) halo patch once in LDS and reuses it for all nine taps
// (9x reuse of every activation load), together with the chunk's weights
// for the nine taps.  Four waves each own a (BM/WM) x (BN/WN) sub-tile of
// 16x16 MFMA fragments with FP32 accumulators.
//
//   BF16: v_mfma_f32_16x16x32_bf16, one 16-byte LDS read per operand and
//         fragment covers K = 32.
//   FP32: v_mfma_f32_16x16x4_f32.  A 16-byte LDS read gives a lane four
//         consecutive K values; MFMA step s (s = 0..3) feeds element s, so
//         lane group j covers K = 4 j + s.  A and B use the same mapping, so
//         the four steps together sum over all 16 K values of the fragment.
//
// Loaders fuse the layer's input transform: PLAIN (NHWC), POOL (2x2 max of
// the previous level's output, read at twice the resolution) and UPCAT
// (nearest 2x upsampling of the coarser decoder output for the first cu_p
// channels, then the encoder skip).  Zero padding applies at the tile
// border.  Epilogues: bias + ReLU, or bias + residual (the conv's own input)
// + ReLU.
#include "internal.h"

#include <type_traits>

namespace omniseg {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (inputs are finite)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename T>
struct ConvTraits;
template <>
struct ConvTraits<float> {
  static constexpr int KC = 16;   // channels per LDS chunk
  static constexpr int VEC = 4;   // elements per 16-byte vector
  static constexpr int ROW = 20;  // LDS row length (80 bytes)
};
template <>
struct ConvTraits<uint16_t> {
  static constexpr int KC = 32;
  static constexpr int VEC = 8;
  static constexpr int ROW = 40;
};
template <>
struct ConvTraits<uint8_t> {
  static constexpr int KC = kFp8Chunk;  // 64 FP8 channels = 64 bytes per pixel
  static constexpr int VEC = 16;
  static constexpr int ROW = 80;
};

struct ConvArgs {
  const void* x0;
  const void* x1;
  const void* aux;  // EPI_RES_MASK: the activation whose sign gates the output
  void* y;
  const void* w;
  const float* bias;
  int H, W;
  int cin_p, cu_p, cout_p;
  const int32_t* count;
  int chunk_base;
  int tiles_y, tiles_x, n_nblk;
  const float* wscale;  // FP8 epilogue scales (see ConvLayer)
  const float* rscale;
  const float* oinv;
  void* pool_out;  // row-reuse epilogues: also write the 2x2 max-pool of y here (or null)
  int batch;       // tiles the launch covers (the persistent form loops over them)
  const float* pre_w;  // EPI_RES_RELU_PRECLS: precls weights [8][64] and bias [8];
  const float* pre_b;  // F = ReLU(W_p D + b_p) goes to fpre [tile][H W][8] instead
  float* fpre;         // of D to y
};

__device__ __forceinline__ uint4 vmax(uint4 a, uint4 b, float) {
  uint4 r;
  r.x = __float_as_uint(fmaxf(__uint_as_float(a.x), __uint_as_float(b.x)));
  r.y = __float_as_uint(fmaxf(__uint_as_float(a.y), __uint_as_float(b.y)));
  r.z = __float_as_uint(fmaxf(__uint_as_float(a.z), __uint_as_float(b.z)));
  r.w = __float_as_uint(fmaxf(__uint_as_float(a.w), __uint_as_float(b.w)));
  return r;
}
__device__ __forceinline__ uint32_t bmax2(uint32_t a, uint32_t b) {
  float a0 = bf2f(a & 0xffff), a1 = bf2f(a >> 16), b0 = bf2f(b & 0xffff), b1 = bf2f(b >> 16);
  return (uint32_t)f2bf(fmaxf(a0, b0)) | ((uint32_t)f2bf(fmaxf(a1, b1)) << 16);
}
__device__ __forceinline__ uint4 vmax(uint4 a, uint4 b, uint16_t) {
  return make_uint4(bmax2(a.x, b.x), bmax2(a.y, b.y), bmax2(a.z, b.z), bmax2(a.w, b.w));
}
// FP8 activations are ReLU outputs: non-negative E4M3 codes (sign bit clear)
// order like their values, so the max of the codes is the code of the max.
__device__ __forceinline__ uint32_t u8max4(uint32_t a, uint32_t b) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 32; i += 8) r |= max((a >> i) & 0xffu, (b >> i) & 0xffu) << i;
  return r;
}
__device__ __forceinline__ uint4 vmax(uint4 a, uint4 b, uint8_t) {
  return make_uint4(u8max4(a.x, b.x), u8max4(a.y, b.y), u8max4(a.z, b.z), u8max4(a.w, b.w));
}

template <typename T, int LOADER>
__device__ __forceinline__ uint4 load_vec(const ConvArgs& a, int b, int y, int x, int c) {
  if (LOADER == LOAD_PLAIN) {
    const T* p = (const T*)a.x0 + (((int64_t)b * a.H + y) * a.W + x) * a.cin_p + c;
    return *reinterpret_cast<const uint4*>(p);
  } else if (LOADER == LOAD_POOL) {
    const int H2 = 2 * a.H, W2 = 2 * a.W;
    const T* p = (const T*)a.x0 + (((int64_t)b * H2 + 2 * y) * W2 + 2 * x) * a.cin_p + c;
    uint4 v00 = *reinterpret_cast<const uint4*>(p);
    uint4 v01 = *reinterpret_cast<const uint4*>(p + a.cin_p);
    uint4 v10 = *reinterpret_cast<const uint4*>(p + (int64_t)W2 * a.cin_p);
    uint4 v11 = *reinterpret_cast<const uint4*>(p + (int64_t)W2 * a.cin_p + a.cin_p);
    return vmax(vmax(v00, v01, T()), vmax(v10, v11, T()), T());
  } else {
    if (c < a.cu_p) {
      const int Hh = a.H >> 1, Wh = a.W >> 1;
      const T* p = (const T*)a.x0 + (((int64_t)b * Hh + (y >> 1)) * Wh + (x >> 1)) * a.cu_p + c;
      return *reinterpret_cast<const uint4*>(p);
    } else {
      const int ce_p = a.cin_p - a.cu_p;
      const T* p = (const T*)a.x1 + (((int64_t)b * a.H + y) * a.W + x) * ce_p + (c - a.cu_p);
      return *reinterpret_cast<const uint4*>(p);
    }
  }
}

// Issue the global loads of one 16-byte input vector without waiting for
// them: POOL keeps its four raw vectors (reduced when committed to LDS).
template <typename T, int LOADER>
__device__ __forceinline__ void fetch_vec(const ConvArgs& a, int b, int y, int x, int c, uint4* r) {
  if (LOADER == LOAD_POOL) {
    const int W2 = 2 * a.W;
    const T* p = (const T*)a.x0 + (((int64_t)b * 2 * a.H + 2 * y) * W2 + 2 * x) * a.cin_p + c;
    r[0] = *reinterpret_cast<const uint4*>(p);
    r[1] = *reinterpret_cast<const uint4*>(p + a.cin_p);
    r[2] = *reinterpret_cast<const uint4*>(p + (int64_t)W2 * a.cin_p);
    r[3] = *reinterpret_cast<const uint4*>(p + (int64_t)W2 * a.cin_p + a.cin_p);
  } else {
    r[0] = load_vec<T, LOADER>(a, b, y, x, c);
  }
}

__device__ __forceinline__ void mma(f32x4& acc, uint4 av, uint4 bv, float) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.x), __uint_as_float(bv.x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.y), __uint_as_float(bv.y), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.z), __uint_as_float(bv.z), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.w), __uint_as_float(bv.w), acc, 0, 0, 0);
}
__device__ __forceinline__ void mma(f32x4& acc, uint4 av, uint4 bv, uint16_t) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
}

__device__ __forceinline__ float load_scalar(const float* p) { return *p; }
__device__ __forceinline__ float load_scalar(const uint16_t* p) { return bf2f(*p); }
__device__ __forceinline__ void store_scalar(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_scalar(uint16_t* p, float v) { *p = f2bf(v); }

// Global -> register -> LDS staging of one input-channel chunk.  Each thread
// owns HPT halo vectors (LPV raw loads each; HALO_V in total) and WPT weight
// vectors (W_V in total); fetch issues the loads, commit writes LDS.
// LDS slot of 16-byte vector v of row p.  SWZ: rows of exactly NV = 4
// vectors (64 bytes, no padding) with the vectors of row p rotated by
// (p >> 1) & 3.  With gfx950's ds_read_b128 lane grouping (16 lanes per
// cycle over 64 four-byte banks; a cycle takes lanes 0-31 or 32-63 and the
// quads (lane / 4) of equal bit-0..2 parity) that makes the MFMA operand
// reads -- 16 consecutive rows, vector g = lane / 16 -- conflict-free for
// every starting row, where an 80-byte pitch costs 4 extra cycles each.
template <bool SWZ>
__device__ __forceinline__ int vslot(int p, int v) {
  return SWZ ? ((v + (p >> 1)) & 3) : v;
}

template <typename T, int LOADER, int HALO_V, int W_V, int LPV, int NV, int VEC, int KC, int ROW, int PX, int BN,
          bool SWZ = false, int NT = 256>
struct Stager {
  static_assert(!SWZ || (NV == 4 && ROW == NV * VEC), "swizzled rows hold exactly four vectors");
  static constexpr int HPT = (HALO_V + NT - 1) / NT;
  static constexpr int WPT = (W_V + NT - 1) / NT;
  __device__ __forceinline__ static void fetch(const ConvArgs& a, int b, int tid, int y0, int x0, int n0, int ch,
                                               uint4 (&hreg)[HPT][LPV], uint4 (&wreg)[WPT]) {
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const int idx = tid + i * NT;
#pragma unroll
      for (int j = 0; j < LPV; ++j) hreg[i][j] = make_uint4(0, 0, 0, 0);
      if (idx < HALO_V) {
        const int p = idx / NV, v = idx % NV;
        const int y = y0 + p / PX - 1, x = x0 + p % PX - 1;
        const int c = ch * KC + v * VEC;  // beyond cin_p only in an FP8 chunk's padding
        if (y >= 0 && y < a.H && x >= 0 && x < a.W && c < a.cin_p) fetch_vec<T, LOADER>(a, b, y, x, c, hreg[i]);
      }
    }
    const T* wsrc = (const T*)a.w + (int64_t)ch * 9 * a.cout_p * KC;
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int idx = tid + i * NT;
      wreg[i] = make_uint4(0, 0, 0, 0);
      if (idx < W_V) {
        const int v = idx % NV, r = idx / NV;
        const int tap = r / BN, n = r % BN;
        wreg[i] = *reinterpret_cast<const uint4*>(wsrc + ((int64_t)tap * a.cout_p + n0 + n) * KC + v * VEC);
      }
    }
  }
  __device__ __forceinline__ static void commit(int tid, const uint4 (&hreg)[HPT][LPV], const uint4 (&wreg)[WPT],
                                                T* sX, T* sW) {
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const int idx = tid + i * NT;
      if (idx < HALO_V) {
        const int p = idx / NV, v = idx % NV;
        uint4 val = hreg[i][0];
        if (LPV == 4)
          val = vmax(vmax(hreg[i][0], hreg[i][LPV > 1 ? 1 : 0], T()),
                     vmax(hreg[i][LPV > 2 ? 2 : 0], hreg[i][LPV > 3 ? 3 : 0], T()), T());
        *reinterpret_cast<uint4*>(&sX[p * ROW + vslot<SWZ>(p, v) * VEC]) = val;
      }
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int idx = tid + i * NT;
      if (idx < W_V) {
        const int v = idx % NV, r = idx / NV;
        *reinterpret_cast<uint4*>(&sW[r * ROW + vslot<SWZ>(r, v) * VEC]) = wreg[i];
      }
    }
  }
};

// Buffer resource (gfx9 layout: 48-bit base, stride 0, byte range, default
// format word) over `bytes` bytes at p.  A buffer load whose offset lies at
// or beyond the range returns zeros and touches no memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint4 buffer_load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
constexpr uint32_t kOutside = 0x80000000u;  // a byte offset beyond every range used here

// Staging for the row-reuse kernels (BF16 and FP8) with the address
// arithmetic hoisted out of the chunk loop.  A thread's halo vectors sit at
// fixed pixels and always at vector v = tid % NV of a pixel's chunk, so
// their byte offsets inside the tile (one per source tensor; kOutside for
// pixels outside the image, which then load zeros) and its weight vectors'
// offsets inside a chunk are computed once.  Each chunk builds buffer
// resources that start at its channel offset and end at the end of the tile
// (or of the chunk's weights), so a load is one instruction with no branch.
// Two uniform cases need more: an FP8 chunk (64 channels) that runs past
// cin_p (multiples of 32) zeroes the vectors beyond it, and an FP8 UPCAT
// chunk that straddles the end of the upsampled channels issues both loads,
// one of them outside its range.  A tile holds at most 512^2 pixels x 4096
// channels x 2 bytes = 2^31 bytes.
template <typename T, int LOADER, int HALO_V, int W_V, int LPV, int NV, int VEC, int KC, int ROW, int PX, int BN,
          bool SWZ, int NT>
struct RowStager {
  static constexpr int HPT = (HALO_V + NT - 1) / NT;
  static constexpr int WPT = (W_V + NT - 1) / NT;
  static_assert(NT % NV == 0, "a thread's halo vectors share one vector slot");
  const T* x0b;  // this tile's first element in x0
  const T* x1b;  // and in x1 (UPCAT)
  uint32_t bytes0, bytes1;
  uint32_t o0[HPT], o1[HPT], wo[WPT];
  int vc;  // channel offset of this thread's halo vectors inside a chunk
  int cu_p, cin_p, chunk_w;
  uint32_t pool_dx, pool_dy;

  __device__ __forceinline__ RowStager(const ConvArgs& a, int b, int tid, int y0, int x0, int n0) {
    const int H = a.H, W = a.W;
    cu_p = a.cu_p;
    cin_p = a.cin_p;
    chunk_w = 9 * a.cout_p * KC;
    pool_dx = (uint32_t)a.cin_p * sizeof(T);
    pool_dy = (uint32_t)(2 * W) * a.cin_p * sizeof(T);
    vc = (tid % NV) * VEC;
    int64_t tile0;
    if (LOADER == LOAD_POOL) tile0 = (int64_t)4 * H * W * a.cin_p;
    else if (LOADER == LOAD_UPCAT) tile0 = (int64_t)(H >> 1) * (W >> 1) * a.cu_p;
    else tile0 = (int64_t)H * W * a.cin_p;
    x0b = (const T*)a.x0 + (int64_t)b * tile0;
    bytes0 = (uint32_t)(tile0 * sizeof(T));
    const int64_t tile1 = (int64_t)H * W * (a.cin_p - a.cu_p);
    x1b = LOADER == LOAD_UPCAT ? (const T*)a.x1 + (int64_t)b * tile1 : nullptr;
    bytes1 = (uint32_t)(tile1 * sizeof(T));
    const uint32_t vb = (uint32_t)(vc * sizeof(T));
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const int idx = tid + i * NT;
      const int p = idx / NV;
      const int y = y0 + p / PX - 1, x = x0 + p % PX - 1;
      const bool in = idx < HALO_V && y >= 0 && y < H && x >= 0 && x < W;
      if (LOADER == LOAD_POOL) {
        o0[i] = in ? (uint32_t)(((2 * y) * (2 * W) + 2 * x) * a.cin_p) * sizeof(T) + vb : kOutside;
      } else if (LOADER == LOAD_UPCAT) {
        o0[i] = in ? (uint32_t)(((y >> 1) * (W >> 1) + (x >> 1)) * a.cu_p) * sizeof(T) + vb : kOutside;
        o1[i] = in ? (uint32_t)((y * W + x) * (a.cin_p - a.cu_p)) * sizeof(T) + vb : kOutside;
      } else {
        o0[i] = in ? (uint32_t)((y * W + x) * a.cin_p) * sizeof(T) + vb : kOutside;
      }
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int idx = tid + i * NT;
      const int v = idx % NV, r = idx / NV;
      const int tap = r / BN, n = r % BN;
      wo[i] = idx < W_V ? (uint32_t)(((tap * a.cout_p + n0 + n) * KC + v * VEC) * sizeof(T)) : kOutside;
    }
  }

  // Loads of one source over the chunk starting at channel c of it: every
  // vector at or beyond channel `lim` of the source reads zeros.
  __device__ __forceinline__ void load_src(const T* base, uint32_t bytes, const uint32_t (&off)[HPT], int c, int lim,
                                           uint4 (&hreg)[HPT][LPV], bool live) const {
    const __amdgpu_buffer_rsrc_t r = buffer_rsrc(base + c, live ? bytes - (uint32_t)(c * sizeof(T)) : 0u);
    const bool keep = c + vc < lim;
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const uint32_t o = keep ? off[i] : kOutside;
      hreg[i][0] = buffer_load16(r, o);
      if (LOADER == LOAD_POOL) {
        hreg[i][LPV > 1 ? 1 : 0] = buffer_load16(r, o + pool_dx);
        hreg[i][LPV > 2 ? 2 : 0] = buffer_load16(r, o + pool_dy);
        hreg[i][LPV > 3 ? 3 : 0] = buffer_load16(r, o + pool_dy + pool_dx);
      }
    }
  }

  // live = false issues the same loads over empty ranges: they return zeros
  // without touching memory (the unused fetch of a branch-free loop's last pass).
  __device__ __forceinline__ void fetch(const ConvArgs& a, int ch, uint4 (&hreg)[HPT][LPV], uint4 (&wreg)[WPT],
                                        bool live = true) const {
    const int c = ch * KC;
    if (LOADER == LOAD_UPCAT) {
      if (c + KC <= cu_p) {
        load_src(x0b, bytes0, o0, c, cu_p, hreg, live);
      } else if (c >= cu_p) {
        load_src(x1b, bytes1, o1, c - cu_p, cin_p - cu_p, hreg, live);
      } else {  // the chunk straddles the end of the upsampled channels (FP8 only)
        uint4 h1[HPT][LPV];
        load_src(x0b, bytes0, o0, c, cu_p, hreg, live);
        const __amdgpu_buffer_rsrc_t r1 = buffer_rsrc(x1b, live ? bytes1 : 0u);
        const bool second = c + vc >= cu_p && c + vc < cin_p;
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
          const bool use = second && o1[i] != kOutside;
          h1[i][0] = buffer_load16(r1, use ? o1[i] + (uint32_t)((c - cu_p) * (int)sizeof(T)) : kOutside);
          hreg[i][0] = make_uint4(hreg[i][0].x | h1[i][0].x, hreg[i][0].y | h1[i][0].y, hreg[i][0].z | h1[i][0].z,
                                  hreg[i][0].w | h1[i][0].w);
        }
      }
    } else {
      load_src(x0b, bytes0, o0, c, cin_p, hreg, live);
    }
    const __amdgpu_buffer_rsrc_t rw =
        buffer_rsrc((const T*)a.w + (int64_t)ch * chunk_w, live ? (uint32_t)(chunk_w * sizeof(T)) : 0u);
#pragma unroll
    for (int i = 0; i < WPT; ++i) wreg[i] = buffer_load16(rw, wo[i]);
  }

  __device__ __forceinline__ static void commit(int tid, const uint4 (&hreg)[HPT][LPV], const uint4 (&wreg)[WPT],
                                                T* sX, T* sW) {
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const int idx = tid + i * NT;
      if (idx < HALO_V) {
        const int p = idx / NV, v = idx % NV;
        uint4 val = hreg[i][0];
        if (LPV == 4)
          val = vmax(vmax(hreg[i][0], hreg[i][LPV > 1 ? 1 : 0], T()),
                     vmax(hreg[i][LPV > 2 ? 2 : 0], hreg[i][LPV > 3 ? 3 : 0], T()), T());
        *reinterpret_cast<uint4*>(&sX[p * ROW + vslot<SWZ>(p, v) * VEC]) = val;
      }
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int idx = tid + i * NT;
      if (idx < W_V) {
        const int v = idx % NV, r = idx / NV;
        *reinterpret_cast<uint4*>(&sW[r * ROW + vslot<SWZ>(r, v) * VEC]) = wreg[i];
      }
    }
  }
};

template <typename T, int BY, int BX, int BN, int WM, int WN, int LOADER, int EPI>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a) {
  using TR = ConvTraits<T>;
  constexpr int KC = TR::KC, VEC = TR::VEC, ROW = TR::ROW;
  constexpr int NV = KC / VEC;  // 16-byte vectors per pixel chunk
  constexpr int BM = BY * BX;
  constexpr int PX = BX + 2, NPIX = (BY + 2) * PX;
  constexpr int MW = BM / WM, NW = BN / WN;  // wave sub-tile
  constexpr int FM = MW / 16, FN = NW / 16;
  static_assert(WM * WN == 4, "four waves");
  static_assert(FM >= 1 && FN >= 1 && MW % 16 == 0 && NW % 16 == 0, "fragment shape");
  __shared__ __attribute__((aligned(16))) T sX[NPIX * ROW];
  __shared__ __attribute__((aligned(16))) T sW[9 * BN * ROW];

  int rest = blockIdx.x;
  const int nb = rest % a.n_nblk;
  rest /= a.n_nblk;
  const int sxb = rest % a.tiles_x;
  rest /= a.tiles_x;
  const int syb = rest % a.tiles_y;
  const int b = rest / a.tiles_y;
  if (a.chunk_base + b >= *a.count) return;
  const int y0 = syb * BY, x0 = sxb * BX, n0 = nb * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int kg = (lane >> 4) * VEC;  // K offset of this lane inside a fragment
  const int l16 = lane & 15;

  int a_off[FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
    const int m = wm * MW + fm * 16 + l16;
    a_off[fm] = ((m / BX) * PX + (m % BX)) * ROW + kg;
  }
  int b_off[FN];
#pragma unroll
  for (int fn = 0; fn < FN; ++fn) b_off[fn] = (wn * NW + fn * 16 + l16) * ROW + kg;

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Staging: each thread owns HPT halo vectors and WPT weight vectors of a
  // chunk.  The next chunk's global loads are issued before the current
  // chunk's MFMAs and committed to LDS after them, so their latency overlaps
  // the arithmetic.
  constexpr int HALO_V = NPIX * NV, W_V = 9 * BN * NV;
  constexpr int HPT = (HALO_V + 255) / 256, WPT = (W_V + 255) / 256;
  constexpr int LPV = (LOADER == LOAD_POOL) ? 4 : 1;
  uint4 hreg[HPT][LPV];
  uint4 wreg[WPT];
  const int nchunks = a.cin_p / KC;
  using ST = Stager<T, LOADER, HALO_V, W_V, LPV, NV, VEC, KC, ROW, PX, BN>;
  ST::fetch(a, b, tid, y0, x0, n0, 0, hreg, wreg);
  ST::commit(tid, hreg, wreg, sX, sW);
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    if (ch + 1 < nchunks) ST::fetch(a, b, tid, y0, x0, n0, ch + 1, hreg, wreg);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int sh = ((tap / 3) * PX + (tap % 3)) * ROW;
#pragma unroll
      for (int kk = 0; kk < KC / (4 * VEC); ++kk) {
        uint4 av[FM], bv[FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) av[fm] = *reinterpret_cast<const uint4*>(&sX[a_off[fm] + sh + kk * 4 * VEC]);
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
          bv[fn] = *reinterpret_cast<const uint4*>(&sW[tap * BN * ROW + b_off[fn] + kk * 4 * VEC]);
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn) mma(acc[fm][fn], av[fm], bv[fn], T());
      }
    }
    __syncthreads();
    if (ch + 1 < nchunks) {
      ST::commit(tid, hreg, wreg, sX, sW);
      __syncthreads();
    }
  }

  T* out = (T*)a.y;
  const T* res = (const T*)a.x0;
#pragma unroll
  for (int fn = 0; fn < FN; ++fn) {
    const int n = n0 + wn * NW + fn * 16 + l16;
    const float bias = (EPI == EPI_RELU || EPI == EPI_RES_RELU) ? a.bias[n] : 0.f;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = wm * MW + fm * 16 + (lane >> 4) * 4 + r;
        const int y = y0 + m / BX, x = x0 + m % BX;
        const int64_t o = (((int64_t)b * a.H + y) * a.W + x) * a.cout_p + n;
        if (EPI == EPI_NONE) {
          store_scalar(out + o, acc[fm][fn][r]);
        } else if (EPI == EPI_RES_MASK) {
          // gradient through "ReLU(conv(A) + A)" back to A's pre-activation:
          // (acc + g) where the recomputed A is positive, else 0
          const float v = acc[fm][fn][r] + load_scalar(res + o);
          store_scalar(out + o, load_scalar((const T*)a.aux + o) > 0.f ? v : 0.f);
        } else {
          float v = acc[fm][fn][r] + bias;
          if (EPI == EPI_RES_RELU) v += load_scalar(res + o);
          store_scalar(out + o, fmaxf(v, 0.f));
        }
      }
    }
  }
}

// BF16 row-reuse form.  The block is BY rows x 16 pixels x BN channels; a
// wave owns FM = BY / WM whole rows (one 16-pixel MFMA fragment each) and
// BN / WN channels.  For each horizontal tap offset dx it reads the FM + 2
// halo rows it needs once and feeds them to the three vertical taps, so an
// input fragment read serves up to three MFMA groups instead of one.  The
// weights are the MFMA's A operand (rows = output channels) and the pixels
// its B operand, so each lane's accumulator holds four consecutive channels
// of one pixel; the epilogue stages the FP32 results through LDS and writes
// 16-byte vectors of the output (and reads the residual the same way).
// Rounding is the same as in k_conv3x3: bias, residual and ReLU in FP32 on
// the accumulator, then one rounding to BF16.
template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
// Two waves per SIMD where the registers allow it without spilling; the
// 128-channel block and the pooled loads of the larger blocks (four raw
// vectors staged per halo vector) take one; eight-wave blocks aim at four
// waves per SIMD.
__global__ __launch_bounds__(64 * WM * WN,
                             (WM * WN == 8 ? 4 : ((BN >= 128 || (LOADER == LOAD_POOL && BY * BN > 512)) ? 1 : 2)))
void k_conv3x3_rows(ConvArgs a) {
  using T = uint16_t;
  using TR = ConvTraits<T>;
  constexpr int KC = TR::KC, VEC = TR::VEC;
  constexpr int NV = KC / VEC;
  constexpr int ROW = KC;  // 64-byte rows, vectors rotated per row (vslot<true>)
  constexpr int BX = 16, PX = BX + 2, NPIX = (BY + 2) * PX;
  constexpr int FM = BY / WM;
  constexpr int NW = BN / WN, FN = NW / 16;
  constexpr int NT = 64 * WM * WN;  // four or eight waves
  static_assert((WM * WN == 4 || WM * WN == 8) && BY % WM == 0 && NW % 16 == 0, "wave layout");
  constexpr int MAIN_B = (NPIX + 9 * BN) * ROW * (int)sizeof(T);
  constexpr int OROW = BN + 4;  // FP32 values per pixel in the epilogue staging
  constexpr int EPI_B = BY * BX * OROW * 4;
  constexpr int SMEM_B = MAIN_B > EPI_B ? MAIN_B : EPI_B;
  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM_B];
  T* sX = reinterpret_cast<T*>(smem);
  T* sW = sX + NPIX * ROW;

  int rest = xcd_remap(blockIdx.x, gridDim.x);
  const int nb = rest % a.n_nblk;
  rest /= a.n_nblk;
  const int sxb = rest % a.tiles_x;
  rest /= a.tiles_x;
  const int syb = rest % a.tiles_y;
  const int b = rest / a.tiles_y;
  if (a.chunk_base + b >= *a.count) return;
  const int y0 = syb * BY, x0 = sxb * BX, n0 = nb * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int g = lane >> 4;  // K vector of this lane
  const int l16 = lane & 15;
  const int xrow = wm * FM * PX + l16;  // halo pixel of row wm*FM, column l16 (dx = 0)
  const int wrow = wn * NW + l16;

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  constexpr int HALO_V = NPIX * NV, W_V = 9 * BN * NV;
  constexpr int HPT = (HALO_V + NT - 1) / NT, WPT = (W_V + NT - 1) / NT;
  constexpr int LPV = (LOADER == LOAD_POOL) ? 4 : 1;
  uint4 hreg[HPT][LPV];
  uint4 wreg[WPT];
  const int nchunks = a.cin_p / KC;
  using ST = RowStager<T, LOADER, HALO_V, W_V, LPV, NV, VEC, KC, ROW, PX, BN, true, NT>;
  const ST st(a, b, tid, y0, x0, n0);
  st.fetch(a, 0, hreg, wreg);
  ST::commit(tid, hreg, wreg, sX, sW);
  __syncthreads();
  // The loop body has no branch (the last pass issues an empty fetch and
  // commits zeros, unused), so the scheduler can interleave the next chunk's
  // loads and the LDS address arithmetic with the MFMAs.
  for (int ch = 0; ch < nchunks; ++ch) {
    st.fetch(a, min(ch + 1, nchunks - 1), hreg, wreg, ch + 1 < nchunks);
    // Waves in their MFMA phase issue first.  Measured per layer: 1.5-2.3 %
    // faster for the upsample-and-concat convs, 4 % slower for residual ones.
    if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      uint4 xv[FM + 2];
#pragma unroll
      for (int r = 0; r < FM + 2; ++r) {
        const int px = xrow + r * PX + dx;
        xv[r] = *reinterpret_cast<const uint4*>(&sX[px * ROW + vslot<true>(px, g) * VEC]);
      }
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int tap = dy * 3 + dx;
        uint4 wv[FN];
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
          const int wr = tap * BN + wrow + fn * 16;
          wv[fn] = *reinterpret_cast<const uint4*>(&sW[wr * ROW + vslot<true>(wr, g) * VEC]);
        }
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn) mma(acc[fm][fn], wv[fn], xv[fm + dy], T());
      }
    }
    if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    ST::commit(tid, hreg, wreg, sX, sW);
    __syncthreads();
  }

  // Epilogue: accumulators -> LDS [pixel][channel] (FP32) -> 16-byte rows.
  float* sO = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
      const int p = (wm * FM + fm) * BX + l16;
      const int c = wn * NW + fn * 16 + (lane >> 4) * 4;
      *reinterpret_cast<f32x4*>(&sO[p * OROW + c]) = acc[fm][fn];
    }
  __syncthreads();
  constexpr int NVO = BN / 8;
  T* out = (T*)a.y;
  const T* res = (const T*)a.x0;
  for (int i = tid; i < BY * BX * NVO; i += NT) {
    const int p = i / NVO, c = (i % NVO) * 8;
    const int y = y0 + p / BX, x = x0 + p % BX, n = n0 + c;
    const int64_t o = (((int64_t)b * a.H + y) * a.W + x) * a.cout_p + n;
    const f32x4 lo = *reinterpret_cast<const f32x4*>(&sO[p * OROW + c]);
    const f32x4 hi = *reinterpret_cast<const f32x4*>(&sO[p * OROW + c + 4]);
    float v[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    if (EPI == EPI_RELU || EPI == EPI_RES_RELU) {
      const float4 b0 = *reinterpret_cast<const float4*>(a.bias + n);
      const float4 b1 = *reinterpret_cast<const float4*>(a.bias + n + 4);
      v[0] += b0.x; v[1] += b0.y; v[2] += b0.z; v[3] += b0.w;
      v[4] += b1.x; v[5] += b1.y; v[6] += b1.z; v[7] += b1.w;
    }
    if (EPI == EPI_RES_RELU || EPI == EPI_RES_MASK) {
      const uint4 r = *reinterpret_cast<const uint4*>(res + o);
      const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[2 * j] += bf2f(rw[j] & 0xffff);
        v[2 * j + 1] += bf2f(rw[j] >> 16);
      }
    }
    if (EPI == EPI_RES_MASK) {
      const uint4 g = *reinterpret_cast<const uint4*>((const T*)a.aux + o);
      const uint32_t gw[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!(bf2f(gw[j] & 0xffff) > 0.f)) v[2 * j] = 0.f;
        if (!(bf2f(gw[j] >> 16) > 0.f)) v[2 * j + 1] = 0.f;
      }
    }
    if (EPI == EPI_RELU || EPI == EPI_RES_RELU) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = fmaxf(v[j], 0.f);
    }
    uint4 u;
    u.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
    u.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
    u.z = (uint32_t)f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16);
    u.w = (uint32_t)f2bf(v[6]) | ((uint32_t)f2bf(v[7]) << 16);
    *reinterpret_cast<uint4*>(out + o) = u;
    if (a.pool_out) {  // keep the final values for the pooled copy
      *reinterpret_cast<f32x4*>(&sO[p * OROW + c]) = f32x4{v[0], v[1], v[2], v[3]};
      *reinterpret_cast<f32x4*>(&sO[p * OROW + c + 4]) = f32x4{v[4], v[5], v[6], v[7]};
    }
  }
  if (a.pool_out) {
    // 2x2 max-pool of the block's output (BY and 16 are even, blocks start at
    // even coordinates): max commutes with the monotonic BF16 rounding, so
    // this is the pool of the stored output.
    __syncthreads();
    T* pout = (T*)a.pool_out;
    const int Hh = a.H >> 1, Wh = a.W >> 1;
    for (int i = tid; i < (BY / 2) * (BX / 2) * NVO; i += NT) {
      const int q = i / NVO, c = (i % NVO) * 8;
      const int py = q / (BX / 2), px = q % (BX / 2);
      const int p00 = (2 * py) * BX + 2 * px;
      float m[8];
#pragma unroll
      for (int j = 0; j < 8; j += 4) {
        const f32x4 a0 = *reinterpret_cast<const f32x4*>(&sO[p00 * OROW + c + j]);
        const f32x4 a1 = *reinterpret_cast<const f32x4*>(&sO[(p00 + 1) * OROW + c + j]);
        const f32x4 a2 = *reinterpret_cast<const f32x4*>(&sO[(p00 + BX) * OROW + c + j]);
        const f32x4 a3 = *reinterpret_cast<const f32x4*>(&sO[(p00 + BX + 1) * OROW + c + j]);
#pragma unroll
        for (int k = 0; k < 4; ++k) m[j + k] = fmaxf(fmaxf(a0[k], a1[k]), fmaxf(a2[k], a3[k]));
      }
      const int64_t o = (((int64_t)b * Hh + (y0 >> 1) + py) * Wh + (x0 >> 1) + px) * a.cout_p + n0 + c;
      uint4 u;
      u.x = (uint32_t)f2bf(m[0]) | ((uint32_t)f2bf(m[1]) << 16);
      u.y = (uint32_t)f2bf(m[2]) | ((uint32_t)f2bf(m[3]) << 16);
      u.z = (uint32_t)f2bf(m[4]) | ((uint32_t)f2bf(m[5]) << 16);
      u.w = (uint32_t)f2bf(m[6]) | ((uint32_t)f2bf(m[7]) << 16);
      *reinterpret_cast<uint4*>(pout + o) = u;
    }
  }
}

// Direct global -> LDS staging of one BF16 chunk for k_conv3x3_rows2: buffer
// loads with the LDS bit write 64 consecutive 16-byte LDS slots per wave
// instruction, lane l the slot 64 j + l of group j, so each lane loads the
// vector that belongs in its slot under the rotated layout of vslot<true>
// (slot 4 p + s of row p holds vector (s - (p >> 1)) & 3).  Wave w issues
// groups w, w + NWAVE, ...; the halo groups come first (padded to whole
// groups; slots past the halo, and pixels outside the image, load zeros
// through an offset outside the buffer range), then the weight groups.  The
// loads complete asynchronously (vmcnt); a wait and a barrier make the
// chunk visible.
template <int LOADER, int NPIX, int BN, int NT>
struct DmaStager {
  using T = uint16_t;
  static constexpr int KC = 32, NV = 4, VEC = 8, PX = 18;
  static constexpr int HALO_G = (NPIX * NV + 63) / 64;
  static constexpr int W_G = 9 * BN * NV / 64;
  static constexpr int NWAVE = NT / 64;
  static constexpr int GPW = (HALO_G + W_G + NWAVE - 1) / NWAVE;
  static constexpr int X_ELEMS = HALO_G * 64 * VEC;  // halo region of a stage (elements)
  static constexpr int STAGE = X_ELEMS + 9 * BN * KC;
  static_assert(9 * BN * NV % 64 == 0, "whole weight groups");
  static_assert(LOADER != LOAD_POOL, "the pooled loader reduces in registers");
  const T* x0b;
  const T* x1b;
  uint32_t bytes0, bytes1;
  uint32_t o0[GPW], o1[GPW];  // halo: offsets in source 0 and 1; weights: offset in o0
  int cu_p, cin_p, chunk_w, wave;

  __device__ __forceinline__ DmaStager(const ConvArgs& a, int b, int wave_, int lane, int y0, int x0, int n0) {
    const int H = a.H, W = a.W;
    wave = wave_;
    cu_p = a.cu_p;
    cin_p = a.cin_p;
    chunk_w = 9 * a.cout_p * KC;
    const int64_t tile0 =
        LOADER == LOAD_UPCAT ? (int64_t)(H >> 1) * (W >> 1) * a.cu_p : (int64_t)H * W * a.cin_p;
    x0b = (const T*)a.x0 + (int64_t)b * tile0;
    bytes0 = (uint32_t)(tile0 * sizeof(T));
    const int64_t tile1 = (int64_t)H * W * (a.cin_p - a.cu_p);
    x1b = LOADER == LOAD_UPCAT ? (const T*)a.x1 + (int64_t)b * tile1 : nullptr;
    bytes1 = (uint32_t)(tile1 * sizeof(T));
#pragma unroll
    for (int i = 0; i < GPW; ++i) {
      const int j = wave + i * NWAVE;
      o0[i] = o1[i] = kOutside;
      if (j < HALO_G) {
        const int sl = 64 * j + lane, p = sl >> 2;
        const uint32_t vb = (uint32_t)((((sl & 3) - (p >> 1)) & 3) * VEC * sizeof(T));
        const int y = y0 + p / PX - 1, x = x0 + p % PX - 1;
        const bool in = p < NPIX && y >= 0 && y < H && x >= 0 && x < W;
        if (LOADER == LOAD_UPCAT) {
          o0[i] = in ? (uint32_t)(((y >> 1) * (W >> 1) + (x >> 1)) * a.cu_p) * sizeof(T) + vb : kOutside;
          o1[i] = in ? (uint32_t)((y * W + x) * (a.cin_p - a.cu_p)) * sizeof(T) + vb : kOutside;
        } else {
          o0[i] = in ? (uint32_t)((y * W + x) * a.cin_p) * sizeof(T) + vb : kOutside;
        }
      } else if (j < HALO_G + W_G) {
        const int sl = 64 * (j - HALO_G) + lane, r = sl >> 2;
        const int v = ((sl & 3) - (r >> 1)) & 3;
        const int tap = r / BN, n = r % BN;
        o0[i] = (uint32_t)(((tap * a.cout_p + n0 + n) * KC + v * VEC) * sizeof(T));
      }
    }
  }

  // Loads of chunk ch into the stage at `stage` (an LDS array).
  __device__ __forceinline__ void issue(const ConvArgs& a, int ch, T* stage) const {
    const int c = ch * KC;
    const bool second = LOADER == LOAD_UPCAT && c >= cu_p;
    const __amdgpu_buffer_rsrc_t rh =
        second ? buffer_rsrc(x1b + (c - cu_p), bytes1 - (uint32_t)((c - cu_p) * sizeof(T)))
               : buffer_rsrc(x0b + c, bytes0 - (uint32_t)(c * sizeof(T)));
    const __amdgpu_buffer_rsrc_t rw = buffer_rsrc((const T*)a.w + (int64_t)ch * chunk_w, (uint32_t)(chunk_w * sizeof(T)));
#pragma unroll
    for (int i = 0; i < GPW; ++i) {
      const int j = wave + i * NWAVE;
      if (j < HALO_G) {
        // a blend rather than a select of the two arrays, which would keep
        // the stager out of registers
        const uint32_t off = o0[i] + ((o1[i] - o0[i]) & (0u - (uint32_t)second));
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rh, (__attribute__((address_space(3))) void*)(stage + j * 64 * VEC),
                                                 16, (int)off, 0, 0, 0);
      } else if (j < HALO_G + W_G) {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rw, (__attribute__((address_space(3))) void*)(stage + X_ELEMS + (j - HALO_G) * 64 * VEC), 16, (int)o0[i],
            0, 0, 0);
      }
    }
  }
};

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima)
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// s_waitcnt vmcnt(N), N < 16: all but the last N vector memory instructions
// of the wave done (the counter retires them in issue order)
template <int N>
__device__ __forceinline__ void wait_vmem_but() {
  static_assert(N >= 0 && N < 16, "four-bit count");
  __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

// Lane byte offsets of the MFMA operand reads of k_conv3x3_rows2 inside a
// stage.  A halo read of fragment row r at horizontal offset dx addresses
// pixel px = xrow + r PX + dx at slot (g + (px >> 1)) & 3 of its 64-byte row;
// with PX = 18 and FM even that slot is (c_dx + r) & 3, so the reads of rows
// r and r + 4 differ by the constant 4 PX 64 bytes and twelve per-lane bases
// xo[dx][r % 4] cover every read.  A weight read of row wr = tap BN + wrow +
// 16 fn has slot (g + (l16 >> 1)) & 3 for every tap and fragment (BN and NW
// multiples of 8), so one base wo covers them.  Writing the addresses this
// way keeps the compiler from holding one address register per read.
struct RowsOffsets {
  uint32_t xo[3][4];
  uint32_t wo;
};

template <int FM>
__device__ __forceinline__ RowsOffsets rows_offsets(int xrow, int wrow, int g, int l16, int wm) {
  constexpr int PX = 18;
  RowsOffsets o;
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) {
    const int c = g + wm * FM + ((l16 + dx) >> 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) o.xo[dx][k] = (uint32_t)((xrow + k * PX + dx) * 64 + ((c + k) & 3) * 16);
  }
  o.wo = (uint32_t)(wrow * 64 + ((g + (l16 >> 1)) & 3) * 16);
  return o;
}

// Operand reads of horizontal offset dx of one chunk: the FM + 2 halo rows
// and the weights of the three taps (dy = 0..2) of that offset, issued in
// the order the MFMAs of rows_mfma consume them (the weights of tap dy
// before the first row that tap adds), so the first MFMA of a chunk waits
// for three reads, not the whole group.
template <int FM, int FN, int BN>
__device__ __forceinline__ void rows_load(uint4 (&xv)[FM + 2], uint4 (&wv)[3][FN], const char* sX, const char* sW,
                                          const RowsOffsets& o, int dx) {
  constexpr int PX = 18;
  auto row = [&](int r) { xv[r] = *reinterpret_cast<const uint4*>(sX + o.xo[dx][r & 3] + (r >> 2) * (4 * PX * 64)); };
  auto wts = [&](int dy) {
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
      wv[dy][fn] = *reinterpret_cast<const uint4*>(sW + o.wo + ((dy * 3 + dx) * BN + fn * 16) * 64);
  };
  wts(0);
#pragma unroll
  for (int r = 0; r < FM; ++r) row(r);
  wts(1);
  row(FM);
  wts(2);
  row(FM + 1);
}

template <int FM, int FN>
__device__ __forceinline__ void rows_mfma(f32x4 (&acc)[FM][FN], const uint4 (&xv)[FM + 2], const uint4 (&wv)[3][FN]) {
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) mma(acc[fm][fn], wv[dy][fn], xv[fm + dy], uint16_t());
}

// Interleave the MFMAs of a group with the operand reads of the next one:
// `reads` groups of (MFMAs, one LDS read).
template <int MFMAS, int READS>
__device__ __forceinline__ void interleave_reads() {
  constexpr int PER = MFMAS / READS;
#pragma unroll
  for (int i = 0; i < READS; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);  // MFMA
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);    // LDS read
  }
  __builtin_amdgcn_sched_group_barrier(0x008, MFMAS - PER * READS, 0);
}

// One chunk of the row-reuse MFMA loop (k_conv3x3_rows's order: dx, then
// dy, then the fragments) from a stage whose halo starts at sX and whose
// weights start at sW (byte pointers into LDS).  The reads of offset dx + 1
// go into a second register set while the MFMAs of offset dx issue.
template <int FM, int FN, int BN>
__device__ __forceinline__ void rows_chunk(f32x4 (&acc)[FM][FN], const char* sX, const char* sW,
                                           const RowsOffsets& o) {
  static_assert(BN % 8 == 0, "weight reads share one slot rotation");
  constexpr int NM = 3 * FM * FN, NR = FM + 2 + 3 * FN;
  uint4 xa[FM + 2], xb[FM + 2];
  uint4 wa[3][FN], wb[3][FN];
  rows_load<FM, FN, BN>(xa, wa, sX, sW, o, 0);
  __builtin_amdgcn_sched_barrier(0);
  rows_load<FM, FN, BN>(xb, wb, sX, sW, o, 1);
  rows_mfma<FM, FN>(acc, xa, wa);
  interleave_reads<NM, NR>();
  __builtin_amdgcn_sched_barrier(0);
  rows_load<FM, FN, BN>(xa, wa, sX, sW, o, 2);
  rows_mfma<FM, FN>(acc, xb, wb);
  interleave_reads<NM, NR>();
  __builtin_amdgcn_sched_barrier(0);
  rows_mfma<FM, FN>(acc, xa, wa);
  __builtin_amdgcn_sched_barrier(0);
}

// Epilogue of the eight-wave large-block forms on the accumulators: lane
// (g, l16) of fragment (fm, fn) holds channels c .. c + 3 of pixel
// (y0 + wm FM + fm, x0 + l16).  Bias, residual, sign gate and ReLU in that
// order, BF16 rounding, 8-byte stores; the 2x2 max-pool takes the vertical
// pair from the lane's own rows and the horizontal one from the
// neighbouring lane.
template <int FN, int NW, int EPI>
__device__ __forceinline__ void rows2_bias(const ConvArgs& a, int n0, int wn, int g, float4 (&bb)[FN]) {
#pragma unroll
  for (int fn = 0; fn < FN; ++fn)
    bb[fn] = (EPI == EPI_RELU || EPI == EPI_RES_RELU)
                 ? *reinterpret_cast<const float4*>(a.bias + n0 + wn * NW + fn * 16 + g * 4)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
}

// The residual of every output piece of the lane (RES_RELU, RES_MASK: the
// conv's own input at the output pixel and channels), read ahead of the
// epilogue so that the loads are in flight together rather than each waited
// for between the stores.
template <int FM, int FN, int NW, int EPI>
__device__ __forceinline__ void rows2_residual(const ConvArgs& a, int b, int y0, int x0, int n0, int wm, int wn,
                                               int g, int l16, uint2 (&r)[FM][FN]) {
  if constexpr (EPI == EPI_RES_RELU || EPI == EPI_RES_MASK) {
    const uint16_t* res = (const uint16_t*)a.x0;
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        const int64_t o =
            (((int64_t)b * a.H + y0 + wm * FM + fm) * a.W + x0 + l16) * a.cout_p + n0 + wn * NW + fn * 16 + g * 4;
        r[fm][fn] = *reinterpret_cast<const uint2*>(res + o);
      }
  }
}

template <int FM, int FN, int NW, int EPI>
__device__ __forceinline__ void rows2_epilogue(const ConvArgs& a, const f32x4 (&acc)[FM][FN], const float4 (&bias)[FN],
                                               const uint2 (&resid)[FM][FN], int b, int y0, int x0, int n0, int wm,
                                               int wn, int g, int l16) {
  using T = uint16_t;
  T* out = (T*)a.y;
  const int x = x0 + l16;
#pragma unroll
  for (int fn = 0; fn < FN; ++fn) {
    const int c = n0 + wn * NW + fn * 16 + g * 4;
    const float4 bb = bias[fn];
#pragma unroll
    for (int fm = 0; fm < FM; fm += 2) {
      float v[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int y = y0 + wm * FM + fm + h;
        const int64_t o = (((int64_t)b * a.H + y) * a.W + x) * a.cout_p + c;
        const f32x4 s = acc[fm + h][fn];
        float* vv = v[h];
        vv[0] = s[0];
        vv[1] = s[1];
        vv[2] = s[2];
        vv[3] = s[3];
        if (EPI == EPI_RELU || EPI == EPI_RES_RELU) {
          vv[0] += bb.x;
          vv[1] += bb.y;
          vv[2] += bb.z;
          vv[3] += bb.w;
        }
        if (EPI == EPI_RES_RELU || EPI == EPI_RES_MASK) {
          const uint2 r = resid[fm + h][fn];
          vv[0] += bf2f(r.x & 0xffff);
          vv[1] += bf2f(r.x >> 16);
          vv[2] += bf2f(r.y & 0xffff);
          vv[3] += bf2f(r.y >> 16);
        }
        if (EPI == EPI_RES_MASK) {
          const uint2 q = *reinterpret_cast<const uint2*>((const T*)a.aux + o);
          if (!(bf2f(q.x & 0xffff) > 0.f)) vv[0] = 0.f;
          if (!(bf2f(q.x >> 16) > 0.f)) vv[1] = 0.f;
          if (!(bf2f(q.y & 0xffff) > 0.f)) vv[2] = 0.f;
          if (!(bf2f(q.y >> 16) > 0.f)) vv[3] = 0.f;
        }
        if (EPI == EPI_RELU || EPI == EPI_RES_RELU) {
#pragma unroll
          for (int j = 0; j < 4; ++j) vv[j] = fmaxf(vv[j], 0.f);
        }
        uint2 u;
        u.x = (uint32_t)f2bf(vv[0]) | ((uint32_t)f2bf(vv[1]) << 16);
        u.y = (uint32_t)f2bf(vv[2]) | ((uint32_t)f2bf(vv[3]) << 16);
        *reinterpret_cast<uint2*>(out + o) = u;
      }
      if (a.pool_out) {
        // rows y and y + 1 (y even: y0, wm FM and fm are even) in this lane,
        // columns x and x ^ 1 in lanes l16 and l16 ^ 1; max commutes with the
        // monotonic BF16 rounding, so this is the pool of the stored output
        float m[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float t = fmaxf(v[0][j], v[1][j]);
          m[j] = fmaxf(t, __shfl_xor(t, 1));
        }
        if ((l16 & 1) == 0) {
          const int py = (y0 + wm * FM + fm) >> 1, px = x >> 1;
          const int64_t o = (((int64_t)b * (a.H >> 1) + py) * (a.W >> 1) + px) * a.cout_p + c;
          uint2 u;
          u.x = (uint32_t)f2bf(m[0]) | ((uint32_t)f2bf(m[1]) << 16);
          u.y = (uint32_t)f2bf(m[2]) | ((uint32_t)f2bf(m[3]) << 16);
          *reinterpret_cast<uint2*>((T*)a.pool_out + o) = u;
        }
      }
    }
  }
}

// BF16 row-reuse form for large blocks: BY rows x 16 pixels x BN channels
// with eight waves, one workgroup per CU.  The compute of a chunk is
// k_conv3x3_rows's (same taps, same order, same MFMAs), so the results are
// bit for bit those of the smaller blocks.  The staging is double-buffered
// in LDS, one barrier per chunk: the plain and upsampling loaders load the
// next chunk straight into the other buffer (DmaStager) while this one is
// computed; the pooling loader, which reduces four raw vectors per halo
// vector, goes through registers and writes the other buffer after this
// chunk's MFMAs are issued.  The epilogue works on the accumulators in
// registers (each lane holds four consecutive channels of one pixel) and
// writes 8-byte pieces of the output, with no LDS staging; the 2x2 max-pool
// takes the vertical pair from the lane's own rows and the horizontal one
// from the neighbouring lane.
template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
__global__ __launch_bounds__(64 * WM * WN, 2) void k_conv3x3_rows2(ConvArgs a) {
  using T = uint16_t;
  using TR = ConvTraits<T>;
  constexpr int KC = TR::KC, VEC = TR::VEC;
  constexpr int NV = KC / VEC;
  constexpr int ROW = KC;
  constexpr int BX = 16, PX = BX + 2, NPIX = (BY + 2) * PX;
  constexpr int FM = BY / WM;
  constexpr int NW = BN / WN, FN = NW / 16;
  constexpr int NT = 64 * WM * WN;
  static_assert(WM * WN == 8 && BY % WM == 0 && NW % 16 == 0 && FM % 2 == 0, "wave layout");
  static_assert(PX == 18 && ROW * (int)sizeof(T) == 64, "rows_offsets assumes 18-pixel halo rows of 64 bytes");
  constexpr bool DMA = LOADER != LOAD_POOL;
  using DS = DmaStager<DMA ? LOADER : LOAD_PLAIN, NPIX, BN, NT>;
  constexpr int XR = DMA ? DS::X_ELEMS : NPIX * ROW;  // halo region of a stage (elements)
  constexpr int STAGE = XR + 9 * BN * ROW;
  static_assert(2 * STAGE * (int)sizeof(T) <= 160 * 1024, "two staging buffers fit the LDS");
  // two arrays, so that the LDS accesses of either stage are known not to
  // touch the other
  __shared__ __attribute__((aligned(16))) T sA[STAGE];
  __shared__ __attribute__((aligned(16))) T sB[STAGE];

  int rest = xcd_remap(blockIdx.x, gridDim.x);
  const int nb = rest % a.n_nblk;
  rest /= a.n_nblk;
  const int sxb = rest % a.tiles_x;
  rest /= a.tiles_x;
  const int syb = rest % a.tiles_y;
  const int b = rest / a.tiles_y;
  if (a.chunk_base + b >= *a.count) return;
  const int y0 = syb * BY, x0 = sxb * BX, n0 = nb * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int g = lane >> 4;
  const int l16 = lane & 15;
  const int xrow = wm * FM * PX + l16;
  const int wrow = wn * NW + l16;
  const RowsOffsets ro = rows_offsets<FM>(xrow, wrow, g, l16, wm);
  const char* cA = reinterpret_cast<const char*>(sA);
  const char* cB = reinterpret_cast<const char*>(sB);
  constexpr int XB = XR * (int)sizeof(T);  // bytes of a stage's halo region

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nchunks = a.cin_p / KC;
  if constexpr (DMA) {
    const DS ds(a, b, wave, lane, y0, x0, n0);
    ds.issue(a, 0, sA);
    wait_vmem();
    __syncthreads();
    // chunk ch is in sA for even ch, in sB for odd ch
    for (int ch = 0; ch < nchunks; ch += 2) {
      if (ch + 1 < nchunks) ds.issue(a, ch + 1, sB);
      if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(1);
      rows_chunk<FM, FN, BN>(acc, cA, cA + XB, ro);
      if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(0);
      wait_vmem();
      __syncthreads();
      if (ch + 1 >= nchunks) break;
      if (ch + 2 < nchunks) ds.issue(a, ch + 2, sA);
      if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(1);
      rows_chunk<FM, FN, BN>(acc, cB, cB + XB, ro);
      if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(0);
      wait_vmem();
      __syncthreads();
    }
  } else {
    constexpr int HALO_V = NPIX * NV, W_V = 9 * BN * NV;
    constexpr int HPT = (HALO_V + NT - 1) / NT, WPT = (W_V + NT - 1) / NT;
    constexpr int LPV = (LOADER == LOAD_POOL) ? 4 : 1;
    uint4 hreg[HPT][LPV];
    uint4 wreg[WPT];
    using ST = RowStager<T, LOADER, HALO_V, W_V, LPV, NV, VEC, KC, ROW, PX, BN, true, NT>;
    const ST st(a, b, tid, y0, x0, n0);
    st.fetch(a, 0, hreg, wreg);
    ST::commit(tid, hreg, wreg, sA, sA + XR);
    st.fetch(a, min(1, nchunks - 1), hreg, wreg, nchunks > 1);
    __syncthreads();
    for (int ch = 0; ch < nchunks; ch += 2) {
      // chunk ch + 1 (fetched during the previous pass) goes into the other
      // stage, which every wave finished reading before the last barrier;
      // then the loads of chunk ch + 2 (empty past the last chunk)
      rows_chunk<FM, FN, BN>(acc, cA, cA + XB, ro);
      ST::commit(tid, hreg, wreg, sB, sB + XR);
      st.fetch(a, min(ch + 2, nchunks - 1), hreg, wreg, ch + 2 < nchunks);
      __syncthreads();
      if (ch + 1 >= nchunks) break;
      rows_chunk<FM, FN, BN>(acc, cB, cB + XB, ro);
      ST::commit(tid, hreg, wreg, sA, sA + XR);
      st.fetch(a, min(ch + 3, nchunks - 1), hreg, wreg, ch + 3 < nchunks);
      __syncthreads();
    }
  }

  float4 bb[FN];
  rows2_bias<FN, NW, EPI>(a, n0, wn, g, bb);
  uint2 resid[FM][FN];
  rows2_residual<FM, FN, NW, EPI>(a, b, y0, x0, n0, wm, wn, g, l16, resid);
  rows2_epilogue<FM, FN, NW, EPI>(a, acc, bb, resid, b, y0, x0, n0, wm, wn, g, l16);
}

// s_waitcnt vmcnt(N) for N < 64 (the count's two high bits sit at 15:14)
template <int N>
__device__ __forceinline__ void wait_vmem_below() {
  static_assert(N >= 0 && N < 64, "six-bit count");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

// Persistent form of k_conv3x3_rows2 for the loaders that stage by DMA and
// an even number of input-channel chunks.  A fixed grid of one workgroup
// per CU walks the launch's blocks (the XCD of workgroup w, w mod 8, takes a
// contiguous range of them, so neighbouring blocks share its L2), and the
// chunk pipeline runs on across blocks: the first chunk of a workgroup's next
// block is loaded into the free stage while the last chunk of the current
// one is computed, and the current block's epilogue runs while that load is
// in flight.  A one-block-per-workgroup launch pays that load and that
// epilogue with the CU otherwise idle.  Per block the MFMAs, their order and
// the epilogue are k_conv3x3_rows2's, so the outputs equal it bit for bit.
template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
__global__ __launch_bounds__(64 * WM * WN, 2) void k_conv3x3_rows2p(ConvArgs a) {
  using T = uint16_t;
  constexpr int KC = 32;
  constexpr int BX = 16, PX = BX + 2, NPIX = (BY + 2) * PX;
  constexpr int FM = BY / WM;
  constexpr int NW = BN / WN, FN = NW / 16;
  constexpr int NT = 64 * WM * WN;
  static_assert(WM * WN == 8 && BY % WM == 0 && NW % 16 == 0 && FM % 2 == 0, "wave layout");
  static_assert(LOADER != LOAD_POOL, "the persistent form stages by DMA");
  using DS = DmaStager<LOADER, NPIX, BN, NT>;
  constexpr int XR = DS::X_ELEMS;
  constexpr int STAGE = XR + 9 * BN * KC;
  static_assert(2 * STAGE * (int)sizeof(T) <= 160 * 1024, "two staging buffers fit the LDS");
  // Epilogue memory instructions issued after the next block's loads: its
  // stores, its residual loads (waited for before use), and with a sign gate
  // the gate's loads as well (then the wait covers everything).
  constexpr bool EPI_LOADS = EPI == EPI_RES_MASK;
  constexpr int EPI_STORES = FM * FN + FM / 2 * FN;  // outputs, and the pooled copy (fewer without one)
  __shared__ __attribute__((aligned(16))) T sA[STAGE];
  __shared__ __attribute__((aligned(16))) T sB[STAGE];

  const int per_tile = a.tiles_y * a.tiles_x * a.n_nblk;
  const int valid = max(0, min(a.batch, *a.count - a.chunk_base));
  const int total = valid * per_tile;
  const int per_xcd = gridDim.x / 8;
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int lo = (int)((int64_t)xcd * total / 8), hi = (int)((int64_t)(xcd + 1) * total / 8);
  int i = lo + slot;
  if (i >= hi) return;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int g = lane >> 4;
  const int l16 = lane & 15;
  const RowsOffsets ro = rows_offsets<FM>(wm * FM * PX + l16, wn * NW + l16, g, l16, wm);
  const char* cA = reinterpret_cast<const char*>(sA);
  const char* cB = reinterpret_cast<const char*>(sB);
  constexpr int XB = XR * (int)sizeof(T);
  const int nchunks = a.cin_p / KC;  // even (checked by the launch)

  auto decode = [&](int j, int& b, int& y0, int& x0, int& n0) {
    int rest = j;
    n0 = (rest % a.n_nblk) * BN;
    rest /= a.n_nblk;
    x0 = (rest % a.tiles_x) * BX;
    rest /= a.tiles_x;
    y0 = (rest % a.tiles_y) * BY;
    b = rest / a.tiles_y;
  };
  int b, y0, x0, n0;
  decode(i, b, y0, x0, n0);
  DS ds(a, b, wave, lane, y0, x0, n0);
  ds.issue(a, 0, sA);
  wait_vmem();
  __syncthreads();
  f32x4 acc[FM][FN];
  while (true) {
#pragma unroll
    for (int r = 0; r < FM; ++r)
#pragma unroll
      for (int f = 0; f < FN; ++f) acc[r][f] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int next = i + per_xcd;
    const bool more = next < hi;
    // the block's bias, read here so that the chunk loop's waits cover it
    // and the epilogue need not wait for the next block's loads
    float4 bb[FN];
    rows2_bias<FN, NW, EPI>(a, n0, wn, g, bb);
    // chunk ch is in sA for even ch, in sB for odd ch
    __builtin_assume(nchunks >= 2);
    for (int ch = 0; ch < nchunks; ch += 2) {
      ds.issue(a, ch + 1, sB);
      if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(1);
      rows_chunk<FM, FN, BN>(acc, cA, cA + XB, ro);
      if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(0);
      wait_vmem();
      __syncthreads();
      if (ch + 2 < nchunks) {
        ds.issue(a, ch + 2, sA);
        if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(1);
        rows_chunk<FM, FN, BN>(acc, cB, cB + XB, ro);
        if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(0);
        wait_vmem();
        __syncthreads();
      }
    }
    // the last chunk (in sB): the next block's first chunk goes into sA
    // meanwhile, then this block's epilogue
    int nb_, ny0, nx0, nn0;
    if (more) {
      decode(next, nb_, ny0, nx0, nn0);
      ds = DS(a, nb_, wave, lane, ny0, nx0, nn0);
      ds.issue(a, 0, sA);
    }
    if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(1);
    rows_chunk<FM, FN, BN>(acc, cB, cB + XB, ro);
    if (LOADER == LOAD_UPCAT) __builtin_amdgcn_s_setprio(0);
    // a residual is read after the MFMAs (holding it through a chunk would
    // spill); waiting for it waits for the loads issued above as well, which
    // have had the chunk's compute to land
    uint2 resid[FM][FN];
    rows2_residual<FM, FN, NW, EPI>(a, b, y0, x0, n0, wm, wn, g, l16, resid);
    rows2_epilogue<FM, FN, NW, EPI>(a, acc, bb, resid, b, y0, x0, n0, wm, wn, g, l16);
    if (!more) break;
    if (EPI_LOADS) {
      wait_vmem();
    } else {
      if (a.pool_out) wait_vmem_below<EPI_STORES>();
      else wait_vmem_below<FM * FN>();
    }
    __syncthreads();
    i = next;
    b = nb_;
    y0 = ny0;
    x0 = nx0;
    n0 = nn0;
  }
}

// Weight-stationary persistent form of the eight-wave row-reuse conv for
// layers with 64 input channels (two 32-channel chunks) and the plain
// loader, any epilogue: in the bench network the level-0 residual convs, the
// level-1 encoder conv_a and the level-0 data-gradient convs, whose short K (two
// chunks) leaves a one-block-per-item kernel paying its first load and its
// epilogue for every 16 x 16 pixel block.  One workgroup per CU keeps the
// 64-channel weight block of its output channels in LDS (both chunks,
// 72 KB, loaded once) and walks pixel blocks; the halo of the next block
// (both chunks, 42 KB) is loaded straight into the other of two LDS stages
// while the current block is computed and written.  The residual is read
// from the halo in LDS (the block's own input).  Per pixel block the MFMAs,
// their order and the epilogue arithmetic are the eight-wave form's, so the
// outputs equal it bit for bit.
template <int EPI>
__global__ __launch_bounds__(512, 2) void k_conv3x3_ws(ConvArgs a) {
  constexpr int PX = 18, NPIX = 18 * 18, WM = 4, WN = 2, FM = 4, NW = 32, FN = 2, BN = 64, NCH = 2;
  constexpr int HG = (NPIX * 4 + 63) / 64;  // 64-slot groups of one halo chunk plane
  constexpr int PLANE = HG * 64 * 16;       // bytes of a halo chunk plane
  constexpr int STAGE = NCH * PLANE;        // bytes of a halo stage (both chunks)
  constexpr int WG = 9 * BN * 4 / 64;       // 64-slot groups of one weight chunk plane
  constexpr int WPLANE = WG * 64 * 16;      // bytes of a weight chunk plane
  static_assert(NCH * WPLANE + 2 * STAGE <= 160 * 1024, "weights and two halo stages fit the LDS");
  // PRECLS: the residual conv with bias and ReLU whose output D only feeds
  // the head's precls; the epilogue computes F = ReLU(W_p D + b_p) from the
  // BF16-rounded D instead of storing D
  constexpr bool PRECLS = EPI == EPI_RES_RELU_PRECLS;
  constexpr bool RES = EPI == EPI_RES_RELU || EPI == EPI_RES_MASK || PRECLS;  // residual = the conv's own input
  constexpr bool BIAS_RELU = EPI == EPI_RELU || EPI == EPI_RES_RELU || PRECLS;
  __shared__ __attribute__((aligned(16))) char sWt[NCH * WPLANE];
  __shared__ __attribute__((aligned(16))) char sH0[STAGE];
  __shared__ __attribute__((aligned(16))) char sH1[STAGE];
  using T = uint16_t;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int g = lane >> 4, l16 = lane & 15;
  // workgroup -> output-channel block and its place among that block's
  // workgroups; the workgroups of one pixel block's channel blocks share an XCD
  const int n_nblk = a.n_nblk;
  const int nb = (blockIdx.x / 8) % n_nblk;
  const int per_nb = gridDim.x / n_nblk;
  const int q = (blockIdx.x / (8 * n_nblk)) * 8 + blockIdx.x % 8;
  const int n0 = nb * BN;
  const int bpt = a.tiles_y * a.tiles_x;
  const int valid = max(0, min(a.batch, *a.count - a.chunk_base));
  const int total = valid * bpt;
  if (q >= total) return;
  const int64_t tile_px = (int64_t)a.H * a.W;
  const uint32_t tile_bytes = (uint32_t)(tile_px * 64 * sizeof(T));

  // the weight block, both chunks, once
  {
    const int chunk_w = 9 * a.cout_p * 32;
    for (int j = wave; j < NCH * WG; j += 8) {
      const int ch = j / WG, jj = j % WG;
      const int sl = 64 * jj + lane, r = sl >> 2;
      const int v = ((sl & 3) - (r >> 1)) & 3;
      const int tap = r / BN, n = r % BN;
      const __amdgpu_buffer_rsrc_t rw =
          buffer_rsrc((const T*)a.w + (int64_t)ch * chunk_w, (uint32_t)(chunk_w * sizeof(T)));
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rw, (__attribute__((address_space(3))) void*)(sWt + ch * WPLANE + jj * 1024), 16,
          (int)(((tap * a.cout_p + n0 + n) * 32 + v * 8) * sizeof(T)), 0, 0, 0);
    }
  }
  // halo of pixel block i into `stage`
  auto halo = [&](int i, char* stage) {
    const int b = i / bpt, rem = i % bpt;
    const int y0 = (rem / a.tiles_x) * 16, x0 = (rem % a.tiles_x) * 16;
    const __amdgpu_buffer_rsrc_t rh = buffer_rsrc((const T*)a.x0 + (int64_t)b * tile_px * 64, tile_bytes);
#pragma unroll
    for (int k = 0; k < (NCH * HG + 7) / 8; ++k) {
      const int j = wave + 8 * k;
      if (j < NCH * HG) {
        const int ch = j / HG, jj = j % HG;
        const int sl = 64 * jj + lane, p = sl >> 2;
        const int v = ((sl & 3) - (p >> 1)) & 3;
        const int y = y0 + p / PX - 1, x = x0 + p % PX - 1;
        const bool in = p < NPIX && y >= 0 && y < a.H && x >= 0 && x < a.W;
        const uint32_t off = in ? (uint32_t)((y * a.W + x) * 64 + ch * 32 + v * 8) * sizeof(T) : kOutside;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rh, (__attribute__((address_space(3))) void*)(stage + ch * PLANE + jj * 1024),
                                                 16, (int)off, 0, 0, 0);
      }
    }
  };

  const int xrow = wm * FM * PX + l16;
  const int wrow = wn * NW + l16;
  const RowsOffsets ro = rows_offsets<FM>(xrow, wrow, g, l16, wm);
  f32x4 acc[FM][FN];
  T* out = (T*)a.y;
  float4 bb[FN];
#pragma unroll
  for (int fn = 0; fn < FN; ++fn)
    bb[fn] = BIAS_RELU ? *reinterpret_cast<const float4*>(a.bias + n0 + wn * NW + fn * 16 + g * 4)
                       : make_float4(0.f, 0.f, 0.f, 0.f);

  // the residual of pixel block i (RES, RES_MASK): input channels c .. c + 3 (cin =
  // cout) of the block's own pixels, halo pixel (row + 1, l16 + 1), chunk
  // c / 32, vector (c % 32) / 8.  Read into registers before the next
  // block's halo loads are issued, so that no LDS read of the epilogue
  // follows a load into LDS it could be taken to overlap.
  uint2 res[FM][FN];
  auto residual = [&](const char* stage) {
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
      const int c = wn * NW + fn * 16 + g * 4;
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        const int px = (wm * FM + fm + 1) * PX + l16 + 1, cv = (c % 32) >> 3;
        res[fm][fn] =
            *reinterpret_cast<const uint2*>(stage + (c / 32) * PLANE + px * 64 + ((cv + (px >> 1)) & 3) * 16 + (c & 4) * 2);
      }
    }
  };

  // PRECLS: this wave's half of the precls weights (channels 32 wn .. 32 wn
  // + 31) and, for lanes g < 2, the bias of outputs 4 g .. 4 g + 3
  uint4 Apre[3];
  float4 bpre = make_float4(0.f, 0.f, 0.f, 0.f);
  if constexpr (PRECLS) {
    precls_weights(a.pre_w, 64, wn, lane, Apre);
    if (g < 2) bpre = *reinterpret_cast<const float4*>(a.pre_b + 4 * g);
  }

  // compute pixel block i from `stage` and write it (PRECLS: the stage is
  // then free and carries the precls halves between the waves)
  auto block = [&](int i, char* stage) {
#pragma unroll
    for (int r = 0; r < FM; ++r)
#pragma unroll
      for (int f = 0; f < FN; ++f) acc[r][f] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) rows_chunk<FM, FN, BN>(acc, stage + ch * PLANE, sWt + ch * WPLANE, ro);
    const int b = i / bpt, rem = i % bpt;
    const int y0 = (rem / a.tiles_x) * 16, x0 = (rem % a.tiles_x) * 16;
    const int x = x0 + l16;
    uint2 dq[FM][FN];  // PRECLS: the BF16 output pieces
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
      const int c = wn * NW + fn * 16 + g * 4;  // channel inside the block
#pragma unroll
      for (int fm = 0; fm < FM; fm += 2) {
        float v[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int row = wm * FM + fm + h;
          const int64_t o = (((int64_t)b * a.H + y0 + row) * a.W + x) * a.cout_p + n0 + c;
          const f32x4 s = acc[fm + h][fn];
          float* vv = v[h];
          vv[0] = s[0];
          vv[1] = s[1];
          vv[2] = s[2];
          vv[3] = s[3];
          if (BIAS_RELU) {
            vv[0] += bb[fn].x;
            vv[1] += bb[fn].y;
            vv[2] += bb[fn].z;
            vv[3] += bb[fn].w;
          }
          if (RES) {
            const uint2 rr = res[fm + h][fn];
            vv[0] += bf2f(rr.x & 0xffff);
            vv[1] += bf2f(rr.x >> 16);
            vv[2] += bf2f(rr.y & 0xffff);
            vv[3] += bf2f(rr.y >> 16);
          }
          if (EPI == EPI_RES_MASK) {
            const uint2 q = *reinterpret_cast<const uint2*>((const T*)a.aux + o);
            if (!(bf2f(q.x & 0xffff) > 0.f)) vv[0] = 0.f;
            if (!(bf2f(q.x >> 16) > 0.f)) vv[1] = 0.f;
            if (!(bf2f(q.y & 0xffff) > 0.f)) vv[2] = 0.f;
            if (!(bf2f(q.y >> 16) > 0.f)) vv[3] = 0.f;
          }
          if (BIAS_RELU) {
#pragma unroll
            for (int j = 0; j < 4; ++j) vv[j] = fmaxf(vv[j], 0.f);
          }
          uint2 u;
          u.x = (uint32_t)f2bf(vv[0]) | ((uint32_t)f2bf(vv[1]) << 16);
          u.y = (uint32_t)f2bf(vv[2]) | ((uint32_t)f2bf(vv[3]) << 16);
          if constexpr (PRECLS) dq[fm + h][fn] = u;
          else *reinterpret_cast<uint2*>(out + o) = u;
        }
        if (!PRECLS && a.pool_out) {
          float m[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float t = fmaxf(v[0][j], v[1][j]);
            m[j] = fmaxf(t, __shfl_xor(t, 1));
          }
          if ((l16 & 1) == 0) {
            const int py = (y0 + wm * FM + fm) >> 1, ppx = x >> 1;
            const int64_t o = (((int64_t)b * (a.H >> 1) + py) * (a.W >> 1) + ppx) * a.cout_p + n0 + c;
            uint2 u;
            u.x = (uint32_t)f2bf(m[0]) | ((uint32_t)f2bf(m[1]) << 16);
            u.y = (uint32_t)f2bf(m[2]) | ((uint32_t)f2bf(m[3]) << 16);
            *reinterpret_cast<uint2*>((T*)a.pool_out + o) = u;
          }
        }
      }
    }
    if constexpr (PRECLS) {
      // a row's two 16-channel pieces are this wave's half of the precls K
      pf32x4 P[FM];
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
        P[fm] = precls_half(Apre, make_uint4(dq[fm][0].x, dq[fm][0].y, dq[fm][1].x, dq[fm][1].y));
      __syncthreads();  // every wave has finished reading the stage
      pf32x4* xch = reinterpret_cast<pf32x4*>(stage);  // [wm][fm][l16][g < 2]
      if (wn == 1 && g < 2) {
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) xch[((wm * FM + fm) * 16 + l16) * 2 + g] = P[fm];
      }
      __syncthreads();
      if (wn == 0 && g < 2) {
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
          const pf32x4 s = P[fm] + xch[((wm * FM + fm) * 16 + l16) * 2 + g];
          const int64_t o = (((int64_t)b * a.H + y0 + wm * FM + fm) * a.W + x) * 8 + 4 * g;
          *reinterpret_cast<float4*>(a.fpre + o) =
              make_float4(fmaxf(s[0] + bpre.x, 0.f), fmaxf(s[1] + bpre.y, 0.f), fmaxf(s[2] + bpre.z, 0.f),
                          fmaxf(s[3] + bpre.w, 0.f));
        }
      }
    }
  };

  halo(q, sH0);
  wait_vmem();
  __syncthreads();
  // The wait after a block is for the next block's halo, issued before the
  // block's output stores (FM FN, and FM FN / 2 for the pooled copy; with
  // PRECLS the FM stores of F, by the waves of the first channel half only):
  // those stay in flight across the barrier.
  constexpr int ST = FM * FN, STP = FM * FN + FM * FN / 2;
  auto wait_halo = [&]() {
    if constexpr (PRECLS) {
      if (wn == 0) wait_vmem_but<FM>();
      else wait_vmem();
    } else {
      if (a.pool_out) wait_vmem_but<STP>();
      else wait_vmem_but<ST>();
    }
  };
  // blocks q, q + per_nb, ... alternate between the stages (two arrays, so
  // that the loads into one are known not to touch the other)
  for (int i = q; i < total; i += 2 * per_nb) {
    if (RES) residual(sH0);
    if (i + per_nb < total) halo(i + per_nb, sH1);
    block(i, sH0);
    wait_halo();
    __syncthreads();
    if (i + per_nb >= total) break;
    if (RES) residual(sH1);
    if (i + 2 * per_nb < total) halo(i + 2 * per_nb, sH0);
    block(i + per_nb, sH1);
    wait_halo();
    __syncthreads();
  }
}

// The weight-stationary form applies to an eight-wave row-reuse launch with
// 64 input channels, a plain loader, a forward epilogue and enough pixel
// blocks to keep one workgroup per CU busy.
constexpr int kWsGrid = 256;
inline bool ws_applies(int loader, int epi, const ConvLayer& L, int H, int W, int batch) {
  const bool res = epi == EPI_RES_RELU || epi == EPI_RES_MASK;
  return loader == LOAD_PLAIN && L.cin_p == 64 && L.cout_p % 64 == 0 && L.cout_p / 64 <= 4 &&
         (!res || L.cout_p == 64) && H % 16 == 0 && W % 16 == 0 && (int64_t)batch * (H / 16) * (W / 16) >= 8 * kWsGrid;
}
// Workgroups of the weight-stationary form: a multiple of 8 per output-channel block, at most one per CU.
inline int ws_grid(int n_nblk) { return 8 * n_nblk * (kWsGrid / (8 * n_nblk)); }

bool conv_precls_fusable(const ConvLayer& L, int H, int W, int batch) {
  return L.cin_p == 64 && L.cout_p == 64 && !L.pool_out && ws_applies(LOAD_PLAIN, EPI_RES_RELU, L, H, W, batch);
}

hipError_t launch_conv_ws_precls(const ConvLayer& L, int H, int W, int batch, const int32_t* count, int chunk_base,
                                 const void* x0, const float* pre_w, const float* pre_b, float* fpre,
                                 hipStream_t st) {
  if (!conv_precls_fusable(L, H, W, batch) || !pre_w || !pre_b || !fpre) return hipErrorInvalidValue;
  ConvArgs a{};
  a.x0 = x0;
  a.w = L.w;
  a.bias = L.b;
  a.H = H;
  a.W = W;
  a.cin_p = L.cin_p;
  a.cu_p = L.cu_p;
  a.cout_p = L.cout_p;
  a.count = count;
  a.chunk_base = chunk_base;
  a.tiles_y = H / 16;
  a.tiles_x = W / 16;
  a.n_nblk = 1;
  a.batch = batch;
  a.pre_w = pre_w;
  a.pre_b = pre_b;
  a.fpre = fpre;
  hipLaunchKernelGGL((k_conv3x3_ws<EPI_RES_RELU_PRECLS>), dim3(ws_grid(1)), dim3(512), 0, st, a);
  return hipGetLastError();
}

// FP8 (E4M3) row-reuse form on v_mfma_scale_f32_32x32x64_f8f6f4 (unit block
// scales): one MFMA is one tap of a 64-channel chunk for 32 output channels
// (A, weights) x 32 pixels (B).  A pixel fragment is two 16-pixel rows; lane
// l holds pixel column l & 15 of row (l >> 4) & 1 and K half l >> 5 (32
// channels, two 16-byte LDS reads).  Per horizontal offset dx a wave reads
// the 2 FM + 1 halo rows its FM fragments need once and feeds them to the
// three vertical taps.  The accumulator of lane l holds channels
// 8 (r / 4) + 4 (l >> 5) + r % 4 (r = 0..15) of pixel l & 31.  Epilogue:
// v = wscale[o] acc + bias[o] (+ residual code * rscale[o]), ReLU, then
// E4M3(min(v * oinv[o], 448)).
typedef __attribute__((ext_vector_type(8))) int i32x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

__device__ __forceinline__ float fp8_decode(uint32_t word, int byte) {
  switch (byte) {
    case 0: return __builtin_amdgcn_cvt_f32_fp8(word, 0);
    case 1: return __builtin_amdgcn_cvt_f32_fp8(word, 1);
    case 2: return __builtin_amdgcn_cvt_f32_fp8(word, 2);
    default: return __builtin_amdgcn_cvt_f32_fp8(word, 3);
  }
}
// four non-negative values -> four E4M3 codes (saturated at 448)
__device__ __forceinline__ uint32_t fp8_encode4(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(fminf(a, kFp8Max), fminf(b, kFp8Max), 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(fminf(c, kFp8Max), fminf(d, kFp8Max), w, true);
  return (uint32_t)w;
}

template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
__global__ __launch_bounds__(256, ((BN >= 128 || LOADER == LOAD_POOL) ? 1 : 2))
void k_conv3x3_fp8(ConvArgs a) {
  using T = uint8_t;
  using TR = ConvTraits<T>;
  constexpr int KC = TR::KC, VEC = TR::VEC, ROW = TR::ROW;
  constexpr int NV = KC / VEC;
  constexpr int BX = 16, PX = BX + 2, NPIX = (BY + 2) * PX;
  constexpr int RPW = BY / WM;       // pixel rows per wave
  constexpr int FM = RPW / 2;        // two-row pixel fragments per wave
  constexpr int NW = BN / WN, FN = NW / 32;
  constexpr int NT = 256;
  static_assert(WM * WN == 4 && BY % WM == 0 && RPW % 2 == 0 && NW % 32 == 0, "wave layout");
  constexpr int MAIN_B = (NPIX + 9 * BN) * ROW;
  constexpr int OROW = BN + 4;
  constexpr int EPI_B = BY * BX * OROW * 4;
  constexpr int SMEM_B = MAIN_B > EPI_B ? MAIN_B : EPI_B;
  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM_B];
  T* sX = reinterpret_cast<T*>(smem);
  T* sW = sX + NPIX * ROW;

  int rest = xcd_remap(blockIdx.x, gridDim.x);
  const int nb = rest % a.n_nblk;
  rest /= a.n_nblk;
  const int sxb = rest % a.tiles_x;
  rest /= a.tiles_x;
  const int syb = rest % a.tiles_y;
  const int b = rest / a.tiles_y;
  if (a.chunk_base + b >= *a.count) return;
  const int y0 = syb * BY, x0 = sxb * BX, n0 = nb * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int kh = (lane >> 5) * 32;       // K half of this lane, in bytes
  const int ro = (lane >> 4) & 1;        // row of this lane inside a pixel fragment
  const int l16 = lane & 15;
  const int xoff = ((wm * RPW + ro) * PX + l16) * ROW + kh;
  const int woff = (wn * NW + (lane & 31)) * ROW + kh;

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  constexpr int HALO_V = NPIX * NV, W_V = 9 * BN * NV;
  constexpr int HPT = (HALO_V + NT - 1) / NT, WPT = (W_V + NT - 1) / NT;
  constexpr int LPV = (LOADER == LOAD_POOL) ? 4 : 1;
  uint4 hreg[HPT][LPV];
  uint4 wreg[WPT];
  const int nchunks = (a.cin_p + KC - 1) / KC;
  using ST = RowStager<T, LOADER, HALO_V, W_V, LPV, NV, VEC, KC, ROW, PX, BN, false, NT>;
  const ST st(a, b, tid, y0, x0, n0);
  st.fetch(a, 0, hreg, wreg);
  ST::commit(tid, hreg, wreg, sX, sW);
  __syncthreads();
  // branch-free loop body, as in the BF16 row-reuse kernel
  for (int ch = 0; ch < nchunks; ++ch) {
    st.fetch(a, min(ch + 1, nchunks - 1), hreg, wreg, ch + 1 < nchunks);
#pragma unroll 1  // one dx at a time: the halo rows of all three would not fit in registers
    for (int dx = 0; dx < 3; ++dx) {
      i32x8 xv[2 * FM + 1];
#pragma unroll
      for (int r = 0; r < 2 * FM + 1; ++r) {
        const uint4 lo = *reinterpret_cast<const uint4*>(&sX[xoff + (r * PX + dx) * ROW]);
        const uint4 hi = *reinterpret_cast<const uint4*>(&sX[xoff + (r * PX + dx) * ROW + 16]);
        xv[r] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int tap = dy * 3 + dx;
        i32x8 wv[FN];
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
          const T* src = &sW[tap * BN * ROW + woff + fn * 32 * ROW];
          const uint4 lo = *reinterpret_cast<const uint4*>(src);
          const uint4 hi = *reinterpret_cast<const uint4*>(src + 16);
          wv[fn] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn)
            acc[fm][fn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(wv[fn], xv[2 * fm + dy], acc[fm][fn],
                                                                          0, 0, 0, 127, 0, 127);
      }
    }
    __syncthreads();
    ST::commit(tid, hreg, wreg, sX, sW);
    __syncthreads();
  }

  // Epilogue: accumulators -> LDS [pixel][channel] (FP32) -> 16-byte rows of codes.
  float* sO = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = (wm * RPW + 2 * fm + ro) * BX + l16;
        const int c = wn * NW + fn * 32 + 8 * q + 4 * (lane >> 5);
        *reinterpret_cast<f32x4*>(&sO[p * OROW + c]) =
            f32x4{acc[fm][fn][4 * q], acc[fm][fn][4 * q + 1], acc[fm][fn][4 * q + 2], acc[fm][fn][4 * q + 3]};
      }
  __syncthreads();
  constexpr int NVO = BN / 16;
  T* out = (T*)a.y;
  const T* res = (const T*)a.x0;
  for (int i = tid; i < BY * BX * NVO; i += NT) {
    const int p = i / NVO, c = (i % NVO) * 16;
    const int y = y0 + p / BX, x = x0 + p % BX, n = n0 + c;
    const int64_t o = (((int64_t)b * a.H + y) * a.W + x) * a.cout_p + n;
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
      const f32x4 t = *reinterpret_cast<const f32x4*>(&sO[p * OROW + c + j]);
      const float4 ws = *reinterpret_cast<const float4*>(a.wscale + n + j);
      const float4 bs = *reinterpret_cast<const float4*>(a.bias + n + j);
      v[j] = fmaf(t[0], ws.x, bs.x);
      v[j + 1] = fmaf(t[1], ws.y, bs.y);
      v[j + 2] = fmaf(t[2], ws.z, bs.z);
      v[j + 3] = fmaf(t[3], ws.w, bs.w);
    }
    if (EPI == EPI_RES_RELU) {
      const uint4 r = *reinterpret_cast<const uint4*>(res + o);
      const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] += fp8_decode(rw[j / 4], j % 4) * a.rscale[n + j];
    }
    uint32_t ow[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float e[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float t = v[4 * j + k];
        e[k] = (t > 0.f ? t : 0.f) * a.oinv[n + 4 * j + k];  // ReLU; +0 for the rest
      }
      ow[j] = fp8_encode4(e[0], e[1], e[2], e[3]);
      if (a.pool_out) *reinterpret_cast<f32x4*>(&sO[p * OROW + c + 4 * j]) = f32x4{e[0], e[1], e[2], e[3]};
    }
    *reinterpret_cast<uint4*>(out + o) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
  }
  if (a.pool_out) {
    // 2x2 max-pool of the scaled outputs; encoding is monotonic, so the pooled
    // code is the max of the four stored codes (the scales carry over).
    __syncthreads();
    T* pout = (T*)a.pool_out;
    const int Hh = a.H >> 1, Wh = a.W >> 1;
    for (int i = tid; i < (BY / 2) * (BX / 2) * NVO; i += NT) {
      const int q = i / NVO, c = (i % NVO) * 16;
      const int py = q / (BX / 2), px = q % (BX / 2);
      const int p00 = (2 * py) * BX + 2 * px;
      uint32_t ow[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f32x4 a0 = *reinterpret_cast<const f32x4*>(&sO[p00 * OROW + c + 4 * j]);
        const f32x4 a1 = *reinterpret_cast<const f32x4*>(&sO[(p00 + 1) * OROW + c + 4 * j]);
        const f32x4 a2 = *reinterpret_cast<const f32x4*>(&sO[(p00 + BX) * OROW + c + 4 * j]);
        const f32x4 a3 = *reinterpret_cast<const f32x4*>(&sO[(p00 + BX + 1) * OROW + c + 4 * j]);
        float m[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) m[k] = fmaxf(fmaxf(a0[k], a1[k]), fmaxf(a2[k], a3[k]));
        ow[j] = fp8_encode4(m[0], m[1], m[2], m[3]);
      }
      const int64_t o = (((int64_t)b * Hh + (y0 >> 1) + py) * Wh + (x0 >> 1) + px) * a.cout_p + n0 + c;
      *reinterpret_cast<uint4*>(pout + o) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
    }
  }
}

template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
static hipError_t launch_conv_fp8_t(const ConvLayer& L, int H, int W, int batch, const int32_t* count,
                                    int chunk_base, const void* x0, const void* x1, void* y, hipStream_t st) {
  ConvArgs a{};
  a.x0 = x0;
  a.x1 = x1;
  a.aux = nullptr;
  a.y = y;
  a.w = L.w;
  a.bias = L.b;
  a.H = H;
  a.W = W;
  a.cin_p = L.cin_p;
  a.cu_p = L.cu_p;
  a.cout_p = L.cout_p;
  a.count = count;
  a.chunk_base = chunk_base;
  a.tiles_y = H / BY;
  a.tiles_x = W / 16;
  a.n_nblk = L.cout_p / BN;
  a.wscale = L.wscale;
  a.rscale = L.rscale;
  a.oinv = L.oinv;
  a.pool_out = L.pool_out;
  if (L.pool_out && EPI != EPI_RES_RELU) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)batch * a.tiles_y * a.tiles_x * a.n_nblk;
  hipLaunchKernelGGL((k_conv3x3_fp8<BY, BN, WM, WN, LOADER, EPI>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
static hipError_t launch_conv_rows_t(const ConvLayer& L, int H, int W, int batch, const int32_t* count,
                                     int chunk_base, const void* x0, const void* x1, const void* aux,
                                     void* y, hipStream_t st) {
  ConvArgs a{};
  a.x0 = x0;
  a.x1 = x1;
  a.aux = aux;
  a.y = y;
  a.w = L.w;
  a.bias = L.b;
  a.H = H;
  a.W = W;
  a.cin_p = L.cin_p;
  a.cu_p = L.cu_p;
  a.cout_p = L.cout_p;
  a.count = count;
  a.chunk_base = chunk_base;
  a.tiles_y = H / BY;
  a.tiles_x = W / 16;
  a.n_nblk = L.cout_p / BN;
  a.pool_out = L.pool_out;
  a.batch = batch;
  if (L.pool_out && EPI != EPI_RES_RELU) return hipErrorInvalidValue;
  if constexpr (BY == 16 && BN == 64 && WM == 4 && WN == 2 && LOADER == LOAD_PLAIN) {
    if (ws_applies(LOADER, EPI, L, H, W, batch)) {
      a.tiles_y = H / 16;
      hipLaunchKernelGGL((k_conv3x3_ws<EPI>), dim3(ws_grid(a.n_nblk)), dim3(512), 0, st, a);
      return hipGetLastError();
    }
  }
  const int64_t blocks = (int64_t)batch * a.tiles_y * a.tiles_x * a.n_nblk;
  hipLaunchKernelGGL((k_conv3x3_rows<BY, BN, WM, WN, LOADER, EPI>), dim3((unsigned)blocks), dim3(64 * WM * WN), 0, st,
                     a);
  return hipGetLastError();
}

template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
static hipError_t launch_conv_rows2_t(const ConvLayer& L, int H, int W, int batch, const int32_t* count,
                                      int chunk_base, const void* x0, const void* x1, const void* aux,
                                      void* y, hipStream_t st) {
  ConvArgs a{};
  a.x0 = x0;
  a.x1 = x1;
  a.aux = aux;
  a.y = y;
  a.w = L.w;
  a.bias = L.b;
  a.H = H;
  a.W = W;
  a.cin_p = L.cin_p;
  a.cu_p = L.cu_p;
  a.cout_p = L.cout_p;
  a.count = count;
  a.chunk_base = chunk_base;
  a.tiles_y = H / BY;
  a.tiles_x = W / 16;
  a.n_nblk = L.cout_p / BN;
  a.pool_out = L.pool_out;
  if (L.pool_out && EPI != EPI_RES_RELU) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)batch * a.tiles_y * a.tiles_x * a.n_nblk;
  hipLaunchKernelGGL((k_conv3x3_rows2<BY, BN, WM, WN, LOADER, EPI>), dim3((unsigned)blocks), dim3(64 * WM * WN), 0,
                     st, a);
  return hipGetLastError();
}

// Workgroups of the persistent large-block form: one per CU.
constexpr int kRows2pGrid = 256;

template <int BY, int BN, int WM, int WN, int LOADER, int EPI>
static hipError_t launch_conv_rows2p_t(const ConvLayer& L, int H, int W, int batch, const int32_t* count,
                                       int chunk_base, const void* x0, const void* x1, const void* aux,
                                       void* y, hipStream_t st) {
  // the pooling loader (whose register staging does not fit beside the
  // large block's accumulators) takes the eight-wave 16-row form, an odd
  // number of input-channel chunks the one-block-per-workgroup large block
  if constexpr (LOADER == LOAD_POOL) {
    return launch_conv_rows_t<16, BN, WM, WN, LOADER, EPI>(L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
  } else {
    if ((L.cin_p / 32) % 2 != 0)
      return launch_conv_rows2_t<BY, BN, WM, WN, LOADER, EPI>(L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
    ConvArgs a{};
    a.x0 = x0;
    a.x1 = x1;
    a.aux = aux;
    a.y = y;
    a.w = L.w;
    a.bias = L.b;
    a.H = H;
    a.W = W;
    a.cin_p = L.cin_p;
    a.cu_p = L.cu_p;
    a.cout_p = L.cout_p;
    a.count = count;
    a.chunk_base = chunk_base;
    a.tiles_y = H / BY;
    a.tiles_x = W / 16;
    a.n_nblk = L.cout_p / BN;
    a.pool_out = L.pool_out;
    a.batch = batch;
    if (L.pool_out && EPI != EPI_RES_RELU) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_conv3x3_rows2p<BY, BN, WM, WN, LOADER, EPI>), dim3(kRows2pGrid), dim3(64 * WM * WN), 0, st,
                       a);
    return hipGetLastError();
  }
}

template <typename T, int BY, int BX, int BN, int WM, int WN, int LOADER, int EPI>
static hipError_t launch_conv_t(const ConvLayer& L, int H, int W, int batch, const int32_t* count,
                                int chunk_base, const void* x0, const void* x1, const void* aux,
                                void* y, hipStream_t st) {
  ConvArgs a{};
  a.x0 = x0;
  a.x1 = x1;
  a.aux = aux;
  a.y = y;
  a.w = L.w;
  a.bias = L.b;
  a.H = H;
  a.W = W;
  a.cin_p = L.cin_p;
  a.cu_p = L.cu_p;
  a.cout_p = L.cout_p;
  a.count = count;
  a.chunk_base = chunk_base;
  a.tiles_y = H / BY;
  a.tiles_x = W / BX;
  a.n_nblk = L.cout_p / BN;
  a.pool_out = nullptr;
  if (L.pool_out) return hipErrorInvalidValue;  // the pooled copy needs a row-reuse configuration
  const int64_t blocks = (int64_t)batch * a.tiles_y * a.tiles_x * a.n_nblk;
  hipLaunchKernelGGL((k_conv3x3<T, BY, BX, BN, WM, WN, LOADER, EPI>), dim3((unsigned)blocks),
                     dim3(256), 0, st, a);
  return hipGetLastError();
}

// Tile configurations: pixel block BY x BX, BN output channels, and the
// 4-wave layout WM x WN (each wave owns (BY BX / WM) x (BN / WN) outputs).
#define OMNISEG_CONV_TILE_CONFIGS(X)  \
  X(CONV_CFG_8x16_32, 8, 16, 32, 4, 1)    \
  X(CONV_CFG_8x16_64, 8, 16, 64, 2, 2)    \
  X(CONV_CFG_16x16_64, 16, 16, 64, 4, 1)  \
  X(CONV_CFG_8x16_128, 8, 16, 128, 2, 2)  \
  X(CONV_CFG_8x8_32, 8, 8, 32, 4, 1)      \
  X(CONV_CFG_8x8_64, 8, 8, 64, 2, 2)
// Row-reuse configurations (BF16): BY rows of 16 pixels, BN channels, waves.
#define OMNISEG_CONV_ROW_CONFIGS(X)             \
  X(CONV_CFG_ROWS_16x16_64, 16, 16, 64, 2, 2)   \
  X(CONV_CFG_ROWS_16x16_128, 16, 16, 128, 2, 2) \
  X(CONV_CFG_ROWS_32x16_32, 32, 16, 32, 4, 1)   \
  X(CONV_CFG_ROWS_16x16_32, 16, 16, 32, 4, 1)
// Eight-wave row-reuse configuration (BF16 only)
#define OMNISEG_CONV_ROW8_CONFIGS(X) X(CONV_CFG_ROWS8_16x16_64, 16, 16, 64, 4, 2)
// Eight-wave large-block row-reuse configuration (BF16 only; k_conv3x3_rows2)
#define OMNISEG_CONV_ROW2_CONFIGS(X) X(CONV_CFG_ROWS2_32x16_64, 32, 16, 64, 4, 2)
// its persistent form (k_conv3x3_rows2p)
#define OMNISEG_CONV_ROW2P_CONFIGS(X) X(CONV_CFG_ROWS2P_32x16_64, 32, 16, 64, 4, 2)

static const int kCfgShape[][5] = {
#define OMNISEG_SHAPE(id, by, bx, bn, wm, wn) {by, bx, bn, wm, wn},
    OMNISEG_CONV_TILE_CONFIGS(OMNISEG_SHAPE) OMNISEG_CONV_ROW_CONFIGS(OMNISEG_SHAPE) OMNISEG_CONV_ROW8_CONFIGS(OMNISEG_SHAPE)
        OMNISEG_CONV_ROW2_CONFIGS(OMNISEG_SHAPE) OMNISEG_CONV_ROW2P_CONFIGS(OMNISEG_SHAPE)
#undef OMNISEG_SHAPE
};
static_assert(sizeof(kCfgShape) / sizeof(kCfgShape[0]) == CONV_CFG_COUNT, "one shape per configuration");

void conv_config_shape(int cfg, int* by, int* bx, int* bn, int* wm, int* wn) {
  *by = kCfgShape[cfg][0];
  *bx = kCfgShape[cfg][1];
  *bn = kCfgShape[cfg][2];
  *wm = kCfgShape[cfg][3];
  *wn = kCfgShape[cfg][4];
}

int conv_config_precisions(int cfg) {
  if (cfg < 0 || cfg >= CONV_CFG_COUNT) return 0;
  if (cfg >= CONV_CFG_ROWS8_16x16_64) return 1 << OMNISEG_BF16;
  return cfg >= CONV_CFG_ROWS_16x16_64 ? (1 << OMNISEG_BF16) | (1 << OMNISEG_FP8)
                                       : (1 << OMNISEG_FP32) | (1 << OMNISEG_BF16);
}

bool conv_config_valid(int cfg, int precision, int H, int W, int cout_p) {
  if (cfg < 0 || cfg >= CONV_CFG_COUNT || precision < 0 || precision > 30) return false;
  if (!(conv_config_precisions(cfg) & (1 << precision))) return false;
  return H % kCfgShape[cfg][0] == 0 && W % kCfgShape[cfg][1] == 0 && cout_p % kCfgShape[cfg][2] == 0;
}

int conv_default_config(int precision, int H, int W, int cout_p) {
  // row-reuse forms first (the training path runs these defaults untuned)
  const int order_bf16[] = {CONV_CFG_ROWS8_16x16_64, CONV_CFG_ROWS_16x16_64, CONV_CFG_ROWS_16x16_32, CONV_CFG_16x16_64,
                            CONV_CFG_8x16_64, CONV_CFG_8x16_32, CONV_CFG_8x8_64, CONV_CFG_8x8_32};
  const int order_f32[] = {CONV_CFG_8x16_64, CONV_CFG_8x16_32, CONV_CFG_8x8_64, CONV_CFG_8x8_32};
  const int order_fp8[] = {CONV_CFG_ROWS_16x16_64, CONV_CFG_ROWS_16x16_32};
  if (precision == OMNISEG_FP8) {
    for (int c : order_fp8)
      if (conv_config_valid(c, precision, H, W, cout_p)) return c;
  } else if (precision == OMNISEG_BF16) {
    for (int c : order_bf16)
      if (conv_config_valid(c, precision, H, W, cout_p)) return c;
  } else {
    for (int c : order_f32)
      if (conv_config_valid(c, precision, H, W, cout_p)) return c;
  }
  return -1;
}

template <typename T, int LOADER, int EPI>
static hipError_t launch_conv_cfg(int cfg, const ConvLayer& L, int H, int W, int batch, const int32_t* count,
                                  int chunk_base, const void* x0, const void* x1, const void* aux, void* y,
                                  hipStream_t st) {
  switch (cfg) {
#define OMNISEG_CASE(id, by, bx, bn, wm, wn) \
  case id:                                   \
    return launch_conv_t<T, by, bx, bn, wm, wn, LOADER, EPI>(L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
    OMNISEG_CONV_TILE_CONFIGS(OMNISEG_CASE)
#undef OMNISEG_CASE
    default:
      break;
  }
  if constexpr (std::is_same<T, uint16_t>::value) {
    switch (cfg) {
#define OMNISEG_CASE(id, by, bx, bn, wm, wn) \
  case id:                                   \
    return launch_conv_rows_t<by, bn, wm, wn, LOADER, EPI>(L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
      OMNISEG_CONV_ROW_CONFIGS(OMNISEG_CASE)
      OMNISEG_CONV_ROW8_CONFIGS(OMNISEG_CASE)
#undef OMNISEG_CASE
#define OMNISEG_CASE(id, by, bx, bn, wm, wn) \
  case id:                                   \
    return launch_conv_rows2_t<by, bn, wm, wn, LOADER, EPI>(L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
      OMNISEG_CONV_ROW2_CONFIGS(OMNISEG_CASE)
#undef OMNISEG_CASE
#define OMNISEG_CASE(id, by, bx, bn, wm, wn) \
  case id:                                   \
    return launch_conv_rows2p_t<by, bn, wm, wn, LOADER, EPI>(L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
      OMNISEG_CONV_ROW2P_CONFIGS(OMNISEG_CASE)
#undef OMNISEG_CASE
      default:
        break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_conv_mode(int cfg, int loader, int epi, const ConvLayer& L, int H, int W, int batch,
                                   const int32_t* count, int chunk_base, const void* x0, const void* x1,
                                   const void* aux, void* y, hipStream_t st) {
#define OMNISEG_CONV_CASE(LD, EP)  \
  if (loader == LD && epi == EP) \
    return launch_conv_cfg<T, LD, EP>(cfg, L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
  OMNISEG_CONV_CASE(LOAD_PLAIN, EPI_RES_RELU)
  OMNISEG_CONV_CASE(LOAD_POOL, EPI_RELU)
  OMNISEG_CONV_CASE(LOAD_UPCAT, EPI_RELU)
  OMNISEG_CONV_CASE(LOAD_PLAIN, EPI_RELU)
  OMNISEG_CONV_CASE(LOAD_PLAIN, EPI_NONE)
  OMNISEG_CONV_CASE(LOAD_PLAIN, EPI_RES_MASK)
#undef OMNISEG_CONV_CASE
  return hipErrorInvalidValue;
}

template <int LOADER, int EPI>
static hipError_t launch_fp8_cfg(int cfg, const ConvLayer& L, int H, int W, int batch, const int32_t* count,
                                 int chunk_base, const void* x0, const void* x1, void* y, hipStream_t st) {
  switch (cfg) {
#define OMNISEG_CASE(id, by, bx, bn, wm, wn) \
  case id:                                   \
    return launch_conv_fp8_t<by, bn, wm, wn, LOADER, EPI>(L, H, W, batch, count, chunk_base, x0, x1, y, st);
    OMNISEG_CONV_ROW_CONFIGS(OMNISEG_CASE)
#undef OMNISEG_CASE
    default:
      return hipErrorInvalidValue;
  }
}

static hipError_t launch_fp8_mode(int cfg, int loader, int epi, const ConvLayer& L, int H, int W, int batch,
                                  const int32_t* count, int chunk_base, const void* x0, const void* x1, void* y,
                                  hipStream_t st) {
  if (!L.wscale || !L.oinv || (epi == EPI_RES_RELU && !L.rscale)) return hipErrorInvalidValue;
#define OMNISEG_FP8_CASE(LD, EP) \
  if (loader == LD && epi == EP) return launch_fp8_cfg<LD, EP>(cfg, L, H, W, batch, count, chunk_base, x0, x1, y, st);
  OMNISEG_FP8_CASE(LOAD_PLAIN, EPI_RES_RELU)
  OMNISEG_FP8_CASE(LOAD_POOL, EPI_RELU)
  OMNISEG_FP8_CASE(LOAD_UPCAT, EPI_RELU)
  OMNISEG_FP8_CASE(LOAD_PLAIN, EPI_RELU)
#undef OMNISEG_FP8_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_conv3x3(int precision, int loader, int epi, const ConvLayer& L, int H, int W,
                          int batch, const int32_t* count, int chunk_base, const void* x0,
                          const void* x1, void* y, hipStream_t st, const void* aux, int cfg) {
  if (cfg < 0 || !conv_config_valid(cfg, precision, H, W, L.cout_p)) {
    cfg = conv_default_config(precision, H, W, L.cout_p);
    // BF16 launches that come with no configuration (the training backward,
    // the stand-alone call with -1) take the persistent large-block form
    // where it fits, except for 64 input channels, where the eight-wave
    // configuration's weight-stationary form is faster
    if (precision == OMNISEG_BF16 && loader != LOAD_POOL && L.cin_p != 64 &&
        conv_config_valid(CONV_CFG_ROWS2P_32x16_64, precision, H, W, L.cout_p))
      cfg = CONV_CFG_ROWS2P_32x16_64;
  }
  if (cfg < 0) return hipErrorInvalidValue;
  if (precision == OMNISEG_FP8) return launch_fp8_mode(cfg, loader, epi, L, H, W, batch, count, chunk_base, x0, x1, y, st);
  if (precision == OMNISEG_BF16)
    return launch_conv_mode<uint16_t>(cfg, loader, epi, L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
  return launch_conv_mode<float>(cfg, loader, epi, L, H, W, batch, count, chunk_base, x0, x1, aux, y, st);
}

// ---------------------------------------------------------------------------
// First conv, 3 -> C_0, from the slide (40x) or the box-sum pyramid.  One
// workgroup per 16-pixel-wide column of BH rows of one tile; the
// (BH + 2) x 18 x 3 input patch is staged in FP32 in LDS, with the pad
// colour outside the slide and zeros outside the tile, and the input is
// normalised to [0, 1] (value / (255 * 4^k)).  FP32 sums of exact products
// for every precision (FP32 MFMA for the FP32 path, exact BF16 splits on BF16
// MFMA for BF16 and FP8); the output is stored in the backbone's storage type.
// ---------------------------------------------------------------------------

constexpr int kFirstMaxC0 = 128;

// Four consecutive channels of one pixel.
__device__ __forceinline__ void store4(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(uint16_t* p, const float* v) {
  *reinterpret_cast<uint2*>(p) = make_uint2((uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                                            (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16));
}
__device__ __forceinline__ void store4(uint8_t* p, const float* v) {
  *reinterpret_cast<uint32_t*>(p) = fp8_encode4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store_vec(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
// FP8: 16 channels per vector, each multiplied by its inverse channel scale
// before encoding (values are ReLU outputs, >= 0).
__device__ __forceinline__ void store_vec(uint8_t* p, const float* v) {
  *reinterpret_cast<uint4*>(p) = make_uint4(fp8_encode4(v[0], v[1], v[2], v[3]), fp8_encode4(v[4], v[5], v[6], v[7]),
                                            fp8_encode4(v[8], v[9], v[10], v[11]),
                                            fp8_encode4(v[12], v[13], v[14], v[15]));
}
__device__ __forceinline__ void store_vec(uint16_t* p, const float* v) {
  uint4 u;
  u.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
  u.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
  u.z = (uint32_t)f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16);
  u.w = (uint32_t)f2bf(v[6]) | ((uint32_t)f2bf(v[7]) << 16);
  *reinterpret_cast<uint4*>(p) = u;
}

// The (BH + 2) x 18 input patch of column block (sy, sx) of tile t at scale k,
// channel-major in sp[c][py][px]: each raw value (a colour, or a box sum of
// the pyramid) times `mul`, the pad colour beyond the slide and zeros beyond
// the tile.
template <int BH>
__device__ __forceinline__ void first_stage_patch(const FirstConvArgs& a, const int4 t, int k, int sy, int sx,
                                                  float mul, float (&sp)[3][BH + 2][19]) {
  const SlideDev& sd = a.slides[t.x];
  const int oy = t.z * a.scale_s[t.y], ox = t.w * a.scale_s[t.y];  // tile origin at scale k
  for (int i = threadIdx.x; i < (BH + 2) * 18; i += 256) {
    const int py = i / 18, px = i % 18;
    const int ty = sy * BH + py - 1, tx = sx * 16 + px - 1;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
    if (ty >= 0 && ty < a.T && tx >= 0 && tx < a.T) {
      const int Y = oy + ty, X = ox + tx;
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
        v0 = r * mul;
        v1 = g * mul;
        v2 = bb * mul;
      } else {
        const ushort4 s4 = reinterpret_cast<const ushort4*>(sd.pyr[t.y])[(int64_t)Y * sd.pyr_ex[t.y] + X];
        v0 = s4.x * mul;
        v1 = s4.y * mul;
        v2 = s4.z * mul;
      }
    }
    sp[0][py][px] = v0;
    sp[1][py][px] = v1;
    sp[2][py][px] = v2;
  }
}

// BH output rows (64 when the tile allows, else 16) of a 16-pixel-wide column
// per workgroup; a wave owns BH / 4 rows and loads its weight fragments once.
template <typename T, int BH>
__global__ __launch_bounds__(256) void k_first_conv(FirstConvArgs a) {
  constexpr int RPW = BH / 4;                           // output rows per wave
  constexpr int OPAD = 16 / (int)sizeof(T);             // one 16-byte slot per staged pixel row
  constexpr int OPITCH = kFirstMaxC0 + OPAD;            // staged values per pixel (at most)
  __shared__ float sIn[3][BH + 2][19];
  __shared__ float sBias[kFirstMaxC0], sOinv[kFirstMaxC0];  // zero / one beyond c0
  __shared__ __attribute__((aligned(16))) T sOut[4][16 * OPITCH];
  const int nbx = a.T / 16, nby = a.T / BH;
  int rest = blockIdx.x;
  const int sx = rest % nbx;
  rest /= nbx;
  const int sy = rest % nby;
  const int b = rest / nby;
  if (a.chunk_base + b >= *a.count) return;
  const int4 t = reinterpret_cast<const int4*>(a.list)[a.chunk_base + b];
  const int k = a.scale_k[t.y];
  const float scale = 1.0f / (255.0f * (float)(1 << (2 * k)));
  first_stage_patch<BH>(a, t, k, sy, sx, scale, sIn);
  if (threadIdx.x < kFirstMaxC0) {
    const int o = threadIdx.x;
    sBias[o] = o < a.c0 ? a.b[o] : 0.f;
    sOinv[o] = (std::is_same<T, uint8_t>::value && o < a.c0) ? a.oinv[o] : 1.f;
  }
  __syncthreads();
  // The 3 -> C_0 conv as a GEMM on FP32 MFMA (v_mfma_f32_16x16x4f32): A =
  // weights [16 output channels x 4 K], B = the im2col rows of 16 pixels
  // [4 K x 16 pixels], K = 27 taps x channels padded to 28 (seven steps).
  // Lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; the accumulator
  // holds channels 4 (l / 16) .. + 3 of pixel l % 16.
  constexpr int KS = 7, MAXM = 8;  // C_0 <= 128: at most eight 16-channel fragments
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int nm = a.c0_p / 16;
  float wa[MAXM][KS];
  // Branch-free (an out-of-range entry loads element 0 and is replaced by
  // zero), so the 56 loads are in flight together instead of one by one.
#pragma unroll
  for (int m = 0; m < MAXM; ++m)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int o = m * 16 + l16, k = 4 * ks + g;
      const bool ok = m < nm && o < a.c0 && k < 27;
      const float v = a.w[ok ? o * 27 + k : 0];
      wa[m][ks] = ok ? v : 0.f;
    }
  // im2col offsets inside sIn of this lane's K entries (k = c*9 + dy*3 + dx)
  int koff[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = 4 * ks + g;
    const int c = k / 9, dy = (k % 9) / 3, dx = k % 3;
    koff[ks] = k < 27 ? (c * (BH + 2) + dy) * 19 + dx : -1;
  }
  const float* sflat = &sIn[0][0][0];
  // A wave's 16 output pixels of one row are contiguous in the output (16 x
  // c0_p values): they are staged in LDS and written as 16-byte vectors.
  T* srow = sOut[wave];
  const int pitch = a.c0_p + OPAD;  // staged row pitch, padded against bank conflicts
  const int vpp = a.c0_p * (int)sizeof(T) / 16;  // 16-byte vectors per pixel
  constexpr int VE = 16 / (int)sizeof(T);
  for (int r = 0; r < RPW; ++r) {
    const int py = wave * RPW + r;
    float xb[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) xb[ks] = koff[ks] >= 0 ? sflat[koff[ks] + py * 19 + l16] : 0.f;
#pragma unroll
    for (int m = 0; m < MAXM; ++m) {
      if (m >= nm) break;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[m][ks], xb[ks], acc, 0, 0, 0);
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // channels at or beyond c0 have zero weights and bias: t = 0 there
        const int o = m * 16 + 4 * g + q;
        float t = acc[q] + sBias[o];
        t = t > 0.f ? t : 0.f;
        if (std::is_same<T, uint8_t>::value) t *= sOinv[o];
        v[q] = t;
      }
      store4(srow + l16 * pitch + m * 16 + 4 * g, v);
    }
    // the wave reads back what its own lanes wrote (LDS keeps a wave's
    // accesses in order; the fence keeps the compiler from moving them)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int y = sy * BH + py;
    T* out = (T*)a.y + (((int64_t)b * a.T + y) * a.T + sx * 16) * a.c0_p;
    for (int v = lane; v < 16 * vpp; v += 64) {
      const int px = v / vpp, j = v % vpp;
      *reinterpret_cast<uint4*>(out + v * VE) = *reinterpret_cast<const uint4*>(srow + px * pitch + j * VE);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// BF16 and FP8 storage: the same conv on BF16 MFMA (v_mfma_f32_16x16x32_bf16)
// with every product exact, so that the sums are FP32 sums of exact products
// as on the FP32 MFMA above.  The patch holds the raw integers (colours, or
// box sums below 2^14 since k <= 3), each split into hi = v & ~255 and
// lo = v & 255, both exact in BF16; each FP32 weight is split into three BF16
// terms, w = hi + mid + lo exactly (hi = bf16(w), mid = bf16(w - hi), and the
// remainder has at most eight significant bits).  The normalisation
// 1 / (255 * 4^k) multiplies the sum; at 40x the inputs' hi parts are zero and
// their three MFMAs are skipped.  K slot 8 g + j of lane (g, l16) is tap
// t = 8 g + j (c * 9 + dy * 3 + dx; slots from 27 on are zero) of pixel l16,
// and a lane's result holds channels 16 m + 4 g .. + 3 of pixel l16 as above.
template <typename T, int BH, int NMX>
__global__ __launch_bounds__(256) void k_first_conv_split(FirstConvArgs a) {
  constexpr int RPW = BH / 4;
  constexpr int OPAD = 16 / (int)sizeof(T);
  constexpr int OPITCH = NMX * 16 + OPAD;
  __shared__ float sIn[3][BH + 2][19];
  __shared__ float sBias[NMX * 16], sOinv[NMX * 16];  // zero / one beyond c0
  __shared__ __attribute__((aligned(16))) T sOut[4][16 * OPITCH];
  const int nbx = a.T / 16, nby = a.T / BH;
  int rest = blockIdx.x;
  const int sx = rest % nbx;
  rest /= nbx;
  const int sy = rest % nby;
  const int b = rest / nby;
  if (a.chunk_base + b >= *a.count) return;
  const int4 t = reinterpret_cast<const int4*>(a.list)[a.chunk_base + b];
  const int k = a.scale_k[t.y];
  const float scale = 1.0f / (255.0f * (float)(1 << (2 * k)));
  first_stage_patch<BH>(a, t, k, sy, sx, 1.0f, sIn);
  if (threadIdx.x < NMX * 16) {
    const int o = threadIdx.x;
    sBias[o] = o < a.c0 ? a.b[o] : 0.f;
    sOinv[o] = (std::is_same<T, uint8_t>::value && o < a.c0) ? a.oinv[o] : 1.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int nm = a.c0_p / 16;
  // A operands: wa[m][q] = term q (0 hi, 1 mid, 2 lo) of the weights of
  // output channel 16 m + l16 at taps 8 g .. 8 g + 7.  Branch-free loads (an
  // out-of-range entry loads element 0 and is replaced by zero).
  uint4 wa[NMX][3];
#pragma unroll
  for (int m = 0; m < NMX; ++m) {
    uint32_t tq[3][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int o = m * 16 + l16, tap = 8 * g + j;
      const bool ok = m < nm && o < a.c0 && tap < 27;
      const float v = a.w[ok ? o * 27 + tap : 0];
      const float w = ok ? v : 0.f;
      const uint32_t hi = precls_bf16_rne(w);
      const float r1 = w - __uint_as_float(hi << 16);
      const uint32_t mid = precls_bf16_rne(r1);
      tq[0][j] = hi;
      tq[1][j] = mid;
      tq[2][j] = precls_bf16_rne(r1 - __uint_as_float(mid << 16));
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
      wa[m][q] = make_uint4(tq[q][0] | (tq[q][1] << 16), tq[q][2] | (tq[q][3] << 16), tq[q][4] | (tq[q][5] << 16),
                            tq[q][6] | (tq[q][7] << 16));
  }
  // patch offsets of this lane's taps
  int koff[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int tap = 8 * g + j;
    const int c = tap / 9, dy = (tap % 9) / 3, dx = tap % 3;
    koff[j] = tap < 27 ? (c * (BH + 2) + dy) * 19 + dx : -1;
  }
  const float* sflat = &sIn[0][0][0];
  T* srow = sOut[wave];
  const int pitch = a.c0_p + OPAD;
  const int vpp = a.c0_p * (int)sizeof(T) / 16;
  constexpr int VE = 16 / (int)sizeof(T);
  const bool two = k > 0;  // uniform across the block
  for (int r = 0; r < RPW; ++r) {
    const int py = wave * RPW + r;
    uint32_t lo[8], hi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t iv = koff[j] >= 0 ? (uint32_t)sflat[koff[j] + py * 19 + l16] : 0u;
      // integers below 2^14: each part has at most eight significant bits,
      // so its FP32 pattern's upper half is its BF16 value
      lo[j] = __float_as_uint((float)(iv & 255u)) >> 16;
      hi[j] = __float_as_uint((float)(iv & ~255u)) >> 16;
    }
    const uint4 blo = make_uint4(lo[0] | (lo[1] << 16), lo[2] | (lo[3] << 16), lo[4] | (lo[5] << 16),
                                 lo[6] | (lo[7] << 16));
    const uint4 bhi = make_uint4(hi[0] | (hi[1] << 16), hi[2] | (hi[3] << 16), hi[4] | (hi[5] << 16),
                                 hi[6] | (hi[7] << 16));
#pragma unroll
    for (int m = 0; m < NMX; ++m) {
      if (m >= nm) break;
      pf32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 2; q >= 0; --q)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(pbf16x8, wa[m][q]),
                                                      __builtin_bit_cast(pbf16x8, blo), acc, 0, 0, 0);
      if (two) {
#pragma unroll
        for (int q = 2; q >= 0; --q)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(pbf16x8, wa[m][q]),
                                                        __builtin_bit_cast(pbf16x8, bhi), acc, 0, 0, 0);
      }
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = m * 16 + 4 * g + q;
        float u = acc[q] * scale + sBias[o];
        u = u > 0.f ? u : 0.f;
        if (std::is_same<T, uint8_t>::value) u *= sOinv[o];
        v[q] = u;
      }
      store4(srow + l16 * pitch + m * 16 + 4 * g, v);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int y = sy * BH + py;
    T* out = (T*)a.y + (((int64_t)b * a.T + y) * a.T + sx * 16) * a.c0_p;
    for (int v = lane; v < 16 * vpp; v += 64) {
      const int px = v / vpp, j = v % vpp;
      *reinterpret_cast<uint4*>(out + v * VE) = *reinterpret_cast<const uint4*>(srow + px * pitch + j * VE);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

hipError_t launch_first_conv(int precision, const FirstConvArgs& a, hipStream_t st) {
  if (a.c0 > kFirstMaxC0 || a.T % 16 || a.c0_p % 16) return hipErrorInvalidValue;
  const bool tall = a.T % 64 == 0;
  const int64_t blocks = (int64_t)a.batch * (a.T / 16) * (a.T / (tall ? 64 : 16));
  const dim3 grid((unsigned)blocks);
  const bool narrow = a.c0_p <= 64;  // at most four 16-channel fragments
  if (precision == OMNISEG_FP8) {
    if (!a.oinv) return hipErrorInvalidValue;
    if (tall && narrow) hipLaunchKernelGGL((k_first_conv_split<uint8_t, 64, 4>), grid, dim3(256), 0, st, a);
    else if (tall) hipLaunchKernelGGL((k_first_conv_split<uint8_t, 64, 8>), grid, dim3(256), 0, st, a);
    else if (narrow) hipLaunchKernelGGL((k_first_conv_split<uint8_t, 16, 4>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_first_conv_split<uint8_t, 16, 8>), grid, dim3(256), 0, st, a);
  } else if (precision == OMNISEG_BF16) {
    if (tall && narrow) hipLaunchKernelGGL((k_first_conv_split<uint16_t, 64, 4>), grid, dim3(256), 0, st, a);
    else if (tall) hipLaunchKernelGGL((k_first_conv_split<uint16_t, 64, 8>), grid, dim3(256), 0, st, a);
    else if (narrow) hipLaunchKernelGGL((k_first_conv_split<uint16_t, 16, 4>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_first_conv_split<uint16_t, 16, 8>), grid, dim3(256), 0, st, a);
  } else {
    if (tall) hipLaunchKernelGGL((k_first_conv<float, 64>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_first_conv<float, 16>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace omniseg

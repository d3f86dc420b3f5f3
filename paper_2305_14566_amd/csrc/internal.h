// Internal declarations of the omniseg HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "../../include/omniseg.h"

namespace omniseg {

// Channel counts are padded to a multiple of this in every activation tensor
// and packed weight; padded channels hold zeros.
constexpr int kChanAlign = 32;

inline int pad_ch(int c) { return (c + kChanAlign - 1) / kChanAlign * kChanAlign; }
inline int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// ---- per-slide / per-scale geometry --------------------------------------

struct ScaleGeom {
  int k;        // log2 downsampling factor
  int Hk, Wk;   // ceil(H / 2^k), ceil(W / 2^k)
  int ny, nx;   // tile grid
  int Ey, Ex;   // grid extent: (n - 1) * s + T
};

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int grid_count(int n, int T, int s) { return n <= T ? 1 : ceil_div(n - T, s) + 1; }

inline ScaleGeom make_geom(int H, int W, int k, int T, int s) {
  ScaleGeom g;
  g.k = k;
  g.Hk = ceil_div(H, 1 << k);
  g.Wk = ceil_div(W, 1 << k);
  g.ny = grid_count(g.Hk, T, s);
  g.nx = grid_count(g.Wk, T, s);
  g.Ey = (g.ny - 1) * s + T;
  g.Ex = (g.nx - 1) * s + T;
  return g;
}

// ---- tile groups: one (slide, scale slot) grid each ------------------------

constexpr int kMaxGroups = OMNISEG_MAX_SLIDES * OMNISEG_MAX_SCALES;

struct TileGroups {
  int n;                       // number of groups
  int base[kMaxGroups + 1];    // first canonical tile index of each group
  short ny[kMaxGroups], nx[kMaxGroups];
  char slide[kMaxGroups], slot[kMaxGroups], k[kMaxGroups];
};

// Geometry of one slide as the kernels need it.
struct SlideDev {
  const uint8_t* rgb;
  int64_t pitch;
  int H, W;
  const int32_t* pad;                       // int32[4] pad colour
  const uint16_t* pyr[OMNISEG_MAX_SCALES];  // box sums per slot (null for 40x)
  int pyr_ex[OMNISEG_MAX_SCALES];           // row length of each pyramid level
  const uint8_t* fg;                        // tissue map (or null)
  int Hc, Wc;                               // tissue map size
};

// ---- kernel launchers (each returns a hipError_t) ---------------------------

hipError_t launch_pad_colour(const uint8_t* rgb, int64_t pitch, int32_t* pad, hipStream_t st);
hipError_t launch_pyramid(const uint8_t* rgb, int64_t pitch, int H, int W, const int32_t* pad,
                          int kmax, uint16_t* const* lvl /*[4], index k*/, const int* Ey,
                          const int* Ex, hipStream_t st);
hipError_t launch_tissue(const uint8_t* rgb, int64_t pitch, int H, int W, const int32_t* pad,
                         const uint16_t* sums_kc, int ex_kc, int kc, int Hc, int Wc, int thr,
                         uint8_t* fg, hipStream_t st);
hipError_t launch_tile_flags(const TileGroups& g, const SlideDev* slides_dev, int T, int s,
                             int kc, int fg_filter, int32_t* flags, hipStream_t st);
hipError_t launch_compact(int32_t* flags_to_index, int total, const TileGroups& g,
                          int32_t* list, int32_t* count, hipStream_t st);

struct ConvLayer {
  int cin_p;      // padded input channels (concat: cu_p + ce_p)
  int cu_p;       // UPCAT: padded channels of the upsampled source
  int cout_p;     // padded output channels
  const void* w;  // packed weights [cin_p / KC][9][cout_p][KC]
  const float* b; // bias [cout_p]
};

enum Loader { LOAD_PLAIN = 0, LOAD_POOL = 1, LOAD_UPCAT = 2 };
enum Epilogue { EPI_RELU = 0, EPI_RES_RELU = 1 };

// 3x3 conv on a batch of tiles (NHWC, padded channels), output H x W per tile.
hipError_t launch_conv3x3(int precision, int loader, int epi, const ConvLayer& L, int H, int W,
                          int batch, const int32_t* count, int chunk_base, const void* x0,
                          const void* x1, void* y, hipStream_t st);

// First conv (3 -> C_0) straight from the slide / pyramid.
struct FirstConvArgs {
  const int32_t* list;  // tile list int32[4] per tile
  const int32_t* count;
  int chunk_base;
  int batch;
  int T, s;
  const float* w;  // [C_0][27] (c, dy, dx order: w[o][c*9 + dy*3 + dx])
  const float* b;  // [C_0]
  int c0, c0_p;
  void* y;  // [batch][T][T][c0_p]
  const SlideDev* slides;  // device array, one per slide
  int scale_k[OMNISEG_MAX_SCALES];
};
hipError_t launch_first_conv(int precision, const FirstConvArgs& a, hipStream_t st);

hipError_t launch_gap(int precision, const void* e, int batch, int hw, int c_p, int c,
                      const int32_t* count, int chunk_base, float* g, hipStream_t st);

struct SlotTable {
  int n_slots[OMNISEG_MAX_SCALES];
  int cls[OMNISEG_MAX_SCALES][OMNISEG_MAX_CLASSES];
};

hipError_t launch_controller(const float* g, int batch, int G, const float* wc, const float* bc,
                             int P, int n_classes, int n_scales, const SlotTable& slots,
                             int max_slots, const int32_t* list, const int32_t* count,
                             int chunk_base, float* theta, hipStream_t st);

hipError_t launch_head(int precision, const void* d0, int batch, int T, int c0, int c0_p,
                       const float* wp, const float* bp, const float* theta, int P, int o,
                       const SlotTable& slots, int max_slots, const int32_t* list,
                       const int32_t* count, int chunk_base, float* tile_logits,
                       hipStream_t st);

struct StitchArgs {
  const float* logits;     // tile logits base
  int64_t tile_stride;     // floats between consecutive tiles
  int64_t slot_off;        // float offset of the slot plane inside a tile
  const int32_t* index;    // grid [ny][nx] of list indices (or -1)
  int ny, nx, T, s, Hk, Wk;
  uint8_t* mask;
  int64_t mask_pitch;
  float* logit;
  int64_t logit_pitch;
  const uint8_t* fg;  // tissue map for mask_and_fg (or null)
  int fg_shift, Hc, Wc;
};
hipError_t launch_stitch(const StitchArgs& a, hipStream_t st);
hipError_t launch_grid_from_list(const int32_t* tile_yx, int n_tiles, int ny, int nx,
                                 int32_t* grid, hipStream_t st);

// Weight packing
struct PackConv {
  int64_t src;     // canonical offset of W
  int64_t src_b;   // canonical offset of b
  int cout, cin;   // real channel counts
  int cu, cu_p;    // UPCAT split: real / padded channels of the first source
  int cin_p, cout_p;
  int64_t dst;     // byte offset of packed weights
  int64_t dst_b;   // byte offset of packed bias
};
hipError_t launch_pack_conv(int precision, const float* canon, void* packed, const PackConv& p,
                            hipStream_t st);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st);

}  // namespace omniseg

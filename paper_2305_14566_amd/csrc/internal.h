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
// The hardware deals the workgroups of a launch to the eight XCDs round
// robin (workgroup x to XCD x % 8), and each XCD has its own L2.  The conv
// kernels read their block index through this bijection, under which XCD j
// runs one contiguous range of logical indices: the output-channel blocks of
// a pixel block and neighbouring pixel blocks, which read the same input
// rows, then share an L2 instead of each XCD fetching them.
__device__ __forceinline__ int xcd_remap(int x, int n) {
  constexpr int X = 8;
  const int q = n / X, r = n % X, j = x % X, i = x / X;
  return (j < r ? j * (q + 1) : r * (q + 1) + (j - r) * q) + i;
}

// Largest grid extent the kernels launch in y (row loops stride over the rest).
constexpr int kMaxGridY = 65535;

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
  short s[kMaxGroups];         // tile stride of the group's scale slot
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
hipError_t launch_tile_flags(const TileGroups& g, const SlideDev* slides_dev, int T, int kc,
                             int fg_filter, int32_t* flags, hipStream_t st);
// Merge of per-class planes to the 40x base, and the colour overlay (k_map.hip).
struct MergePlane {
  const uint8_t* mask;   // nearest: the scale-k mask
  const float* logit;    // bilinear: the scale-k logit plane
  int64_t pitch;         // source row pitch in elements
  int k, Hk, Wk;
  int bilinear;
  uint8_t* out;          // the 40x mask
  int64_t out_pitch;
  int vec4;              // out and out_pitch are multiples of 4: 4-byte stores
  int vec16;             // out and out_pitch are multiples of 16: 16-byte stores
  int vec_src;           // source rows start 16-byte aligned: vector loads
};
struct MergeArgs {
  int H, W;
  MergePlane plane[OMNISEG_MAX_CLASSES];
};
hipError_t launch_merge_base(const MergeArgs& a, int n_planes, hipStream_t st);
struct OverlayClass {
  const uint8_t* mask;   // mask at scale k
  int64_t pitch;
  int k;
  int alpha;             // [0, 256]
  int rgb[3];
  int vec4;              // mask and pitch are multiples of 4: 4-byte mask loads at k = 0
};
struct OverlayArgs {
  const uint8_t* rgb;
  int64_t pitch;
  int H, W;
  int n;
  OverlayClass cls[OMNISEG_MAX_CLASSES];
  uint8_t* out;
  int64_t out_pitch;
  uint8_t* out10;        // optional 4x4 box-mean map
  int64_t out10_pitch;
  int vec;               // rgb, out and their pitches are multiples of 4: word loads and stores
};
hipError_t launch_overlay(const OverlayArgs& a, hipStream_t st);

// Otsu tissue detection of one slide on the coarse scale kc (k_tissue.hip).
struct TissueOtsuArgs {
  const uint8_t* rgb;     // the 40x slide (read when kc == 0)
  int64_t pitch;
  const uint16_t* sums;   // box sums of scale kc (kc >= 1), row pitch ex pixels
  int ex;
  int kc, Hc, Wc;
  int median;             // odd median kernel size; 1 = no blur
  int min_area;           // smallest kept 8-connected component, in coarse pixels
  uint8_t* tmp;           // Hc*Wc: the gray map before the blur (median > 1)
  uint8_t* gray;          // Hc*Wc: the blurred gray map
  uint32_t* hist;         // 256 counts
  int32_t* stats;         // threshold, components, kept components, error flag
  int32_t* label;         // Hc*Wc
  int32_t* area;          // Hc*Wc
  uint8_t* fg;            // Hc*Wc: the tissue map
};
hipError_t launch_tissue_otsu(const TissueOtsuArgs& a, hipStream_t st);
hipError_t launch_compact(int32_t* flags_to_index, int total, const TileGroups& g,
                          int32_t* list, int32_t* count, int32_t* pre, hipStream_t st);

struct ConvLayer {
  int cin_p;      // padded input channels (concat: cu_p + ce_p)
  int cu_p;       // UPCAT: padded channels of the upsampled source
  int cout_p;     // padded output channels
  const void* w;  // packed weights [ceil(cin_p / KC)][9][cout_p][KC]
  const float* b; // bias [cout_p]
  // FP8 only: per-output-channel weight scale, the residual input's channel
  // scales (residual epilogues) and the output tensor's inverse channel scales
  const float* wscale = nullptr;
  const float* rscale = nullptr;
  const float* oinv = nullptr;
  // BF16 / FP8 row-reuse configurations, RES_RELU: also write the 2x2
  // max-pool of the output here ([batch][H/2][W/2][cout_p]); null = no pool
  void* pool_out = nullptr;
};

// FP8 E4M3 storage: channels per LDS chunk of the FP8 conv (one K = 64 MFMA
// step per tap), and the largest finite magnitude.
constexpr int kFp8Chunk = 64;
constexpr float kFp8Max = 448.0f;

enum Loader { LOAD_PLAIN = 0, LOAD_POOL = 1, LOAD_UPCAT = 2 };
// RELU: ReLU(acc + bias).  RES_RELU: ReLU(acc + bias + x0).  NONE: acc (data
// gradients).  RES_MASK: (acc + x0) where aux > 0, else 0 (the data gradient
// of a residual conv block, through the ReLU of its first conv).
enum Epilogue { EPI_RELU = 0, EPI_RES_RELU = 1, EPI_NONE = 2, EPI_RES_MASK = 3, EPI_RES_RELU_PRECLS = 4 };

// 3x3 conv on a batch of tiles (NHWC, padded channels), output H x W per tile.
// Conv tile configurations (pixel block, output channels, wave layout).  The
// first six run for FP32 and BF16 with 16-pixel M fragments inside the
// block; the ROWS configurations (BF16 only) give each wave whole 16-pixel
// rows of the block and reuse every loaded halo row across the three
// vertical taps.
enum ConvConfig {
  CONV_CFG_8x16_32 = 0,
  CONV_CFG_8x16_64,
  CONV_CFG_16x16_64,
  CONV_CFG_8x16_128,
  CONV_CFG_8x8_32,
  CONV_CFG_8x8_64,
  CONV_CFG_ROWS_16x16_64,
  CONV_CFG_ROWS_16x16_128,
  CONV_CFG_ROWS_32x16_32,
  CONV_CFG_ROWS_16x16_32,
  CONV_CFG_ROWS8_16x16_64,  // eight waves (BF16)
  CONV_CFG_ROWS2_32x16_64,  // eight waves, double-buffered staging, register epilogue (BF16)
  CONV_CFG_ROWS2P_32x16_64, // the same, persistent: one workgroup per CU walks the blocks (BF16)
  CONV_CFG_COUNT
};
bool conv_config_valid(int cfg, int precision, int H, int W, int cout_p);
void conv_config_shape(int cfg, int* by, int* bx, int* bn, int* wm, int* wn);
// Bit p set when the configuration runs at precision p.
int conv_config_precisions(int cfg);
int conv_default_config(int precision, int H, int W, int cout_p);

// The decoder's last residual conv fused with the head's precls (BF16,
// 64 -> 64 channels, weight-stationary form): writes F = ReLU(W_p D + b_p)
// (FP32, [tile][H W][8]) instead of D.  The launch applies when
// conv_precls_fusable holds (else hipErrorInvalidValue).
bool conv_precls_fusable(const ConvLayer& L, int H, int W, int batch);
hipError_t launch_conv_ws_precls(const ConvLayer& L, int H, int W, int batch, const int32_t* count, int chunk_base,
                                 const void* x0, const float* pre_w, const float* pre_b, float* fpre,
                                 hipStream_t st);
// cfg < 0 (or not valid for the shape) picks the default configuration.
hipError_t launch_conv3x3(int precision, int loader, int epi, const ConvLayer& L, int H, int W,
                          int batch, const int32_t* count, int chunk_base, const void* x0,
                          const void* x1, void* y, hipStream_t st, const void* aux = nullptr,
                          int cfg = -1);

// First conv (3 -> C_0) straight from the slide / pyramid.
struct FirstConvArgs {
  const int32_t* list;  // tile list int32[4] per tile
  const int32_t* count;
  int chunk_base;
  int batch;
  int T;
  int scale_s[OMNISEG_MAX_SCALES];  // tile stride per scale slot
  const float* w;  // [C_0][27] (c, dy, dx order: w[o][c*9 + dy*3 + dx])
  const float* b;  // [C_0]
  int c0, c0_p;
  void* y;  // [batch][T][T][c0_p]
  const SlideDev* slides;  // device array, one per slide
  int scale_k[OMNISEG_MAX_SCALES];
  const float* oinv = nullptr;  // FP8: inverse channel scales of the output
};
hipError_t launch_first_conv(int precision, const FirstConvArgs& a, hipStream_t st);

// scale: FP8 channel scales of e (null otherwise)
hipError_t launch_gap(int precision, const void* e, int batch, int hw, int c_p, int c,
                      const int32_t* count, int chunk_base, float* g, hipStream_t st,
                      const float* scale = nullptr);

struct SlotTable {
  int n_slots[OMNISEG_MAX_SCALES];
  int cls[OMNISEG_MAX_SCALES][OMNISEG_MAX_CLASSES];
};

hipError_t launch_controller(const float* g, int batch, int G, const float* wc, const float* bc,
                             int P, int n_classes, int n_scales, const SlotTable& slots,
                             int max_slots, const int32_t* list, const int32_t* count,
                             int chunk_base, float* theta, hipStream_t st);

// Tile chunk_base + b of the list writes its logits to slot out_base + b of
// tile_logits.  d0_scale: FP8 channel scales of d0 (null otherwise).
// fpre: the precls output F (8 FP32 values per pixel, [tile][T^2][8]) already
// computed by the decoder's last conv (see launch_conv_ws_precls); d0 is then
// not read.
hipError_t launch_head(int precision, const void* d0, int batch, int T, int c0, int c0_p,
                       const float* wp, const float* bp, const float* theta, int P, int o,
                       const SlotTable& slots, int max_slots, const int32_t* list,
                       const int32_t* count, int chunk_base, int out_base, float* tile_logits,
                       hipStream_t st, const float* d0_scale = nullptr, const float* fpre = nullptr);

// ---- BF16 precls on MFMA (shared by the head and the fused conv epilogue) ----
//
// F = ReLU((P_0 + P_1) + b_p) with P_h = W_p[:, 32 h .. 32 h + 31] D_0[32 h ..
// 32 h + 31] for C_0 = 64 (P_1 = 0 for C_0 <= 32), each P_h one chain of
// three v_mfma_f32_16x16x32_bf16: every FP32 weight is split into three BF16
// terms, w = hi + mid + lo exactly (hi = bf16(w), mid = bf16(w - hi), and the
// remainder has at most eight significant bits), so with BF16 D_0 each
// product is exact and the sums run in FP32.  Operand layout of half h: lane
// (g, l16) of the A operand holds output row o = l16 (rows 8-15 zero) and of
// the B operand pixel l16; K slot 8 g + j holds channel 32 h + 4 g + j for
// j < 4 and 32 h + 16 + 4 g + (j - 4) for j >= 4 (the channels a lane of the
// conv epilogue holds as its two 16-channel fragments).  Result lane (g, l16),
// g < 2, holds outputs 4 g .. 4 g + 3 of pixel l16.
typedef __attribute__((ext_vector_type(4))) float pf32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 pbf16x8;

__device__ __forceinline__ uint32_t precls_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return u >> 16;
}

// The three A operands (hi, mid, lo) of half h for this lane.
__device__ __forceinline__ void precls_weights(const float* __restrict__ wp, int c0, int h, int lane,
                                               uint4 (&A)[3]) {
  const int g = lane >> 4, o = lane & 15;
  uint32_t t[3][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = 32 * h + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
    const float w = (o < 8 && c < c0) ? wp[o * c0 + c] : 0.f;
    const uint32_t hi = precls_bf16_rne(w);
    const float r1 = w - __uint_as_float(hi << 16);
    const uint32_t mid = precls_bf16_rne(r1);
    t[0][j] = hi;
    t[1][j] = mid;
    t[2][j] = precls_bf16_rne(r1 - __uint_as_float(mid << 16));
  }
#pragma unroll
  for (int q = 0; q < 3; ++q)
    A[q] = make_uint4(t[q][0] | (t[q][1] << 16), t[q][2] | (t[q][3] << 16), t[q][4] | (t[q][5] << 16),
                      t[q][6] | (t[q][7] << 16));
}

// P_h for 16 pixels: B = the lane's eight BF16 values in the K-slot order above.
__device__ __forceinline__ pf32x4 precls_half(const uint4 (&A)[3], uint4 B) {
  pf32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 3; ++q)
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(pbf16x8, A[q]), __builtin_bit_cast(pbf16x8, B),
                                                  acc, 0, 0, 0);
  return acc;
}

// ---- FP8 calibration and packing --------------------------------------------

// amax[c] = max(amax[c], max over pixels of x[p][c]) for an FP32 tensor of
// npix pixels x c_p channels whose values are >= 0 (ReLU outputs).
hipError_t launch_amax_channels(const float* x, int64_t npix, int c_p, float* amax, hipStream_t st);
// Padded-order scales of one stand-alone FP8 conv: s_in_pad[cp] = the real
// input channel's scale (1 for padding), oinv[o] = 1 / out_scale[o] (1 for
// padding).
hipError_t launch_fp8_conv_scales(const float* in_scale, int cin, int cu, int cu_p, int cin_p,
                                  const float* out_scale, int cout, int cout_p, float* s_in_pad, float* oinv,
                                  hipStream_t st);
// scale[i] = 2^ceil(log2(amax[i] / 448)) (1 for amax <= 0), inv[i] = 1 / scale[i].
hipError_t launch_fp8_scales(const float* amax, int64_t n, float* scale, float* inv, hipStream_t st);

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
  int coverage;       // 1: mask = (D > 0) instead of (N > 0)
  int vote;           // > 0: majority vote -- mask = (number of covering tiles with logit > 0) >= vote
  int ring = 0;       // > 0: list index t lives in logit slot t % ring (a ring store)
};
hipError_t launch_stitch(const StitchArgs& a, hipStream_t st);

// ---- streamed stitch of omniseg_segment_slide ---------------------------------
//
// The backbone runs over the kept-tile list in batches of B list positions
// (batch b holds positions [b B, (b + 1) B)), and the tile logits go to a
// ring of slots (position p in slot p % ring).  The output planes are
// stitched in units of one tile row: unit (group g, row j) owns the output
// rows whose last covering tile row is j, [j s, (j + 1) s) (the last row of
// the grid also owns the rows below it, down to H_k).  Its covering tiles are
// list positions before pre[grid index of (j + 1, 0)], so the unit is stitched
// right after the batch that holds the last of them (batch 0 when there is
// none).  Units are enumerated group by group, rows in order, so their
// batches do not decrease.  Each unit is cut into items: one plane (pair),
// kStitchRows output rows and kStitchCols columns each.
constexpr int kStitchRows = 16;
constexpr int kStitchCols = 1024;

struct StreamGroup {
  int64_t grid_base;   // canonical index of the group's first grid tile
  int64_t item_base;   // first item of the group
  int ny, nx, s, Hk, Wk;
  int unit_base;       // first unit of the group
  int nxc;             // column chunks per row: ceil(Wk / kStitchCols)
  int plane_first, n_planes;
  const uint8_t* fg;   // tissue map for mask_and_fg (or null)
  int fg_shift, Hc, Wc;
  int vote;            // > 0: majority vote threshold of the group's scale slot
};
struct StreamPlane {
  uint8_t* mask;
  float* logit;        // or null
  int64_t mask_pitch, logit_pitch;
  int64_t slot_off;    // float offset of the pair's plane inside a tile slot
  int mode;            // 0: one pixel per thread; 1: four; 2: four, at most 2 x 2 covering tiles
  int pad_;
};
struct StreamUnit {
  int batch;           // the batch after which the unit is stitched
  int g, y0, y1;
  int64_t item_base;   // first item of the unit (the entry after the last unit: the item count)
};
struct StreamStitchArgs {
  const StreamGroup* groups;
  const StreamPlane* planes;
  StreamUnit* units;   // n_units + 1 entries
  int32_t* batch_first;  // n_batches + 1 entries: the first unit of each batch (n_units past the last)
  int n_batches;
  int n_groups, n_units;
  const int32_t* pre;  // kept tiles before each grid tile (grid tiles + 1 entries)
  const int32_t* index;  // list index per grid tile, or -1
  const float* logits;
  int64_t tile_stride; // floats per logit slot
  int ring;            // logit slots
  int T, B;            // tile size, list positions per batch
  int batch;           // k_stitch_stream: the batch just computed
  int64_t n_items;     // items of all units
};
// Unit table from the compacted list (one thread per unit).
hipError_t launch_stream_units(const StreamStitchArgs& a, hipStream_t st);
// Stitches every unit of batch a.batch.
hipError_t launch_stitch_stream(const StreamStitchArgs& a, hipStream_t st);
// Writes `bytes` (a multiple of 4) from host memory to device memory with
// kernels whose arguments carry the data, so the write is captured by value
// in a HIP graph (no host pointer is kept).
hipError_t launch_put(void* dst, const void* src, int64_t bytes, hipStream_t st);
hipError_t launch_grid_from_list(const int32_t* tile_yx, int n_tiles, int ny, int nx,
                                 int32_t* grid, hipStream_t st);

// ---- backward ---------------------------------------------------------------

hipError_t launch_input_x(const FirstConvArgs& a, float* x, hipStream_t st);

struct StitchBwdArgs {
  const float* dlam;  // flat per-pair gradient planes
  float* dl;          // [n_tiles][max_slots][T][T]
  const int32_t* list;
  int n_tiles, T, s, max_slots;
  int ny[OMNISEG_MAX_SCALES], nx[OMNISEG_MAX_SCALES], Hk[OMNISEG_MAX_SCALES], Wk[OMNISEG_MAX_SCALES];
  const int32_t* grid[OMNISEG_MAX_SCALES];
  int n_slots[OMNISEG_MAX_SCALES];
  int64_t plane_off[OMNISEG_MAX_SCALES][OMNISEG_MAX_CLASSES];
};
hipError_t launch_stitch_bwd(const StitchBwdArgs& a, hipStream_t st);

struct HeadBwdArgs {
  const void* d0;         // decoder output D_0 [tile][T][T][c0_p]
  const float* theta;     // [tile][max_slots][P]
  const float* dl;        // [tile][max_slots][T][T]
  const float* wp;        // precls W [8][c0] (or null)
  const float* bp;
  const int32_t* list;
  int n_slots[OMNISEG_MAX_SCALES];
  int n_tiles, T, c0, c0_p, o, max_slots;
  float* dtheta_part;     // [tile][max_slots][T*T/256][P]
  float* dwp_part;        // [tile][T*T/256][8 c0 + 8]
  void* dd0;              // dL/dD_0 [tile][T][T][c0_p]
  int mask_d0;            // store dd0 through the ReLU that produced D_0 (zero where D_0 <= 0)
};
hipError_t launch_head_bwd(int precision, const HeadBwdArgs& a, hipStream_t st);
hipError_t launch_sum_mid(const float* in, int R, int K, int I, float* out, float* part, hipStream_t st);
int64_t sum_mid_part_floats(int R, int K, int I);  // scratch launch_sum_mid needs

struct CtrlBwdArgs {
  const float* dtheta;  // [tile][max_slots][P]
  const float* g;       // [tile][g_stride]
  const float* wc;      // [P][row_len]
  const int32_t* list;
  int n_slots[OMNISEG_MAX_SCALES];
  int cls[OMNISEG_MAX_SCALES][OMNISEG_MAX_CLASSES];
  int n_tiles, max_slots, P, G, g_stride, n_classes, row_len;
  float* dwc;  // canonical W_c gradient
  float* dbc;  // canonical b_c gradient
  float* dg;   // [tile][g_stride]
};
hipError_t launch_ctrl_bwd(const CtrlBwdArgs& a, hipStream_t st);

hipError_t launch_gap_bwd(int precision, const float* dg, int g_stride, int G, int hw, int c_p, int n_tiles,
                          void* dE, hipStream_t st);
hipError_t launch_relu_mask(int precision, const void* dy, const void* y, int64_t n, void* out, hipStream_t st);
hipError_t launch_concat_bwd(int precision, const void* dZ, int n_tiles, int H, int W, int cu_p, int ce_p,
                             void* dE, void* dD, int accumulate, const void* ymask, hipStream_t st);
hipError_t launch_maxpool_bwd(int precision, const void* E, const void* dX, int n_tiles, int H, int W, int c_p,
                              void* dE, hipStream_t st, int relu);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);
hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t st);

struct WgradArgs {
  const void* x0;  // forward conv input (loader source)
  const void* x1;  // UPCAT skip source
  const void* dy;  // gradient at the conv output [tile][H][W][cout_p]
  float* part;     // [splits][cout_p][9][cin_p]
  int H, W, cin_p, cu_p, cout_p, n_tiles, splits;
};
int wgrad_bo(int cout_p);
hipError_t launch_wgrad(int precision_x, int precision_g, int loader, const WgradArgs& a, int cout, int cin,
                        int cu, float* dst, hipStream_t st);
// The first conv's weight gradient (3 input channels in FP32, padded to x_cp
// per pixel; dY in precision_g with cout_p channels) into dst[cout][3][9],
// through `splits` partials of cout_p * 36 floats each.
hipError_t launch_wgrad_first(int precision_g, const float* x, int x_cp, const void* dy, int n, int T, int cout,
                              int cout_p, float* part, int splits, float* dst, hipStream_t st);
// Split count of the bias gradient over npix pixels (at most kBiasGradSplits).
constexpr int kBiasGradSplits = 512;
int bias_grad_splits(int64_t npix);
hipError_t launch_bias_grad(int precision, const void* dy, int64_t npix, int c_p, int cout, float* part,
                            int splits, float* dst, hipStream_t st);
hipError_t launch_bce(const float* lg, const float* y, const uint8_t* valid, int64_t n, double* part_sum,
                      int* part_cnt, int nb, double* loss, int* count, float* grad, hipStream_t st);

// Weight packing
struct PackConv {
  int64_t src;     // canonical offset of W
  int64_t src_b;   // canonical offset of b
  int cout, cin;   // real channel counts
  int cu, cu_p;    // UPCAT split: real / padded channels of the first source
  int cin_p, cout_p;
  int64_t dst;     // byte offset of packed weights
  int64_t dst_b;   // byte offset of packed bias (< 0: none)
  int transpose;   // 1: pack the data-gradient conv (channels swapped, taps flipped)
};
// FP8 packing of one conv: input channel scales s_in (padded channel order,
// cin_p entries: the upsampled part's then the skip part's) fold into the
// columns, each output channel gets a power-of-two scale (wscale[o]) and the
// codes go to [ceil(cin_p / 64)][9][cout_p][64]; bias copied to dst_b.
hipError_t launch_pack_conv_fp8(const float* canon, void* packed, const PackConv& p, const float* s_in_u,
                                const float* s_in_e, float* wscale, hipStream_t st);
hipError_t launch_pack_conv(int precision, const float* canon, void* packed, const PackConv& p,
                            hipStream_t st);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st);

}  // namespace omniseg

/*
 * omniseg.h -- C ABI of the MI355X (gfx950) slide-wise Omni-Seg hot path.
 *
 * The library segments whole-slide images (WSIs) the way the accelerated
 * pipeline of arXiv 2305.14566 does on one GPU:
 *   1. pad the slide with the rounded mean colour of its top-left 2x2 block
 *      and resample it into a multi-scale pyramid (Section 2.1; Section 2.2:
 *      several magnifications from the 40x base);
 *   2. keep only tiles that touch tissue (Section 2.1, blank-region removal);
 *   3. run a residual U-Net on every kept tile, whose 1x1 dynamic head is
 *      generated per tile by a controller from a class x scale one-hot code
 *      (the dynamic multi-class multi-scale network the paper applies,
 *      Section 2.2);
 *   4. merge the overlapping tile logits of each class into a whole-slide
 *      mask, by the majority vote of overlapping tile predictions (Section
 *      2.2 overlap tiling; thresholds and strides in Section 3.2) or by a
 *      ramp-weighted average and a threshold (Section 2.3 slide-wise
 *      aggregation).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int32_t status (OMNISEG_OK = 0 or one of the
 *     OMNISEG_ERR_* codes).  No C++ exception crosses the ABI.
 *   - Arguments are validated before any HIP call.  On an error nothing is
 *     launched and no caller buffer is written; omniseg_last_error() gives a
 *     thread-local description of the last failure.
 *   - "device" pointers point to memory on the current HIP device; "host"
 *     pointers to ordinary host memory.  The caller owns every buffer it
 *     passes in (slides, weights, outputs, workspace); the library never
 *     frees caller memory and never allocates device memory.
 *   - Work is enqueued asynchronously on the given stream (NULL = the null
 *     stream).  Device buffers must stay valid until that work completes.
 *   - A plan is not thread-safe; use one plan per stream at a time.
 */
#ifndef OMNISEG_H
#define OMNISEG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OMNISEG_ABI_VERSION 7

/* status codes */
#define OMNISEG_OK 0
#define OMNISEG_ERR_ARG 1         /* a NULL pointer, a size out of range, ... */
#define OMNISEG_ERR_UNSUPPORTED 2 /* a valid but unsupported configuration  */
#define OMNISEG_ERR_WORKSPACE 3   /* the workspace is smaller than required  */
#define OMNISEG_ERR_HIP 4         /* a HIP runtime call failed               */

/* backbone arithmetic */
#define OMNISEG_FP32 0 /* FP32 activations and weights, FP32 MFMA           */
#define OMNISEG_BF16 1 /* BF16 activations and weights, FP32 accumulation   */
#define OMNISEG_FP8 2  /* FP8 E4M3 activations and 3x3 weights with per-channel
                        * power-of-two scales, FP32 accumulation (inference
                        * only; weights from omniseg_pack_weights_fp8)       */

/* flags */
#define OMNISEG_FLAG_EMIT_LOGITS 1 /* also write the stitched FP32 logit map */
#define OMNISEG_FLAG_TRAINING 2    /* also pack the data-gradient weights (training entry points) */
#define OMNISEG_FLAG_GRAPH 4       /* omniseg_segment_slide: capture the whole call in a HIP graph,
                                      replayed on later calls with identical arguments and conv
                                      tile configurations (whatever the slides' pixels hold);
                                      needs a created (non-null) stream */

/* merge of overlapping tile predictions (omniseg_config.merge) */
#define OMNISEG_MERGE_RAMP 0 /* ramp-weighted mean of the tile logits, mask = mean > 0 */
#define OMNISEG_MERGE_VOTE 1 /* majority vote: mask = (number of covering tiles whose
                                logit is > 0) >= vote_threshold of the pair's scale */

/* tissue detection (omniseg_config.tissue_method) */
#define OMNISEG_TISSUE_GRAY 0 /* fixed gray threshold fg_threshold on the coarsest scale */
#define OMNISEG_TISSUE_OTSU 1 /* Otsu threshold of the median-blurred coarsest-scale gray map,
                                 then 8-connected tissue components smaller than
                                 min_tissue_area removed (Sections 2.1 and 3.2) */

/* limits */
#define OMNISEG_MAX_SCALES 4
#define OMNISEG_MAX_CLASSES 16
#define OMNISEG_MAX_SLIDES 32

typedef struct omniseg_hip_stream_opaque* omniseg_stream; /* a hipStream_t */

/*
 * Network and tiling configuration.
 *   base_channels  C_0 >= 1; encoder/decoder level l has C_0 * 2^l channels.
 *   levels         L >= 1 U-Net levels; tile / 2^(L-1) must be a multiple of 8.
 *   head_out       1 or 2 outputs of the dynamic head; with 2 the class logit
 *                  is z_1 - z_0 (two-way softmax), with 1 it is z_0.
 *   n_classes      C in [1, 16] (the class one-hot length).
 *   n_scales       S in [1, 4] (the scale one-hot length).
 *   scale_log2     downsampling exponent of each scale slot: slot i is the
 *                  magnification 40x / 2^scale_log2[i] (0 = 40x, 1 = 20x,
 *                  2 = 10x, 3 = 5x); values in [0, 3].
 *   tile, stride   square tile size T (a multiple of 16, <= 512) and the
 *                  overlap stride s (1 <= s <= T).
 *   scale_stride   per scale slot: the tile stride of that slot's grid in
 *                  [1, T], or 0 for `stride` (Section 3.2 tiles 40x with
 *                  stride 256 and 10x, 5x with stride 64).  Training plans
 *                  need every slot at `stride`.
 *   merge          OMNISEG_MERGE_RAMP or OMNISEG_MERGE_VOTE (Section 2.2
 *                  majority vote; training plans need RAMP).
 *   vote_threshold per scale slot, with MERGE_VOTE: the least number of
 *                  covering kept tiles that must predict the class, in
 *                  [1, ceil(T / s_slot)^2] (Section 3.2: 1 at 40x, 4 at
 *                  10x and 5x); ignored with MERGE_RAMP.
 *   fg_filter      1: keep only tiles whose footprint touches a foreground
 *                  pixel of the tissue map; 0: keep every tile.
 *   fg_threshold   gray threshold of the tissue map (pixels darker than this
 *                  on the coarsest scale are tissue), in [1, 255]; used by
 *                  OMNISEG_TISSUE_GRAY.
 *   tissue_method  OMNISEG_TISSUE_GRAY or OMNISEG_TISSUE_OTSU.  The tissue
 *                  map decides which tiles are kept (fg_filter) and, with
 *                  mask_and_fg, where masks may be on.  OTSU, on the
 *                  coarsest scale kc: gray g = round((299 R + 587 G + 114 B)
 *                  / (1000 4^kc)) of the block sums (an integer in [0, 255]);
 *                  median_kernel x median_kernel median with replicated
 *                  borders; Otsu's threshold t of the blurred map (the first
 *                  t maximising n0 n1 (mu0 - mu1)^2 over the splits {<= t},
 *                  {> t}, compared exactly in integers; a one-valued map has
 *                  no tissue); tissue = blurred gray <= t; then 8-connected
 *                  tissue components of fewer than min_tissue_area pixels are
 *                  removed.  The coarse map must have fewer than 2^28 pixels.
 *   median_kernel  odd, in [1, 255] (1 = no blur); OTSU only.
 *   min_tissue_area  >= 0, in coarse pixels (0 or 1 keep every component);
 *                  OTSU only.
 *   mask_and_fg    1: the output mask is also ANDed with the tissue map.
 *   scale_log2 must not repeat a value across the n_scales slots.
 *   precision      OMNISEG_FP32, OMNISEG_BF16 or OMNISEG_FP8 (not with
 *                  OMNISEG_FLAG_TRAINING).
 *   flags          OR of OMNISEG_FLAG_*.
 *   batch_tiles    list positions per backbone batch B (0 = library
 *                  default, 256).
 *   logit_ring_tiles  slots of the per-tile logit store in the workspace:
 *                  0 gives every grid tile a slot, so every kept tile's
 *                  logits stay readable after the call; n > 0 makes it a
 *                  ring of max(n, the least ring the streamed stitch needs)
 *                  slots rounded up to a multiple of B (at most one per grid
 *                  tile), which bounds the workspace for many or large
 *                  slides.  The least ring is (max over tile rows j of
 *                  (j + 1 - jlo) nx) + B - 1 slots, where jlo is the first
 *                  tile row reaching row j's first output row.  Outputs do
 *                  not depend on the ring size.
 */
typedef struct omniseg_config {
  int32_t abi_version;
  int32_t base_channels;
  int32_t levels;
  int32_t head_out;
  int32_t n_classes;
  int32_t n_scales;
  int32_t scale_log2[OMNISEG_MAX_SCALES];
  int32_t tile;
  int32_t stride;
  int32_t fg_filter;
  int32_t fg_threshold;
  int32_t mask_and_fg;
  int32_t precision;
  int32_t flags;
  int32_t batch_tiles;
  int32_t logit_ring_tiles;
  int32_t scale_stride[OMNISEG_MAX_SCALES];
  int32_t merge;
  int32_t vote_threshold[OMNISEG_MAX_SCALES];
  int32_t tissue_method;
  int32_t median_kernel;
  int32_t min_tissue_area;
} omniseg_config;

/* One slide: uint8 RGB, interleaved (HWC), rows `row_pitch` bytes apart
 * (row_pitch >= 3 * width).  rgb points to device memory.  height, width >= 2. */
typedef struct omniseg_slide {
  const uint8_t* rgb;
  int32_t height;
  int32_t width;
  int64_t row_pitch;
} omniseg_slide;

/* One requested output: class index and scale slot. */
typedef struct omniseg_pair {
  int32_t cls;
  int32_t scale;
} omniseg_pair;

/* Output buffers of one (slide, pair), at the pair's scale:
 * H_k = ceil(height / 2^k) rows, W_k = ceil(width / 2^k) columns.
 * mask: device uint8, 1 = the class is present; rows mask_pitch bytes apart.
 * logit: device float or NULL; written only with OMNISEG_FLAG_EMIT_LOGITS;
 * rows logit_pitch floats apart; 0 where no kept tile covers the pixel.
 * With OMNISEG_MERGE_VOTE the logit plane holds the vote count instead (the
 * number of covering kept tiles whose logit is > 0, as a float). */
typedef struct omniseg_output {
  uint8_t* mask;
  float* logit;
  int64_t mask_pitch;
  int64_t logit_pitch;
} omniseg_output;

typedef struct omniseg_plan omniseg_plan;

/* Text of a status code (static storage). */
const char* omniseg_status_string(int32_t status);
/* Thread-local text of the last error raised on this thread ("" if none). */
const char* omniseg_last_error(void);

/*
 * Validate a configuration and build a plan (host memory only; no HIP call).
 * cfg: host pointer.  *out receives the plan; release it with
 * omniseg_plan_destroy.  Errors: ERR_ARG for NULL pointers or out-of-range
 * fields, ERR_UNSUPPORTED for valid but unsupported shapes.
 */
int32_t omniseg_plan_create(const omniseg_config* cfg, omniseg_plan** out);
/* Free a plan (NULL is accepted). */
int32_t omniseg_plan_destroy(omniseg_plan* plan);

/*
 * Number of FP32 values of the canonical weight vector.  Canonical order:
 * encoder levels 0..L-1 (conv_a W[C_l][C_in][3][3], b[C_l], conv_b W, b),
 * decoder levels L-2..0 (conv_a W[C_l][3 C_l][3][3] whose input channels are
 * the 2 C_l upsampled channels then the C_l skip channels, b, conv_b W, b),
 * precls W[8][C_0], b[8] only when C_0 != 8, then the controller
 * W_c[P][C_{L-1} + C + S] and b_c[P], P = 144 + 9 * head_out.
 */
int32_t omniseg_weight_count(const omniseg_plan* plan, int64_t* count);
/* Bytes of the packed (device-internal) weight buffer for this plan. */
int32_t omniseg_packed_weight_bytes(const omniseg_plan* plan, int64_t* bytes);
/*
 * Convert the canonical FP32 weights (device, omniseg_weight_count floats)
 * into the packed layout the kernels read (device, omniseg_packed_weight_bytes
 * bytes, 256-byte aligned).  Channel padding, MFMA-friendly ordering and the
 * precision conversion happen here, once per weight set.
 */
int32_t omniseg_pack_weights(const omniseg_plan* plan, const float* canonical,
                             void* packed, omniseg_stream stream);

/*
 * FP8 backbone (precision OMNISEG_FP8; the paper's pipeline runs its network
 * in FP32, Section 2.2 -- this is a reduced-precision form of that step).
 * Every stored backbone activation t keeps one power-of-two scale s_t[c] per
 * channel and holds E4M3(x_c / s_t[c]) (OCP FP8 E4M3: 4 exponent bits with
 * bias 7, 3 fraction bits, largest value 448, ties to even, saturating).
 * Each 3x3 conv except the first folds its input's channel scales into the
 * weight columns (W'[o][c] = W[o][c] s_in[c]) and stores W'[o] as E4M3 with
 * its own power-of-two scale w_o; the MFMA sums exact FP8 products in FP32,
 * and the epilogue forms w_o acc + b_o (+ the residual decoded with its
 * scales), applies ReLU and encodes the result with the output's scales.
 * The first conv (from the RGB tile), the controller and the head compute in
 * FP32 (the first conv as FP32 sums of exact products: its MFMAs take exact
 * BF16 splits of the FP32 weights and of the integer inputs).  A scale is 2^ceil(log2(amax / 448)) of the channel's maximum over
 * calibration tiles (1 if that maximum is 0).
 *
 * Activation table: one float per padded channel (pad32(C_l)) of every
 * stored activation, ordered by kind then level: OMNISEG_ACT_ENC_A (conv_a
 * outputs of encoder levels 0..L-1; level 0 is the first conv's output),
 * OMNISEG_ACT_ENC_E (encoder block outputs E_0..E_{L-1}), OMNISEG_ACT_DEC_A
 * (decoder conv_a outputs of levels 0..L-2), OMNISEG_ACT_DEC_D (decoder block
 * outputs D_0..D_{L-2}).
 */
#define OMNISEG_ACT_ENC_A 0
#define OMNISEG_ACT_ENC_E 1
#define OMNISEG_ACT_DEC_A 2
#define OMNISEG_ACT_DEC_D 3
/* Length of the activation table of this plan's network (any precision). */
int32_t omniseg_activation_channels(const omniseg_plan* plan, int64_t* count);
/* Offset (in floats) of (kind, level) inside the activation table; ERR_ARG
 * for a kind or level the network does not have. */
int32_t omniseg_activation_offset(const omniseg_plan* plan, int32_t kind, int32_t level,
                                  int64_t* offset);
/*
 * Calibration pass for the FP8 backbone.  `plan` must be an FP32 plan (no
 * TRAINING flag) of the same network, `packed` its weights from
 * omniseg_pack_weights.  Runs the backbone on the first min(n_tiles, kept)
 * kept tiles of these slides in tile-list order (slide, scale slot, tile row,
 * tile column) and writes each stored activation's per-channel maximum into
 * amax (device, omniseg_activation_channels floats; padded channels get 0).
 * Same slides, pairs and workspace rules as omniseg_segment_slide; no
 * outputs are written.  Waits for the stream.  n_tiles >= 1.
 */
int32_t omniseg_calibrate_fp8(const omniseg_plan* plan, const void* packed,
                              const omniseg_slide* slides, int32_t n_slides,
                              const omniseg_pair* pairs, int32_t n_pairs, int32_t n_tiles,
                              float* amax, void* workspace, int64_t ws_bytes,
                              omniseg_stream stream);
/*
 * Pack canonical weights (device) for an FP8 plan, with the channel scales
 * derived from `amax` (device activation table, e.g. from
 * omniseg_calibrate_fp8).  The packed buffer (omniseg_packed_weight_bytes,
 * 256-byte aligned) then also holds the scale tables the kernels read.
 * omniseg_pack_weights refuses FP8 plans (ERR_UNSUPPORTED).
 */
int32_t omniseg_pack_weights_fp8(const omniseg_plan* plan, const float* canonical,
                                 const float* amax, void* packed, omniseg_stream stream);

/*
 * Workspace bytes that omniseg_segment_slide needs for these slides and
 * pairs (host arrays).  The bound assumes every tile passes the tissue
 * filter.  A tile grid (one slide at one scale) of more than 32767 tiles per
 * side, or more than 2^26 grid tiles over all slides and scales, is
 * ERR_UNSUPPORTED (here and in every call that takes slides).
 */
int32_t omniseg_workspace_bytes(const omniseg_plan* plan, const omniseg_slide* slides,
                                int32_t n_slides, const omniseg_pair* pairs,
                                int32_t n_pairs, int64_t* bytes);

/*
 * Segment n_slides slides for n_pairs (class, scale) pairs.
 *   packed     device weights from omniseg_pack_weights.
 *   slides     host array [n_slides] (1 <= n_slides <= 32).
 *   pairs      host array [n_pairs] (1 <= n_pairs); each pair unique.
 *   outs       host array [n_slides * n_pairs], slide-major: outs[i * n_pairs + p].
 *   workspace  device, ws_bytes >= omniseg_workspace_bytes, 256-byte aligned.
 * All slides share one tile work list: every kept tile of every slide and
 * scale runs through the backbone in batches of B = batch_tiles list
 * positions; the head runs once per (tile, pair at the tile's scale).  The
 * output rows of each tile row of each (slide, scale) grid are stitched
 * right after the batch that holds the last kept tile covering them, so
 * the logit store may be a ring (logit_ring_tiles).  The number of kept
 * tiles stays on the device: the backbone batches are launched for every
 * grid tile and those past the kept-tile count return at once.  Everything
 * is enqueued on `stream` and the call returns without waiting for it
 * (unless profiling is on, see omniseg_set_profiling); outputs are valid
 * once the stream has completed the work.
 */
int32_t omniseg_segment_slide(const omniseg_plan* plan, const void* packed,
                              const omniseg_slide* slides, int32_t n_slides,
                              const omniseg_pair* pairs, int32_t n_pairs,
                              const omniseg_output* outs, void* workspace,
                              int64_t ws_bytes, omniseg_stream stream);

/* Regions of the workspace after omniseg_segment_slide, for inspection. */
#define OMNISEG_REGION_PAD 0        /* int32[4] per slide: pad colour (index = slide) */
#define OMNISEG_REGION_PYRAMID 1    /* uint16[E_y][E_x][4] box sums of (slide, scale slot);
                                       index = slide * n_scales + slot; empty for 40x */
#define OMNISEG_REGION_TISSUE 2     /* uint8[H_c][W_c] tissue map of a slide (index = slide) */
#define OMNISEG_REGION_TILE_COUNT 3 /* int32: number of kept tiles */
#define OMNISEG_REGION_TILE_LIST 4  /* int32[max_tiles][4]: (slide, slot, jy, jx) in list order */
#define OMNISEG_REGION_TILE_INDEX 5 /* int32 per grid tile of (slide, slot): list index or -1,
                                       row-major (jy, jx); index = slide * n_scales + slot */
#define OMNISEG_REGION_TILE_LOGITS 6 /* float[slots][max_pairs_per_scale][T][T]: the logit
                                         store; the kept tile at list position p is in slot
                                         p % slots (slots = bytes / (max_pairs_per_scale T^2 4));
                                         with logit_ring_tiles = 0 every kept tile's slot is p */
#define OMNISEG_REGION_TISSUE_GRAY 7  /* uint8[H_c][W_c]: the median-blurred gray map of a slide
                                         (OMNISEG_TISSUE_OTSU; empty otherwise); index = slide */
#define OMNISEG_REGION_TISSUE_STATS 8 /* int32[4] of a slide (OMNISEG_TISSUE_OTSU; empty otherwise):
                                         Otsu threshold (-1: one-valued map), tissue components,
                                         components kept, error flag (1: the component labelling
                                         stopped at its iteration bound; a bound no input reaches,
                                         kept so every kernel ends); index = slide */
/*
 * Byte offset and size of one region inside the workspace for these slides
 * and pairs (host arrays); the layout depends only on the arguments.
 */
int32_t omniseg_workspace_region(const omniseg_plan* plan, const omniseg_slide* slides,
                                 int32_t n_slides, const omniseg_pair* pairs,
                                 int32_t n_pairs, int32_t region, int32_t index,
                                 int64_t* offset, int64_t* bytes);

/*
 * Stand-alone overlap-weighted stitch of one (slide, class, scale) plane
 * (Section 2.2 overlap tiling; Section 2.3 merge).
 *   tile_logits  device float[n_tiles][tile][tile], tile i at grid position
 *                tile_yx[2 i], tile_yx[2 i + 1] (rows, columns of tiles).
 *   tile_yx      device int32[n_tiles][2]: distinct grid positions inside the
 *                ceil-grid of (height, width).
 *   mask, logit  outputs as in omniseg_output (logit may be NULL).
 *   workspace    device, >= omniseg_stitch_workspace_bytes bytes.
 * For each pixel p: N = sum_t w_t(p) l_t, D = sum_t w_t(p) over the tiles
 * covering p, w(i, j) = r(i) r(j), r(i) = min(i + 1, T - i); the logit is N / D
 * (0 where D = 0), the mask is N > 0.  N is accumulated in FP32 with
 * compensated (Neumaier) summation over the covering tiles in (jy, jx) order;
 * D is an exact integer.
 * vote_threshold > 0 selects the majority vote of Section 2.2 instead: the
 * mask is (number of covering tiles whose logit is > 0) >= vote_threshold,
 * and the logit plane receives that count.  0 = the weighted mean.
 * Grids above 2^30 tile positions are ERR_UNSUPPORTED.
 */
int32_t omniseg_stitch_workspace_bytes(int32_t tile, int32_t stride, int32_t height,
                                       int32_t width, int64_t* bytes);
int32_t omniseg_stitch_tiles(int32_t tile, int32_t stride, int32_t height, int32_t width,
                             int32_t vote_threshold, const float* tile_logits, const int32_t* tile_yx,
                             int32_t n_tiles, uint8_t* mask, int64_t mask_pitch,
                             float* logit, int64_t logit_pitch, void* workspace,
                             int64_t ws_bytes, omniseg_stream stream);
/*
 * omniseg_stitch_tiles for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, outputs and arithmetic, without the
 * workspace.  The tile-index grid lives in a library-owned device array of
 * 2^20 int32 positions (4 MiB per device, held until the process ends), so
 * grids of more than 2^20 tile positions are ERR_UNSUPPORTED.  Allocates
 * nothing: the first call on a device looks the array up
 * (hipGetSymbolAddress).  Every call on one device shares that device's
 * array: calls that overlap on a device (other streams, other threads) race
 * and must be serialised by the caller.  Each call rewrites the whole grid
 * it uses before reading it.
 */
int32_t omniseg_stitch_tiles_noalloc(int32_t tile, int32_t stride, int32_t height, int32_t width,
                                     int32_t vote_threshold, const float* tile_logits,
                                     const int32_t* tile_yx, int32_t n_tiles, uint8_t* mask,
                                     int64_t mask_pitch, float* logit, int64_t logit_pitch,
                                     omniseg_stream stream);

/*
 * Merge of each class's result to the 40x base (Section 2.3: one merged 40x
 * prediction per tissue type; Section 1: each tissue type has its own best
 * magnification, e.g. 5x glomeruli, 10x tubules, 40x capillaries).
 * height, width: the 40x slide, in [1, 2^20].  Plane i has scale k =
 * scale_log2 in [0, 3] and size ceil(height / 2^k) x ceil(width / 2^k):
 *   OMNISEG_UPSAMPLE_NEAREST   out(y, x) = mask(y >> k, x >> k) != 0
 *   OMNISEG_UPSAMPLE_BILINEAR  out(y, x) = bilinear(logit)(y, x) > 0, sampling
 *                              at max(0, (y + 0.5) / 2^k - 0.5) (the same on
 *                              x) with the upper neighbour clamped to the
 *                              plane; weights are exact, the sum is FP32
 * mask: device uint8, logit: device float (the one the mode reads; the other
 * may be NULL), rows `pitch` elements apart; out: device uint8 [height]
 * [width], rows out_pitch bytes apart.  1 <= n_planes <= 16.
 */
#define OMNISEG_UPSAMPLE_NEAREST 0
#define OMNISEG_UPSAMPLE_BILINEAR 1
typedef struct omniseg_base_plane {
  const uint8_t* mask;
  const float* logit;
  int64_t pitch;
  int32_t scale_log2;
  int32_t mode;
  uint8_t* out;
  int64_t out_pitch;
} omniseg_base_plane;
int32_t omniseg_merge_to_base(int32_t height, int32_t width, const omniseg_base_plane* planes,
                              int32_t n_planes, omniseg_stream stream);

/*
 * Colour mapping of the merged results on the 40x slide (Section 2.3: the
 * tissue types are stained in different colours on the WSI, and the 10x
 * result is a resize of the 40x one).  For each pixel, every class whose
 * mask is on blends its colour in class order:
 *   out = (out * (256 - alpha) + rgb * alpha + 128) >> 8  per channel,
 * starting from the slide's pixel (exact integers).  The mask of class i is
 * read at its scale: mask(y >> k, x >> k), k = scale_log2 in [0, 3] (k = 0
 * for a merged 40x mask).  out: device uint8 HWC [height][width][3], rows
 * out_pitch bytes apart (it may be the slide itself).  out10: NULL, or
 * device uint8 HWC [ceil(height / 4)][ceil(width / 4)][3] receiving the
 * rounded (half up) mean of each 4 x 4 block of `out` inside the slide.
 * 0 <= n_classes <= 16; alpha in [0, 256].
 */
typedef struct omniseg_overlay_class {
  const uint8_t* mask;
  int64_t pitch;
  int32_t scale_log2;
  int32_t alpha;
  uint8_t rgb[4]; /* R, G, B, unused */
} omniseg_overlay_class;
int32_t omniseg_overlay(const omniseg_slide* slide, const omniseg_overlay_class* classes,
                        int32_t n_classes, uint8_t* out, int64_t out_pitch, uint8_t* out10,
                        int64_t out10_pitch, omniseg_stream stream);

/*
 * Stand-alone 3x3 convolution of the backbone (verification and reuse).
 * Tensors are NHWC over n images, channels padded to a multiple of 32 with
 * zeros in the padding; element type FP32 or BF16 (precision).  Zero padding
 * of 1 at the image border.  H x W is the output size (multiples of 8).
 *   OMNISEG_CONV_RELU        y = ReLU(conv(x0) + b)
 *   OMNISEG_CONV_RES_RELU    y = ReLU(conv(x0) + b + x0)          (cin = cout)
 *   OMNISEG_CONV_POOL_RELU   y = ReLU(conv(maxpool2x2(x0)) + b)   (x0 is 2H x 2W)
 *   OMNISEG_CONV_UPCAT_RELU  y = ReLU(conv([up2(x0); x1]) + b)    (x0: H/2 x W/2 with cu
 *                            channels, x1: H x W with cin - cu channels)
 *   OMNISEG_CONV_DGRAD       y = data gradient of conv: the 3x3 conv of x0 (cout
 *                            channels) with the weights transposed and flipped;
 *                            y has cin channels (concat padding when cu < cin)
 *   OMNISEG_CONV_DGRAD_RES_MASK  y = (DGRAD(x0) + x0) where aux > 0, else 0 (cin = cout)
 * weights: device FP32 canonical W[cout][cin][3][3]; bias: device FP32 [cout]
 * (ignored by the DGRAD modes).  config: a tile configuration id (see
 * omniseg_conv_config) valid for the shape, or -1 for the default; ERR_ARG
 * if it does not fit H, W and the output channels.
 * y_pool: NULL, or (mode OMNISEG_CONV_RES_RELU, BF16, with a row-reuse
 * configuration or -1) device [n][H/2][W/2][pad32(cout)] that receives the
 * 2x2 max-pool of y as well -- the encoder's next input, written by the same
 * kernel (ERR_UNSUPPORTED for FP32, ERR_ARG for other modes or
 * configurations).
 * workspace: device, >= omniseg_conv3x3_workspace_bytes.
 */
#define OMNISEG_CONV_RELU 0
#define OMNISEG_CONV_RES_RELU 1
#define OMNISEG_CONV_POOL_RELU 2
#define OMNISEG_CONV_UPCAT_RELU 3
#define OMNISEG_CONV_DGRAD 4
#define OMNISEG_CONV_DGRAD_RES_MASK 5
int32_t omniseg_conv3x3_workspace_bytes(int32_t precision, int32_t cin, int32_t cu, int32_t cout,
                                        int64_t* bytes);
int32_t omniseg_conv3x3(int32_t precision, int32_t mode, int32_t n, int32_t height, int32_t width,
                        int32_t cin, int32_t cu, int32_t cout, const float* weights,
                        const float* bias, const void* x0, const void* x1, const void* aux, void* y,
                        void* y_pool, int32_t config, void* workspace, int64_t ws_bytes,
                        omniseg_stream stream);
/*
 * Weight gradient of one stand-alone 3x3 convolution (verification of the
 * backward's kernels): dW[o][c][i][j] = sum over images and output pixels of
 * dY[o][y][x] * Xin[c][y + i - 1][x + j - 1], Xin taken as 0 outside the
 * image, where Xin is the conv's input as omniseg_conv3x3 forms it for
 * `mode`: OMNISEG_CONV_RELU (x0), OMNISEG_CONV_POOL_RELU (maxpool2x2 of the
 * 2H x 2W x0) or OMNISEG_CONV_UPCAT_RELU ([up2(x0); x1], cu < cin).
 *   precision  OMNISEG_FP32 or OMNISEG_BF16: the element type of x0, x1
 *              and dy (BF16 runs on BF16 MFMA with FP32 accumulation).
 *   dy         device NHWC [n][H][W][pad32(cout)] (zeros in the padding).
 *   dw         device FP32, canonical [cout][cin][3][3].
 * The pixel sum is split over fixed slots and reduced in a fixed order
 * (deterministic).  H, W multiples of 8 in [8, 4096]; n >= 1.
 * workspace: device, >= omniseg_conv3x3_wgrad_workspace_bytes.
 */
int32_t omniseg_conv3x3_wgrad_workspace_bytes(int32_t n, int32_t height, int32_t width, int32_t cin,
                                              int32_t cu, int32_t cout, int64_t* bytes);
int32_t omniseg_conv3x3_wgrad(int32_t precision, int32_t mode, int32_t n, int32_t height, int32_t width,
                              int32_t cin, int32_t cu, int32_t cout, const void* x0, const void* x1,
                              const void* dy, float* dw, void* workspace, int64_t ws_bytes,
                              omniseg_stream stream);
/*
 * FP8 form of omniseg_conv3x3 (modes RELU, RES_RELU, POOL_RELU, UPCAT_RELU;
 * the FP8 backbone described at omniseg_pack_weights_fp8).  x0 (and x1 for
 * UPCAT) hold E4M3 codes (uint8, NHWC, channels padded to 32) of
 * non-negative activations whose channel c has the power-of-two scale
 * in_scale[c] (device float[cin], real channel order: for UPCAT the cu
 * upsampled channels, then the skip channels); y receives the E4M3 codes of
 * the result with the power-of-two channel scales out_scale (device
 * float[cout]).  The weights are quantised as omniseg_pack_weights_fp8 does,
 * with in_scale folded into their columns; RES_RELU (cin == cout) decodes
 * the residual with in_scale.  y_pool: NULL, or (RES_RELU) the codes of the
 * 2x2 max-pool of y, [n][H/2][W/2][pad32(cout)], same scales.  config: a
 * configuration whose precisions include OMNISEG_FP8, or -1.  workspace:
 * device, 256-byte aligned, >= omniseg_conv3x3_fp8_workspace_bytes.
 */
int32_t omniseg_conv3x3_fp8_workspace_bytes(int32_t cin, int32_t cu, int32_t cout, int64_t* bytes);
int32_t omniseg_conv3x3_fp8(int32_t mode, int32_t n, int32_t height, int32_t width, int32_t cin,
                            int32_t cu, int32_t cout, const float* weights, const float* bias,
                            const float* in_scale, const float* out_scale, const void* x0,
                            const void* x1, void* y, void* y_pool, int32_t config,
                            void* workspace, int64_t ws_bytes, omniseg_stream stream);

/*
 * ---- training: forward over a tile batch, BCE loss, hand-written backward ----
 *
 * A training step takes a batch of tiles of one slide (or region), runs the
 * backbone, controller and head on them, stitches each requested (class,
 * scale) plane from the batch tiles only, and compares it with a soft target
 * by binary cross-entropy over the pixels the batch covers.  The backward
 * pass returns dLoss/dweights in the canonical FP32 order.  U-Net levels are
 * checkpointed: the forward keeps each level's output (E_l, D_l), the
 * backward recomputes each level's first conv from its saved input.
 *
 * Planes of all pairs are concatenated in one flat array in pair order;
 * plane p holds ceil(height / 2^k) x ceil(width / 2^k) values (k = the
 * pair's scale), rows contiguous, starting at omniseg_plane_offsets()[p].
 */
typedef struct omniseg_tile {
  int32_t scale; /* scale slot */
  int32_t jy;    /* tile row in the slot's grid */
  int32_t jx;    /* tile column */
} omniseg_tile;

#define OMNISEG_MAX_TRAIN_TILES 256

/* offsets[n_pairs + 1] (host): start of each flat plane; offsets[n_pairs] =
 * total number of values. */
int32_t omniseg_plane_offsets(const omniseg_plan* plan, const omniseg_slide* slide,
                              const omniseg_pair* pairs, int32_t n_pairs, int64_t* offsets);
/* Workspace for omniseg_train_forward + omniseg_backward (the same buffer). */
int32_t omniseg_train_workspace_bytes(const omniseg_plan* plan, const omniseg_slide* slide,
                                      const omniseg_tile* tiles, int32_t n_tiles,
                                      const omniseg_pair* pairs, int32_t n_pairs,
                                      int64_t* bytes);
/*
 * Forward pass of a training batch (plan created with OMNISEG_FLAG_TRAINING).
 *   slide       host pointer to one slide (device pixels).
 *   tiles       host array [n_tiles], 1 <= n_tiles <= 256, distinct, inside
 *               the slot grids; no tissue filter is applied.
 *   logit       device float[offsets[n_pairs]]: stitched logits of the batch
 *               (0 where no batch tile covers the pixel).
 *   covered     device uint8[offsets[n_pairs]]: 1 where a batch tile covers.
 * The workspace keeps what omniseg_backward needs; do not modify it between
 * the two calls.
 */
int32_t omniseg_train_forward(const omniseg_plan* plan, const void* packed,
                              const omniseg_slide* slide, const omniseg_tile* tiles,
                              int32_t n_tiles, const omniseg_pair* pairs, int32_t n_pairs,
                              float* logit, uint8_t* covered, void* workspace, int64_t ws_bytes,
                              omniseg_stream stream);
/*
 * Backward pass after omniseg_train_forward with the same arguments.
 *   grad_logit    device float[offsets[n_pairs]]: dLoss/dlogit (0 where uncovered).
 *   grad_weights  device float[omniseg_weight_count]: overwritten with
 *                 dLoss/dweights in canonical order.
 * Deterministic: every reduction sums in a fixed order.
 */
int32_t omniseg_backward(const omniseg_plan* plan, const void* packed, const omniseg_slide* slide,
                         const omniseg_tile* tiles, int32_t n_tiles, const omniseg_pair* pairs,
                         int32_t n_pairs, const float* grad_logit, float* grad_weights,
                         void* workspace, int64_t ws_bytes, omniseg_stream stream);
/*
 * Mean binary cross-entropy with logits over the entries where valid != 0:
 * loss = sum(max(x, 0) - y x + log1p(exp(-|x|))) / count, accumulated in
 * FP64 with a fixed-order reduction; grad (device float[n], may be NULL) =
 * (sigmoid(x) - y) / count where valid, else 0.  loss: device double.
 * workspace: device, >= 16384 bytes.
 */
int32_t omniseg_bce_loss(const float* logit, const float* target, const uint8_t* valid, int64_t n,
                         double* loss, float* grad, void* workspace, int64_t ws_bytes,
                         omniseg_stream stream);

/*
 * Per-launch profiling.  With profiling enabled, omniseg_segment_slide
 * records a pair of HIP events around every kernel launch on the call's
 * stream, plus the launch's algorithmic work: FLOPs of the arithmetic the
 * method defines (2 per multiply-add, real channel counts, no padding) and
 * the HBM bytes the step must move at minimum.  Records accumulate over
 * profiled calls; omniseg_read_profile waits for their events and returns all
 * of them (again on a repeated read), and the next profiled call after a read
 * starts a new list, so several calls can run back to back and be read once.
 * Profiling creates HIP events lazily (two per launch, kept by the plan until
 * it is destroyed, so read the records before the list grows without bound)
 * and is off by default.  A profiled omniseg_segment_slide makes the same
 * launches as an unprofiled one, but waits for the stream once after the
 * tile list to read the kept-tile count and index grid, which make each
 * record's `tiles`, FLOPs and bytes exact (a batch past the count records 0
 * tiles and no work); profiled calls are never captured in a graph.
 */
#define OMNISEG_STAGE_PREP 0       /* pad colour, pyramid, tissue map, tile list */
#define OMNISEG_STAGE_FIRST_CONV 1 /* encoder level 0, first conv (3 -> C_0)     */
#define OMNISEG_STAGE_ENC_A 2      /* encoder first conv (with fused 2x2 max-pool) */
#define OMNISEG_STAGE_ENC_B 3      /* encoder second conv (+ residual)          */
#define OMNISEG_STAGE_DEC_A 4      /* decoder first conv (fused upsample+concat) */
#define OMNISEG_STAGE_DEC_B 5      /* decoder second conv (+ residual)          */
#define OMNISEG_STAGE_GAP_CTRL 6   /* bottleneck mean and controller            */
#define OMNISEG_STAGE_HEAD 7       /* precls and dynamic head                   */
#define OMNISEG_STAGE_STITCH 8     /* stitch: of one plane (omniseg_stitch_tiles), or of the
                                      tile rows one backbone batch completed (segment_slide) */

typedef struct omniseg_launch_record {
  int32_t stage;  /* OMNISEG_STAGE_* */
  int32_t level;  /* U-Net level, or -1 */
  int32_t tiles;  /* tiles the launch processes (0 if not tile-based) */
  int32_t precision;
  int32_t config; /* conv tile configuration (see omniseg_conv_config), or -1 */
  int32_t reserved;
  double flops;   /* algorithmic FLOPs */
  double bytes;   /* algorithmic HBM bytes */
  double ms;      /* elapsed time between the events around the launch */
} omniseg_launch_record;

int32_t omniseg_set_profiling(omniseg_plan* plan, int32_t enable);
/* Shape of conv tile configuration `config`: pixel block by x bx, bn output
 * channels per workgroup, wm x wn waves; *precisions gets bit p set for each
 * precision p (OMNISEG_FP32, OMNISEG_BF16, OMNISEG_FP8) the configuration
 * runs at.
 * Configurations 0..OMNISEG_CONV_CONFIGS-1 exist; ERR_ARG for any other id.
 * 0-5 run at FP32 and BF16; 6-9 (row-reuse forms) at BF16 and FP8; 10 (the
 * eight-wave row-reuse form), 11 (the large-block row-reuse form: 32 x 16
 * pixels x 64 channels, double-buffered direct-to-LDS staging, one workgroup
 * per CU) and 12 (11 as a persistent launch: one workgroup per CU walks the
 * blocks, the next block's first load and this block's epilogue overlapped;
 * the max-pooling loader runs as 10) at BF16 only.  Every configuration sums
 * the taps of a chunk in the same order, so 6-12 give bit-identical BF16
 * results.  Without a configuration (-1) a BF16 conv takes 12 where it fits
 * and the layer has other than 64 input channels, else 10. */
#define OMNISEG_CONV_CONFIGS 13
int32_t omniseg_conv_config(int32_t config, int32_t* by, int32_t* bx, int32_t* bn, int32_t* wm,
                            int32_t* wn, int32_t* precisions);
/*
 * Autotune the conv tile configuration of every backbone layer for these
 * slides and pairs: each valid configuration runs on the plan's batch shape
 * in the workspace (whose contents it overwrites), once untimed and five
 * times timed by HIP events, and the fastest is kept in the plan for later
 * omniseg_segment_slide calls.  Waits
 * for the stream.  Same arguments as omniseg_segment_slide without outputs.
 */
int32_t omniseg_autotune(omniseg_plan* plan, const void* packed, const omniseg_slide* slides,
                         int32_t n_slides, const omniseg_pair* pairs, int32_t n_pairs,
                         void* workspace, int64_t ws_bytes, omniseg_stream stream);
/*
 * The conv tile configuration of one backbone layer.  stage: 0 = encoder
 * conv_a, 1 = encoder residual conv, 2 = decoder conv_a (upsample + concat),
 * 3 = decoder residual conv; level 0 .. levels - 1.  omniseg_autotune sets
 * them; omniseg_set_conv_tuning pins one (config -1 = the default), for
 * instance to repeat a tuned table in another process.  A configuration that
 * is not valid for the layer's shape and precision is ignored when the layer
 * runs (the default runs instead; an encoder residual conv that also writes
 * the pooled copy takes the first valid row-reuse configuration).  Host-only,
 * no GPU work.  ERR_ARG for a NULL plan or output, or a stage, level or
 * config out of range.
 */
int32_t omniseg_set_conv_tuning(omniseg_plan* plan, int32_t stage, int32_t level, int32_t config);
int32_t omniseg_get_conv_tuning(const omniseg_plan* plan, int32_t stage, int32_t level, int32_t* config);
/* Waits for the last profiled call's events; copies min(cap, n) records to
 * recs (host array) and the total number of records to *n. */
int32_t omniseg_read_profile(omniseg_plan* plan, omniseg_launch_record* recs, int32_t cap,
                             int32_t* n);

#ifdef __cplusplus
}
#endif

#endif /* OMNISEG_H */

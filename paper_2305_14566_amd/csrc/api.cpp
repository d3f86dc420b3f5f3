// C ABI of the omniseg library: plan, validation, workspace layout and the
// orchestration of the slide-wise segmentation on one HIP stream.
//
// Validation runs entirely on the host before the first HIP call, so an
// invalid call launches nothing and writes nothing.
#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "plan.h"

using namespace omniseg;

namespace omniseg {

namespace {
thread_local std::string g_last_error;
}

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

const char* last_error_text() { return g_last_error.c_str(); }

}  // namespace omniseg

namespace {

// ---------------------------------------------------------------------------
// workspace layout of one segment call
// ---------------------------------------------------------------------------

struct Layout {
  int n_slides = 0;
  int S = 0;
  int kmax = 0, kc = 0;
  bool need_fg = false;
  ScaleGeom geom[OMNISEG_MAX_SLIDES][OMNISEG_MAX_SCALES];
  int Hc[OMNISEG_MAX_SLIDES], Wc[OMNISEG_MAX_SLIDES];
  TileGroups groups;
  int total_tiles = 0;
  int ring = 0;       // slots of the tile-logit store (kept tile p in slot p % ring)
  bool resident = false;  // one slot per grid tile: no slot is ever reused
  int batch = 0;
  int n_batches = 0;  // batches of `batch` list positions covering every grid tile
  int n_units = 0;    // streamed stitch units (one per tile row of each group)
  int64_t n_items = 0;
  std::vector<StreamGroup> sgroups;  // host copy of the group table (pointers filled per call)
  SlotTable slots;
  int max_slots = 0;
  int pair_slot[256];  // slot index of each pair within its scale
  int64_t off_tab = 0, off_pad[OMNISEG_MAX_SLIDES], off_pyr[OMNISEG_MAX_SLIDES][OMNISEG_MAX_SCALES],
          off_fg[OMNISEG_MAX_SLIDES];
  int64_t sz_pyr[OMNISEG_MAX_SLIDES][OMNISEG_MAX_SCALES], sz_fg[OMNISEG_MAX_SLIDES];
  // Otsu tissue detection: per slide the blurred gray map and four stats;
  // shared scratch for the unblurred map, histogram, labels and areas
  bool otsu = false;
  int64_t off_tgray[OMNISEG_MAX_SLIDES], off_tstats[OMNISEG_MAX_SLIDES];
  int64_t off_ttmp = -1, off_thist = -1, off_tlabel = -1, off_tarea = -1;
  int64_t off_index = 0, off_list = 0, off_count = 0, off_pre = 0;
  int64_t off_sgroups = 0, off_splanes = 0, off_units = 0, off_bfirst = 0;
  int n_planes = 0;
  int64_t off_E[8], off_A = 0, off_g = 0, off_theta = 0, off_logits = 0;
  int64_t sz_E[8], sz_A = 0, sz_logits = 0;
  int64_t off_P = 0, sz_P = 0;  // pooled encoder output (row-reuse precisions)
  int64_t total = 0;
};

// The conv kernels address one image's input with 32-bit byte offsets.
bool per_image_bytes_too_big(int mode, int H, int W, int cin, int precision) {
  const int64_t es = precision == OMNISEG_FP32 ? 4 : precision == OMNISEG_BF16 ? 2 : 1;
  const int64_t px = (int64_t)H * W * (mode == OMNISEG_CONV_POOL_RELU ? 4 : 1);
  return px * ((cin + 31) / 32 * 32) * es >= (1LL << 31);
}

// Tile stride of scale slot si (scale_stride[si], 0 = the common stride).
int stride_of(const omniseg_config& c, int si) { return c.scale_stride[si] > 0 ? c.scale_stride[si] : c.stride; }

int32_t validate_config(const omniseg_config* c) {
  if (!c) return fail(OMNISEG_ERR_ARG, "config is NULL");
  if (c->abi_version != OMNISEG_ABI_VERSION)
    return fail(OMNISEG_ERR_ARG, "abi_version %d, library has %d", c->abi_version, OMNISEG_ABI_VERSION);
  if (c->base_channels < 1 || c->base_channels > 128)
    return fail(OMNISEG_ERR_ARG, "base_channels %d outside [1, 128]", c->base_channels);
  if (c->levels < 1 || c->levels > 7) return fail(OMNISEG_ERR_ARG, "levels %d outside [1, 7]", c->levels);
  if (c->head_out != 1 && c->head_out != 2) return fail(OMNISEG_ERR_ARG, "head_out must be 1 or 2");
  if (c->n_classes < 1 || c->n_classes > OMNISEG_MAX_CLASSES)
    return fail(OMNISEG_ERR_ARG, "n_classes %d outside [1, %d]", c->n_classes, OMNISEG_MAX_CLASSES);
  if (c->n_scales < 1 || c->n_scales > OMNISEG_MAX_SCALES)
    return fail(OMNISEG_ERR_ARG, "n_scales %d outside [1, %d]", c->n_scales, OMNISEG_MAX_SCALES);
  for (int i = 0; i < c->n_scales; ++i)
    if (c->scale_log2[i] < 0 || c->scale_log2[i] > 3)
      return fail(OMNISEG_ERR_ARG, "scale_log2[%d] = %d outside [0, 3]", i, c->scale_log2[i]);
  if (c->tile < 16 || c->tile > 512 || c->tile % 16)
    return fail(OMNISEG_ERR_ARG, "tile %d must be a multiple of 16 in [16, 512]", c->tile);
  if (c->stride < 1 || c->stride > c->tile)
    return fail(OMNISEG_ERR_ARG, "stride %d outside [1, tile]", c->stride);
  for (int i = 0; i < c->n_scales; ++i) {
    for (int j = 0; j < i; ++j)
      if (c->scale_log2[j] == c->scale_log2[i])
        return fail(OMNISEG_ERR_ARG, "scale_log2[%d] repeats scale_log2[%d]", i, j);
    if (c->scale_stride[i] < 0 || c->scale_stride[i] > c->tile)
      return fail(OMNISEG_ERR_ARG, "scale_stride[%d] = %d outside [0, tile]", i, c->scale_stride[i]);
  }
  if (c->merge != OMNISEG_MERGE_RAMP && c->merge != OMNISEG_MERGE_VOTE)
    return fail(OMNISEG_ERR_ARG, "unknown merge %d", c->merge);
  if (c->merge == OMNISEG_MERGE_VOTE)
    for (int i = 0; i < c->n_scales; ++i) {
      const int per = ceil_div(c->tile, stride_of(*c, i));
      if (c->vote_threshold[i] < 1 || c->vote_threshold[i] > per * per)
        return fail(OMNISEG_ERR_ARG, "vote_threshold[%d] = %d outside [1, %d] (most tiles covering a pixel)", i,
                    c->vote_threshold[i], per * per);
    }
  if (c->flags & OMNISEG_FLAG_TRAINING) {
    if (c->merge != OMNISEG_MERGE_RAMP)
      return fail(OMNISEG_ERR_UNSUPPORTED, "training plans merge with the ramp average only");
    for (int i = 0; i < c->n_scales; ++i)
      if (stride_of(*c, i) != c->stride)
        return fail(OMNISEG_ERR_UNSUPPORTED, "training plans use one stride for every scale");
  }
  const int deep = c->tile >> (c->levels - 1);
  if ((c->tile % (1 << (c->levels - 1))) || deep < 8 || deep % 8)
    return fail(OMNISEG_ERR_UNSUPPORTED, "tile / 2^(levels-1) = %d must be a multiple of 8", deep);
  if (c->fg_filter != 0 && c->fg_filter != 1) return fail(OMNISEG_ERR_ARG, "fg_filter must be 0 or 1");
  if (c->mask_and_fg != 0 && c->mask_and_fg != 1) return fail(OMNISEG_ERR_ARG, "mask_and_fg must be 0 or 1");
  if (c->fg_threshold < 1 || c->fg_threshold > 255)
    return fail(OMNISEG_ERR_ARG, "fg_threshold %d outside [1, 255]", c->fg_threshold);
  if (c->precision != OMNISEG_FP32 && c->precision != OMNISEG_BF16 && c->precision != OMNISEG_FP8)
    return fail(OMNISEG_ERR_UNSUPPORTED, "unknown precision %d", c->precision);
  if (c->precision == OMNISEG_FP8) {
    if (c->flags & OMNISEG_FLAG_TRAINING) return fail(OMNISEG_ERR_UNSUPPORTED, "FP8 plans are inference only");
    if (deep % 16) return fail(OMNISEG_ERR_UNSUPPORTED, "FP8 needs tile / 2^(levels-1) = %d a multiple of 16", deep);
  }
  if (c->flags & ~(OMNISEG_FLAG_EMIT_LOGITS | OMNISEG_FLAG_TRAINING | OMNISEG_FLAG_GRAPH))
    return fail(OMNISEG_ERR_ARG, "unknown flags 0x%x", c->flags);
  if (c->batch_tiles < 0 || c->batch_tiles > 65536)
    return fail(OMNISEG_ERR_ARG, "batch_tiles %d outside [0, 65536]", c->batch_tiles);
  if (c->logit_ring_tiles < 0) return fail(OMNISEG_ERR_ARG, "logit_ring_tiles %d < 0", c->logit_ring_tiles);
  if (c->tissue_method != OMNISEG_TISSUE_GRAY && c->tissue_method != OMNISEG_TISSUE_OTSU)
    return fail(OMNISEG_ERR_ARG, "unknown tissue_method %d", c->tissue_method);
  if (c->tissue_method == OMNISEG_TISSUE_OTSU) {
    if (c->median_kernel < 1 || c->median_kernel > 255 || c->median_kernel % 2 == 0)
      return fail(OMNISEG_ERR_ARG, "median_kernel %d must be odd in [1, 255]", c->median_kernel);
    if (c->min_tissue_area < 0) return fail(OMNISEG_ERR_ARG, "min_tissue_area %d < 0", c->min_tissue_area);
  }
  const int64_t G = (int64_t)c->base_channels << (c->levels - 1);
  if (G > 4096) return fail(OMNISEG_ERR_UNSUPPORTED, "bottleneck width %lld > 4096", (long long)G);
  return OMNISEG_OK;
}

int32_t validate_call(const omniseg_plan* plan, const omniseg_slide* slides, int32_t n_slides,
                      const omniseg_pair* pairs, int32_t n_pairs, Layout& lay) {
  if (!plan) return fail(OMNISEG_ERR_ARG, "plan is NULL");
  if (!slides) return fail(OMNISEG_ERR_ARG, "slides is NULL");
  if (!pairs) return fail(OMNISEG_ERR_ARG, "pairs is NULL");
  if (n_slides < 1 || n_slides > OMNISEG_MAX_SLIDES)
    return fail(OMNISEG_ERR_ARG, "n_slides %d outside [1, %d]", n_slides, OMNISEG_MAX_SLIDES);
  const omniseg_config& c = plan->cfg;
  if (n_pairs < 1 || n_pairs > c.n_classes * c.n_scales)
    return fail(OMNISEG_ERR_ARG, "n_pairs %d outside [1, %d]", n_pairs, c.n_classes * c.n_scales);
  for (int i = 0; i < n_slides; ++i) {
    const omniseg_slide& s = slides[i];
    if (!s.rgb) return fail(OMNISEG_ERR_ARG, "slide %d: rgb is NULL", i);
    if (s.height < 2 || s.width < 2) return fail(OMNISEG_ERR_ARG, "slide %d: size %dx%d below 2x2", i, s.height, s.width);
    if (s.height > (1 << 20) || s.width > (1 << 20))
      return fail(OMNISEG_ERR_UNSUPPORTED, "slide %d: side above 2^20", i);
    if (s.row_pitch < 3LL * s.width) return fail(OMNISEG_ERR_ARG, "slide %d: row_pitch %lld < 3*width", i, (long long)s.row_pitch);
  }
  // tile grids: the group table keeps 16-bit grid sides, the tile list int32 indices
  int64_t grid_tiles = 0;
  for (int i = 0; i < n_slides; ++i)
    for (int si = 0; si < c.n_scales; ++si) {
      const int k = c.scale_log2[si];
      const int64_t ny = grid_count(ceil_div(slides[i].height, 1 << k), c.tile, stride_of(c, si));
      const int64_t nx = grid_count(ceil_div(slides[i].width, 1 << k), c.tile, stride_of(c, si));
      if (ny > 32767 || nx > 32767)
        return fail(OMNISEG_ERR_UNSUPPORTED, "slide %d, scale %d: tile grid %lldx%lld above 32767 per side", i, si,
                    (long long)ny, (long long)nx);
      grid_tiles += ny * nx;
    }
  if (grid_tiles > (1LL << 26))
    return fail(OMNISEG_ERR_UNSUPPORTED, "%lld grid tiles above 2^26", (long long)grid_tiles);
  if (c.tissue_method == OMNISEG_TISSUE_OTSU && (c.fg_filter || c.mask_and_fg)) {
    int kc = 0;
    for (int si = 0; si < c.n_scales; ++si) kc = std::max(kc, c.scale_log2[si]);
    for (int i = 0; i < n_slides; ++i) {
      const int64_t hc = ceil_div(slides[i].height, 1 << kc), wc = ceil_div(slides[i].width, 1 << kc);
      if (hc * wc >= (1LL << 28))
        return fail(OMNISEG_ERR_UNSUPPORTED, "slide %d: coarse map of %lld pixels above 2^28 - 1", i,
                    (long long)(hc * wc));
    }
  }
  bool seen[OMNISEG_MAX_CLASSES][OMNISEG_MAX_SCALES] = {};
  lay.S = c.n_scales;
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) lay.slots.n_slots[si] = 0;
  for (int p = 0; p < n_pairs; ++p) {
    const int cl = pairs[p].cls, sc = pairs[p].scale;
    if (cl < 0 || cl >= c.n_classes) return fail(OMNISEG_ERR_ARG, "pair %d: class %d outside [0, %d)", p, cl, c.n_classes);
    if (sc < 0 || sc >= c.n_scales) return fail(OMNISEG_ERR_ARG, "pair %d: scale %d outside [0, %d)", p, sc, c.n_scales);
    if (seen[cl][sc]) return fail(OMNISEG_ERR_ARG, "pair %d: (class %d, scale %d) repeated", p, cl, sc);
    seen[cl][sc] = true;
    lay.pair_slot[p] = lay.slots.n_slots[sc];
    lay.slots.cls[sc][lay.slots.n_slots[sc]++] = cl;
  }
  lay.max_slots = 0;
  for (int si = 0; si < c.n_scales; ++si) lay.max_slots = std::max(lay.max_slots, lay.slots.n_slots[si]);
  return OMNISEG_OK;
}

// BF16 and FP8 inference fuse the encoder's 2x2 max-pool into the residual
// conv that produces E_l (its row-reuse epilogue also writes the pooled
// tensor), so the next level's conv_a reads it with the plain loader.
bool fuse_pool(const omniseg_plan* plan) { return plan->cfg.precision != OMNISEG_FP32 && plan->L >= 2; }

// Conv configuration of an encoder residual conv that writes the pooled copy:
// the tuned one if it is a valid row-reuse configuration, else the first
// valid row-reuse configuration.
int pool_config(const omniseg_plan* plan, int level, int H, int W, int cout_p) {
  const int prec = plan->cfg.precision;
  const int t = plan->tune[1][level];
  if (t >= CONV_CFG_ROWS_16x16_64 && conv_config_valid(t, prec, H, W, cout_p)) return t;
  for (int c : {CONV_CFG_ROWS_16x16_64, CONV_CFG_ROWS_16x16_32, CONV_CFG_ROWS_32x16_32, CONV_CFG_ROWS_16x16_128})
    if (conv_config_valid(c, prec, H, W, cout_p)) return c;
  return -1;
}

void compute_layout(const omniseg_plan* plan, const omniseg_slide* slides, int32_t n_slides,
                    Layout& lay) {
  const omniseg_config& c = plan->cfg;
  const int T = c.tile;
  lay.n_slides = n_slides;
  lay.kmax = 0;
  for (int si = 0; si < c.n_scales; ++si) lay.kmax = std::max(lay.kmax, c.scale_log2[si]);
  lay.kc = lay.kmax;
  lay.need_fg = c.fg_filter || c.mask_and_fg;
  lay.otsu = lay.need_fg && c.tissue_method == OMNISEG_TISSUE_OTSU;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off += align256(std::max<int64_t>(bytes, 1));
    return o;
  };
  lay.off_tab = take((int64_t)n_slides * sizeof(SlideDev));
  lay.groups.n = 0;
  int tiles = 0;
  for (int i = 0; i < n_slides; ++i) {
    lay.off_pad[i] = take(16);
    for (int si = 0; si < c.n_scales; ++si) {
      const ScaleGeom g = make_geom(slides[i].height, slides[i].width, c.scale_log2[si], T, stride_of(c, si));
      lay.geom[i][si] = g;
      lay.sz_pyr[i][si] = g.k >= 1 ? (int64_t)g.Ey * g.Ex * 8 : 0;
      lay.off_pyr[i][si] = g.k >= 1 ? take(lay.sz_pyr[i][si]) : -1;
      const int gi = lay.groups.n++;
      lay.groups.base[gi] = tiles;
      lay.groups.ny[gi] = (short)g.ny;
      lay.groups.nx[gi] = (short)g.nx;
      lay.groups.s[gi] = (short)stride_of(c, si);
      lay.groups.slide[gi] = (char)i;
      lay.groups.slot[gi] = (char)si;
      lay.groups.k[gi] = (char)g.k;
      tiles += g.ny * g.nx;
    }
    lay.Hc[i] = ceil_div(slides[i].height, 1 << lay.kc);
    lay.Wc[i] = ceil_div(slides[i].width, 1 << lay.kc);
    lay.sz_fg[i] = lay.need_fg ? (int64_t)lay.Hc[i] * lay.Wc[i] : 0;
    lay.off_fg[i] = lay.need_fg ? take(lay.sz_fg[i]) : -1;
    lay.off_tgray[i] = lay.otsu ? take(lay.sz_fg[i]) : -1;
    lay.off_tstats[i] = lay.otsu ? take(16) : -1;
  }
  if (lay.otsu) {
    int64_t most = 0;
    for (int i = 0; i < n_slides; ++i) most = std::max(most, lay.sz_fg[i]);
    lay.off_ttmp = take(most);
    lay.off_thist = take(256 * 4);
    lay.off_tlabel = take(most * 4);
    lay.off_tarea = take(most * 4);
  }
  lay.groups.base[lay.groups.n] = tiles;
  lay.total_tiles = tiles;
  lay.off_index = take((int64_t)tiles * 4);
  lay.off_list = take((int64_t)tiles * 16);
  lay.off_count = take(4);
  lay.off_pre = take((int64_t)(tiles + 1) * 4);
  const int bt = c.batch_tiles > 0 ? c.batch_tiles : 256;
  lay.batch = std::min(bt, tiles);
  lay.n_batches = ceil_div(tiles, lay.batch);
  const int es = elem_size(c.precision);
  for (int l = 0; l < plan->L; ++l) {
    const int tl = T >> l;
    lay.sz_E[l] = (int64_t)lay.batch * tl * tl * plan->Cp[l] * es;
    lay.off_E[l] = take(lay.sz_E[l]);
  }
  lay.sz_A = (int64_t)lay.batch * T * T * plan->Cp[0] * es;
  lay.off_A = take(lay.sz_A);
  if (fuse_pool(plan)) {
    // the largest pooled encoder output is level 0's: (T/2)^2 pixels x C_0
    lay.sz_P = (int64_t)lay.batch * (T / 2) * (T / 2) * plan->Cp[0] * es;
    lay.off_P = take(lay.sz_P);
  }
  lay.off_g = take((int64_t)lay.batch * plan->Cp[plan->L - 1] * 4);
  lay.off_theta = take((int64_t)lay.batch * lay.max_slots * plan->P * 4);
  // Streamed stitch: one unit per tile row of each group.  A unit's covering
  // tiles start at tile row jlo (the first row reaching its first output
  // row) and end with its own row, at most (j + 1 - jlo) nx list positions;
  // it is stitched right after the batch that holds its last one, when at
  // most B - 1 later positions have been written.  A ring of at least
  // max (j + 1 - jlo) nx + B - 1 slots therefore still holds every tile
  // logit a unit reads.
  lay.sgroups.assign(lay.groups.n, StreamGroup());
  lay.n_units = 0;
  lay.n_items = 0;
  lay.n_planes = 0;
  int64_t need = 0;
  for (int gi = 0; gi < lay.groups.n; ++gi) {
    const int i = lay.groups.slide[gi], si = lay.groups.slot[gi];
    const ScaleGeom& g = lay.geom[i][si];
    const int ss = stride_of(c, si);
    StreamGroup& sg = lay.sgroups[gi];
    sg.grid_base = lay.groups.base[gi];
    sg.item_base = lay.n_items;
    sg.ny = g.ny;
    sg.nx = g.nx;
    sg.s = ss;
    sg.Hk = g.Hk;
    sg.Wk = g.Wk;
    sg.unit_base = lay.n_units;
    sg.nxc = ceil_div(g.Wk, kStitchCols);
    sg.plane_first = lay.n_planes;
    sg.n_planes = lay.slots.n_slots[si];
    sg.fg = nullptr;
    sg.fg_shift = lay.kc - g.k;
    sg.Hc = lay.Hc[i];
    sg.Wc = lay.Wc[i];
    sg.vote = c.merge == OMNISEG_MERGE_VOTE ? c.vote_threshold[si] : 0;
    lay.n_units += g.ny;
    lay.n_planes += sg.n_planes;
    const int64_t last_rows = g.Hk - (int64_t)(g.ny - 1) * ss;
    lay.n_items += (int64_t)sg.n_planes * sg.nxc *
                   ((int64_t)(g.ny - 1) * ceil_div(ss, kStitchRows) + (last_rows + kStitchRows - 1) / kStitchRows);
    for (int j = 0; j < g.ny; ++j) {
      const int y0 = j * ss;
      const int jlo = y0 < T ? 0 : (y0 - T) / ss + 1;
      need = std::max<int64_t>(need, (int64_t)(j + 1 - jlo) * g.nx);
    }
  }
  lay.off_sgroups = take((int64_t)lay.groups.n * sizeof(StreamGroup));
  lay.off_splanes = take((int64_t)std::max(1, lay.n_planes) * sizeof(StreamPlane));
  lay.off_units = take((int64_t)(lay.n_units + 1) * sizeof(StreamUnit));
  lay.off_bfirst = take((int64_t)(lay.n_batches + 1) * 4);
  const int64_t B = lay.batch;
  const int64_t ring_min = (need + B - 1 + B - 1) / B * B;
  if (c.logit_ring_tiles == 0 || ring_min >= tiles) {
    lay.resident = true;
    lay.ring = tiles;
  } else {
    lay.resident = false;
    lay.ring = (int)std::min<int64_t>(std::max<int64_t>(ring_min, ((int64_t)c.logit_ring_tiles + B - 1) / B * B),
                                      (int64_t)tiles);
    if (lay.ring >= tiles) lay.resident = true;
  }
  lay.sz_logits = (int64_t)lay.ring * lay.max_slots * T * T * 4;
  lay.off_logits = take(lay.sz_logits);
  lay.total = off;
}

// Conv layer view of a packed weight buffer (with the FP8 scale tables).
ConvLayer make_layer(const omniseg_plan* plan, const char* pk, const ConvDesc& d) {
  ConvLayer L;
  L.cin_p = d.cin_p;
  L.cu_p = d.cu_p;
  L.cout_p = d.cout_p;
  L.w = pk + d.pk_w;
  L.b = reinterpret_cast<const float*>(pk + d.pk_b);
  if (plan->cfg.precision == OMNISEG_FP8) {
    L.wscale = reinterpret_cast<const float*>(pk + d.pk_ws);
    L.rscale = reinterpret_cast<const float*>(pk + plan->pk_scale) + d.act_in;
    L.oinv = reinterpret_cast<const float*>(pk + plan->pk_iscale) + d.act_out;
  }
  return L;
}

// FP8 channel scales of the bottleneck E_{L-1} (GAP input) and of D_0 (head
// input); null for other precisions.
const float* fp8_scale_of(const omniseg_plan* plan, const char* pk, int kind, int level) {
  if (plan->cfg.precision != OMNISEG_FP8) return nullptr;
  return reinterpret_cast<const float*>(pk + plan->pk_scale) + plan->act_off[kind][level];
}

// Steps 1-2 of a call: slide table, pad colour, pyramid, tissue map, tile
// flags, the compacted tile list and its prefix counts.  Enqueues only: the
// kept-tile count stays on the device.
int32_t enqueue_tile_list(const omniseg_plan* plan, const omniseg_slide* slides, int32_t n_slides, const Layout& lay,
                          char* ws, hipStream_t sm, Prof& prof, SlideDev** tab_out) {
  const omniseg_config& c = plan->cfg;
  const int T = c.tile;
  plan->slide_tab.assign(n_slides, SlideDev());
  for (int i = 0; i < n_slides; ++i) {
    SlideDev& d = plan->slide_tab[i];
    d.rgb = slides[i].rgb;
    d.pitch = slides[i].row_pitch;
    d.H = slides[i].height;
    d.W = slides[i].width;
    d.pad = reinterpret_cast<const int32_t*>(ws + lay.off_pad[i]);
    for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) {
      d.pyr[si] = nullptr;
      d.pyr_ex[si] = 0;
      if (si < c.n_scales && lay.off_pyr[i][si] >= 0) {
        d.pyr[si] = reinterpret_cast<const uint16_t*>(ws + lay.off_pyr[i][si]);
        d.pyr_ex[si] = lay.geom[i][si].Ex;
      }
    }
    d.fg = lay.need_fg ? reinterpret_cast<const uint8_t*>(ws + lay.off_fg[i]) : nullptr;
    d.Hc = lay.Hc[i];
    d.Wc = lay.Wc[i];
  }
  SlideDev* tab_dev = reinterpret_cast<SlideDev*>(ws + lay.off_tab);
  *tab_out = tab_dev;
  HIP_TRY(launch_put(tab_dev, plan->slide_tab.data(), (int64_t)sizeof(SlideDev) * n_slides, sm));

  double prep_bytes = 0.0;
  for (int i = 0; i < n_slides; ++i) {
    prep_bytes += 3.0 * slides[i].height * slides[i].width;
    for (int si = 0; si < c.n_scales; ++si)
      if (lay.geom[i][si].k >= 1) prep_bytes += 6.0 * lay.geom[i][si].Ey * lay.geom[i][si].Ex;
    prep_bytes += (double)lay.sz_fg[i];
  }
  HIP_TRY(prof.begin());

  // 1. pad colour, pyramid, tissue map
  for (int i = 0; i < n_slides; ++i) {
    int32_t* pad = reinterpret_cast<int32_t*>(ws + lay.off_pad[i]);
    HIP_TRY(launch_pad_colour(slides[i].rgb, slides[i].row_pitch, pad, sm));
    uint16_t* lvl[4] = {nullptr, nullptr, nullptr, nullptr};
    int Ey[4] = {0, 0, 0, 0}, Ex[4] = {0, 0, 0, 0};
    for (int si = 0; si < c.n_scales; ++si) {
      const ScaleGeom& g = lay.geom[i][si];
      if (g.k >= 1) {
        lvl[g.k] = reinterpret_cast<uint16_t*>(ws + lay.off_pyr[i][si]);
        Ey[g.k] = g.Ey;
        Ex[g.k] = g.Ex;
      }
    }
    HIP_TRY(launch_pyramid(slides[i].rgb, slides[i].row_pitch, slides[i].height, slides[i].width, pad,
                           lay.kmax, lvl, Ey, Ex, sm));
    if (lay.otsu) {
      TissueOtsuArgs ta{};
      ta.rgb = slides[i].rgb;
      ta.pitch = slides[i].row_pitch;
      ta.sums = lay.kc >= 1 ? lvl[lay.kc] : nullptr;
      ta.ex = lay.kc >= 1 ? Ex[lay.kc] : 0;
      ta.kc = lay.kc;
      ta.Hc = lay.Hc[i];
      ta.Wc = lay.Wc[i];
      ta.median = c.median_kernel;
      ta.min_area = c.min_tissue_area;
      ta.tmp = reinterpret_cast<uint8_t*>(ws + lay.off_ttmp);
      ta.gray = reinterpret_cast<uint8_t*>(ws + lay.off_tgray[i]);
      ta.hist = reinterpret_cast<uint32_t*>(ws + lay.off_thist);
      ta.stats = reinterpret_cast<int32_t*>(ws + lay.off_tstats[i]);
      ta.label = reinterpret_cast<int32_t*>(ws + lay.off_tlabel);
      ta.area = reinterpret_cast<int32_t*>(ws + lay.off_tarea);
      ta.fg = reinterpret_cast<uint8_t*>(ws + lay.off_fg[i]);
      HIP_TRY(launch_tissue_otsu(ta, sm));
    } else if (lay.need_fg) {
      const uint16_t* sums = lay.kc >= 1 ? lvl[lay.kc] : nullptr;
      const int ex = lay.kc >= 1 ? Ex[lay.kc] : 0;
      HIP_TRY(launch_tissue(slides[i].rgb, slides[i].row_pitch, slides[i].height, slides[i].width, pad,
                            sums, ex, lay.kc, lay.Hc[i], lay.Wc[i], c.fg_threshold,
                            reinterpret_cast<uint8_t*>(ws + lay.off_fg[i]), sm));
    }
  }
  // 2. tile flags, compaction and prefix counts; the later launches are
  // sized for every grid tile and skip list positions at or past the count
  int32_t* index = reinterpret_cast<int32_t*>(ws + lay.off_index);
  int32_t* list = reinterpret_cast<int32_t*>(ws + lay.off_list);
  int32_t* count = reinterpret_cast<int32_t*>(ws + lay.off_count);
  int32_t* pre = reinterpret_cast<int32_t*>(ws + lay.off_pre);
  HIP_TRY(launch_tile_flags(lay.groups, tab_dev, T, lay.kc, c.fg_filter, index, sm));
  HIP_TRY(launch_compact(index, lay.total_tiles, lay.groups, list, count, pre, sm));
  HIP_TRY(prof.end(OMNISEG_STAGE_PREP, -1, 0, 0.0, prep_bytes));
  return OMNISEG_OK;
}

// Waits for the stream and reads the kept-tile count back (calls that are
// synchronous by contract, and profiled calls); also reports a tissue
// labelling that did not converge.
int32_t read_kept(const Layout& lay, int32_t n_slides, const char* ws, hipStream_t sm, int32_t* n_kept_out) {
  int32_t n_kept = 0;
  HIP_TRY(hipMemcpyAsync(&n_kept, ws + lay.off_count, sizeof(int32_t), hipMemcpyDeviceToHost, sm));
  int32_t tstats[OMNISEG_MAX_SLIDES][4] = {};
  if (lay.otsu)
    for (int i = 0; i < n_slides; ++i)
      HIP_TRY(hipMemcpyAsync(tstats[i], ws + lay.off_tstats[i], 16, hipMemcpyDeviceToHost, sm));
  HIP_TRY(hipStreamSynchronize(sm));
  for (int i = 0; i < n_slides; ++i)
    if (tstats[i][3]) return fail(OMNISEG_ERR_HIP, "slide %d: tissue component labelling did not converge", i);
  if (n_kept < 0 || n_kept > lay.total_tiles)
    return fail(OMNISEG_ERR_HIP, "kept-tile count %d outside [0, %d]", n_kept, lay.total_tiles);
  *n_kept_out = n_kept;
  return OMNISEG_OK;
}

// Stitch form of a plane (as launch_stitch chooses it): four pixels per
// thread needs shared covering tiles (s, T multiples of 4) and aligned
// vector reads of the tile logits (output rows may have any alignment); the
// 2 x 2 form also needs T <= 2 s and 32-bit byte offsets inside a logit slot.
int stitch_mode(int T, int s, int64_t tile_stride, int64_t slot_off, const float* logits, const float* logit) {
  const bool span4 = s % 4 == 0 && T % 4 == 0 && tile_stride % 4 == 0 && slot_off % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(logits) % 16 == 0 &&
                     (!logit || reinterpret_cast<uintptr_t>(logit) % 4 == 0);
  if (!span4) return 0;
  return (T <= 2 * s && tile_stride * 4 <= INT32_MAX) ? 2 : 1;
}

// Algorithmic bytes of each batch's streamed stitch: every in-plane pixel of
// every kept covering tile read once (4 B) and every output pixel written
// (1 B mask, + 4 B logit), attributed to the batch after which its unit is
// stitched.  idx: the index grid (list index or -1 per grid tile).
std::vector<double> stream_stitch_bytes(const Layout& lay, const std::vector<int32_t>& idx, int T, bool emit) {
  std::vector<double> out(lay.n_batches, 0.0);
  std::vector<int32_t> pre(lay.total_tiles + 1, 0);
  for (int t = 0; t < lay.total_tiles; ++t) pre[t + 1] = pre[t] + (idx[t] >= 0 ? 1 : 0);
  for (int gi = 0; gi < lay.groups.n; ++gi) {
    const StreamGroup& g = lay.sgroups[gi];
    if (g.n_planes == 0) continue;
    for (int j = 0; j < g.ny; ++j) {
      const int pos_end = pre[g.grid_base + (int64_t)(j + 1) * g.nx];
      const int b = pos_end > 0 ? (pos_end - 1) / lay.batch : 0;
      const int y0 = j * g.s, y1 = j == g.ny - 1 ? g.Hk : (j + 1) * g.s;
      double bytes = (double)(y1 - y0) * g.Wk * (emit ? 5.0 : 1.0);
      const int jlo = y0 < T ? 0 : (y0 - T) / g.s + 1;
      for (int jt = jlo; jt <= j; ++jt) {
        const int r0 = std::max(y0, jt * g.s), r1 = std::min(std::min(y1, jt * g.s + T), g.Hk);
        if (r1 <= r0) continue;
        for (int jx = 0; jx < g.nx; ++jx)
          if (idx[g.grid_base + (int64_t)jt * g.nx + jx] >= 0)
            bytes += 4.0 * (r1 - r0) * std::min(T, g.Wk - jx * g.s);
      }
      out[b] += bytes * g.n_planes;
    }
  }
  return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* omniseg_status_string(int32_t status) {
  switch (status) {
    case OMNISEG_OK: return "ok";
    case OMNISEG_ERR_ARG: return "invalid argument";
    case OMNISEG_ERR_UNSUPPORTED: return "unsupported configuration";
    case OMNISEG_ERR_WORKSPACE: return "workspace too small";
    case OMNISEG_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* omniseg_last_error(void) { return omniseg::last_error_text(); }

int32_t omniseg_plan_create(const omniseg_config* cfg, omniseg_plan** out) {
  if (!out) return fail(OMNISEG_ERR_ARG, "out is NULL");
  int32_t st = validate_config(cfg);
  if (st) return st;
  omniseg_plan* p = new (std::nothrow) omniseg_plan();
  if (!p) return fail(OMNISEG_ERR_ARG, "out of host memory");
  p->cfg = *cfg;
  p->L = cfg->levels;
  for (int st = 0; st < 4; ++st)
    for (int l = 0; l < 8; ++l) p->tune[st][l] = -1;
  for (int l = 0; l < p->L; ++l) {
    p->C[l] = cfg->base_channels << l;
    p->Cp[l] = pad_ch(p->C[l]);
  }
  p->P = 144 + 9 * cfg->head_out;
  p->G = p->C[p->L - 1];
  const int es = elem_size(cfg->precision);
  const bool training = (cfg->flags & OMNISEG_FLAG_TRAINING) != 0;
  const bool fp8 = cfg->precision == OMNISEG_FP8;
  // activation table: kind-major, level ascending
  for (int k = 0; k < 4; ++k)
    for (int l = 0; l < 8; ++l) p->act_off[k][l] = -1;
  {
    int64_t a = 0;
    for (int k = 0; k < 4; ++k) {
      const int nl = k < 2 ? p->L : p->L - 1;
      for (int l = 0; l < nl; ++l) {
        p->act_off[k][l] = a;
        a += p->Cp[l];
      }
    }
    p->n_act = a;
  }
  int64_t canon = 0, pk = 0;
  auto ptake = [&](int64_t bytes) {
    int64_t o = pk;
    pk += align256(std::max<int64_t>(bytes, 1));
    return o;
  };
  auto conv = [&](ConvDesc& d, int cin, int cout, int cu, int cu_p, int cin_p) {
    d.canon_w = canon;
    canon += (int64_t)cout * cin * 9;
    d.canon_b = canon;
    canon += cout;
    d.cin = cin;
    d.cout = cout;
    d.cu = cu;
    d.cu_p = cu_p;
    d.cin_p = cin_p;
    d.cout_p = pad_ch(cout);
    const int64_t kin = fp8 ? (int64_t)ceil_div(d.cin_p, kFp8Chunk) * kFp8Chunk : d.cin_p;
    d.pk_w = ptake(kin * 9 * d.cout_p * es);
    d.pk_b = ptake((int64_t)d.cout_p * 4);
    d.pk_wt = training ? ptake((int64_t)d.cin_p * 9 * d.cout_p * es) : -1;
    d.pk_ws = fp8 ? ptake((int64_t)d.cout_p * 4) : -1;
  };
  for (int l = 0; l < p->L; ++l) {
    if (l == 0) {
      p->canon_first_w = canon;
      canon += (int64_t)p->C[0] * 27;
      p->canon_first_b = canon;
      canon += p->C[0];
      p->pk_first_w = ptake((int64_t)p->C[0] * 27 * 4);
      p->pk_first_b = ptake((int64_t)p->C[0] * 4);
    } else {
      conv(p->enc_a[l], p->C[l - 1], p->C[l], p->C[l - 1], p->Cp[l - 1], p->Cp[l - 1]);
    }
    conv(p->enc_b[l], p->C[l], p->C[l], p->C[l], p->Cp[l], p->Cp[l]);
  }
  for (int l = p->L - 2; l >= 0; --l) {
    const int cu = p->C[l + 1], cu_p = p->Cp[l + 1];
    conv(p->dec_a[l], 3 * p->C[l], p->C[l], cu, cu_p, cu_p + p->Cp[l]);
    conv(p->dec_b[l], p->C[l], p->C[l], p->C[l], p->Cp[l], p->Cp[l]);
  }
  if (p->C[0] != 8) {
    p->canon_pre_w = canon;
    canon += 8LL * p->C[0];
    p->canon_pre_b = canon;
    canon += 8;
    p->pk_pre_w = ptake(8LL * p->C[0] * 4);
    p->pk_pre_b = ptake(8 * 4);
  }
  // activation-table offsets of each conv's input and output channel scales
  for (int l = 0; l < p->L; ++l) {
    if (l > 0) {
      p->enc_a[l].act_in = p->act_off[OMNISEG_ACT_ENC_E][l - 1];
      p->enc_a[l].act_out = p->act_off[OMNISEG_ACT_ENC_A][l];
    }
    p->enc_b[l].act_in = p->act_off[OMNISEG_ACT_ENC_A][l];
    p->enc_b[l].act_out = p->act_off[OMNISEG_ACT_ENC_E][l];
  }
  for (int l = p->L - 2; l >= 0; --l) {
    // D_{L-1} is E_{L-1}
    p->dec_a[l].act_in = l + 1 == p->L - 1 ? p->act_off[OMNISEG_ACT_ENC_E][l + 1] : p->act_off[OMNISEG_ACT_DEC_D][l + 1];
    p->dec_a[l].act_in_e = p->act_off[OMNISEG_ACT_ENC_E][l];
    p->dec_a[l].act_out = p->act_off[OMNISEG_ACT_DEC_A][l];
    p->dec_b[l].act_in = p->act_off[OMNISEG_ACT_DEC_A][l];
    p->dec_b[l].act_out = p->act_off[OMNISEG_ACT_DEC_D][l];
  }
  if (fp8) {
    p->pk_scale = ptake(p->n_act * 4);
    p->pk_iscale = ptake(p->n_act * 4);
  }
  const int row = p->G + cfg->n_classes + cfg->n_scales;
  p->canon_ctrl_w = canon;
  canon += (int64_t)p->P * row;
  p->canon_ctrl_b = canon;
  canon += p->P;
  p->pk_ctrl_w = ptake((int64_t)p->P * row * 4);
  p->pk_ctrl_b = ptake((int64_t)p->P * 4);
  p->n_canon = canon;
  p->packed_bytes = pk;
  *out = p;
  return OMNISEG_OK;
}

int32_t omniseg_plan_destroy(omniseg_plan* plan) {
  delete plan;
  return OMNISEG_OK;
}

int32_t omniseg_weight_count(const omniseg_plan* plan, int64_t* count) {
  if (!plan || !count) return fail(OMNISEG_ERR_ARG, "NULL argument");
  *count = plan->n_canon;
  return OMNISEG_OK;
}

int32_t omniseg_packed_weight_bytes(const omniseg_plan* plan, int64_t* bytes) {
  if (!plan || !bytes) return fail(OMNISEG_ERR_ARG, "NULL argument");
  *bytes = plan->packed_bytes;
  return OMNISEG_OK;
}

int32_t omniseg_pack_weights(const omniseg_plan* plan, const float* canonical, void* packed,
                             omniseg_stream stream) {
  if (!plan || !canonical || !packed) return fail(OMNISEG_ERR_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(packed) % 256) return fail(OMNISEG_ERR_ARG, "packed buffer not 256-byte aligned");
  if (plan->cfg.precision == OMNISEG_FP8)
    return fail(OMNISEG_ERR_UNSUPPORTED, "FP8 plans pack with omniseg_pack_weights_fp8 (activation scales needed)");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const int prec = plan->cfg.precision;
  char* pk = static_cast<char*>(packed);
  auto pack = [&](const ConvDesc& d) -> hipError_t {
    PackConv pc;
    pc.src = d.canon_w;
    pc.src_b = d.canon_b;
    pc.cout = d.cout;
    pc.cin = d.cin;
    pc.cu = d.cu;
    pc.cu_p = d.cu_p;
    pc.cin_p = d.cin_p;
    pc.cout_p = d.cout_p;
    pc.dst = d.pk_w;
    pc.dst_b = d.pk_b;
    pc.transpose = 0;
    hipError_t e = launch_pack_conv(prec, canonical, packed, pc, st);
    if (e != hipSuccess || d.pk_wt < 0) return e;
    pc.dst = d.pk_wt;
    pc.dst_b = -1;
    pc.transpose = 1;
    return launch_pack_conv(prec, canonical, packed, pc, st);
  };
  HIP_TRY(launch_copy_f32(canonical + plan->canon_first_w, (float*)(pk + plan->pk_first_w), (int64_t)plan->C[0] * 27, st));
  HIP_TRY(launch_copy_f32(canonical + plan->canon_first_b, (float*)(pk + plan->pk_first_b), plan->C[0], st));
  for (int l = 0; l < plan->L; ++l) {
    if (l > 0) HIP_TRY(pack(plan->enc_a[l]));
    HIP_TRY(pack(plan->enc_b[l]));
  }
  for (int l = plan->L - 2; l >= 0; --l) {
    HIP_TRY(pack(plan->dec_a[l]));
    HIP_TRY(pack(plan->dec_b[l]));
  }
  if (plan->canon_pre_w >= 0) {
    HIP_TRY(launch_copy_f32(canonical + plan->canon_pre_w, (float*)(pk + plan->pk_pre_w), 8LL * plan->C[0], st));
    HIP_TRY(launch_copy_f32(canonical + plan->canon_pre_b, (float*)(pk + plan->pk_pre_b), 8, st));
  }
  const int row = plan->G + plan->cfg.n_classes + plan->cfg.n_scales;
  HIP_TRY(launch_copy_f32(canonical + plan->canon_ctrl_w, (float*)(pk + plan->pk_ctrl_w), (int64_t)plan->P * row, st));
  HIP_TRY(launch_copy_f32(canonical + plan->canon_ctrl_b, (float*)(pk + plan->pk_ctrl_b), plan->P, st));
  return OMNISEG_OK;
}

int32_t omniseg_activation_channels(const omniseg_plan* plan, int64_t* count) {
  if (!plan || !count) return fail(OMNISEG_ERR_ARG, "NULL argument");
  *count = plan->n_act;
  return OMNISEG_OK;
}

int32_t omniseg_activation_offset(const omniseg_plan* plan, int32_t kind, int32_t level, int64_t* offset) {
  if (!plan || !offset) return fail(OMNISEG_ERR_ARG, "NULL argument");
  if (kind < 0 || kind > 3 || level < 0 || level > 7 || plan->act_off[kind][level] < 0)
    return fail(OMNISEG_ERR_ARG, "no activation (kind %d, level %d) in this network", kind, level);
  *offset = plan->act_off[kind][level];
  return OMNISEG_OK;
}

int32_t omniseg_pack_weights_fp8(const omniseg_plan* plan, const float* canonical, const float* amax, void* packed,
                                 omniseg_stream stream) {
  if (!plan || !canonical || !amax || !packed) return fail(OMNISEG_ERR_ARG, "NULL argument");
  if (plan->cfg.precision != OMNISEG_FP8) return fail(OMNISEG_ERR_ARG, "plan precision is not OMNISEG_FP8");
  if (reinterpret_cast<uintptr_t>(packed) % 256) return fail(OMNISEG_ERR_ARG, "packed buffer not 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  char* pk = static_cast<char*>(packed);
  float* scale = reinterpret_cast<float*>(pk + plan->pk_scale);
  float* iscale = reinterpret_cast<float*>(pk + plan->pk_iscale);
  HIP_TRY(launch_fp8_scales(amax, plan->n_act, scale, iscale, st));
  auto pack = [&](const ConvDesc& d) -> hipError_t {
    PackConv pc;
    pc.src = d.canon_w;
    pc.src_b = d.canon_b;
    pc.cout = d.cout;
    pc.cin = d.cin;
    pc.cu = d.cu;
    pc.cu_p = d.cu_p;
    pc.cin_p = d.cin_p;
    pc.cout_p = d.cout_p;
    pc.dst = d.pk_w;
    pc.dst_b = d.pk_b;
    pc.transpose = 0;
    return launch_pack_conv_fp8(canonical, packed, pc, scale + d.act_in, d.act_in_e >= 0 ? scale + d.act_in_e : nullptr,
                                reinterpret_cast<float*>(pk + d.pk_ws), st);
  };
  HIP_TRY(launch_copy_f32(canonical + plan->canon_first_w, (float*)(pk + plan->pk_first_w), (int64_t)plan->C[0] * 27, st));
  HIP_TRY(launch_copy_f32(canonical + plan->canon_first_b, (float*)(pk + plan->pk_first_b), plan->C[0], st));
  for (int l = 0; l < plan->L; ++l) {
    if (l > 0) HIP_TRY(pack(plan->enc_a[l]));
    HIP_TRY(pack(plan->enc_b[l]));
  }
  for (int l = plan->L - 2; l >= 0; --l) {
    HIP_TRY(pack(plan->dec_a[l]));
    HIP_TRY(pack(plan->dec_b[l]));
  }
  if (plan->canon_pre_w >= 0) {
    HIP_TRY(launch_copy_f32(canonical + plan->canon_pre_w, (float*)(pk + plan->pk_pre_w), 8LL * plan->C[0], st));
    HIP_TRY(launch_copy_f32(canonical + plan->canon_pre_b, (float*)(pk + plan->pk_pre_b), 8, st));
  }
  const int row = plan->G + plan->cfg.n_classes + plan->cfg.n_scales;
  HIP_TRY(launch_copy_f32(canonical + plan->canon_ctrl_w, (float*)(pk + plan->pk_ctrl_w), (int64_t)plan->P * row, st));
  HIP_TRY(launch_copy_f32(canonical + plan->canon_ctrl_b, (float*)(pk + plan->pk_ctrl_b), plan->P, st));
  return OMNISEG_OK;
}

int32_t omniseg_calibrate_fp8(const omniseg_plan* plan, const void* packed, const omniseg_slide* slides,
                              int32_t n_slides, const omniseg_pair* pairs, int32_t n_pairs, int32_t n_tiles,
                              float* amax, void* workspace, int64_t ws_bytes, omniseg_stream stream) {
  Layout lay;
  int32_t st = validate_call(plan, slides, n_slides, pairs, n_pairs, lay);
  if (st) return st;
  if (plan->cfg.precision != OMNISEG_FP32) return fail(OMNISEG_ERR_ARG, "calibration runs on an FP32 plan");
  if (n_tiles < 1) return fail(OMNISEG_ERR_ARG, "n_tiles %d < 1", n_tiles);
  if (!packed || !workspace || !amax) return fail(OMNISEG_ERR_ARG, "NULL packed weights, workspace or amax");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 || reinterpret_cast<uintptr_t>(packed) % 256)
    return fail(OMNISEG_ERR_ARG, "workspace and packed weights must be 256-byte aligned");
  compute_layout(plan, slides, n_slides, lay);
  if (ws_bytes < lay.total)
    return fail(OMNISEG_ERR_WORKSPACE, "workspace has %lld bytes, needs %lld", (long long)ws_bytes, (long long)lay.total);
  (void)hipGetLastError();
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const char* pk = static_cast<const char*>(packed);
  const omniseg_config& c = plan->cfg;
  Prof prof = profile_start(plan, sm);
  SlideDev* tab_dev = nullptr;
  int32_t n_kept = 0;
  st = enqueue_tile_list(plan, slides, n_slides, lay, ws, sm, prof, &tab_dev);
  if (st) return st;
  st = read_kept(lay, n_slides, ws, sm, &n_kept);
  if (st) return st;
  const int n = std::min(n_kept, n_tiles);
  int32_t* list = reinterpret_cast<int32_t*>(ws + lay.off_list);
  int32_t* count = reinterpret_cast<int32_t*>(ws + lay.off_count);
  HIP_TRY(launch_zero(amax, plan->n_act * 4, sm));
  const int T = c.tile, L = plan->L, B = lay.batch;
  void* E[8];
  for (int l = 0; l < L; ++l) E[l] = ws + lay.off_E[l];
  void* A = ws + lay.off_A;
  auto layer = [&](const ConvDesc& d) { return make_layer(plan, pk, d); };
  auto stat = [&](const void* x, int nb, int h, int l, int kind) {
    return launch_amax_channels(static_cast<const float*>(x), (int64_t)nb * h * h, plan->Cp[l],
                                amax + plan->act_off[kind][l], sm);
  };
  FirstConvArgs fa{};
  fa.list = list;
  fa.count = count;
  fa.T = T;
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) fa.scale_s[si] = si < c.n_scales ? stride_of(c, si) : c.stride;
  fa.w = reinterpret_cast<const float*>(pk + plan->pk_first_w);
  fa.b = reinterpret_cast<const float*>(pk + plan->pk_first_b);
  fa.c0 = plan->C[0];
  fa.c0_p = plan->Cp[0];
  fa.y = A;
  fa.slides = tab_dev;
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) fa.scale_k[si] = si < c.n_scales ? c.scale_log2[si] : 0;
  const int prec = OMNISEG_FP32;
  for (int base = 0; base < n; base += B) {
    const int nb = std::min(B, n - base);
    fa.chunk_base = base;
    fa.batch = nb;
    HIP_TRY(launch_first_conv(prec, fa, sm));
    HIP_TRY(stat(A, nb, T, 0, OMNISEG_ACT_ENC_A));
    int cf = layer_config(plan, 1, 0, T, T, plan->enc_b[0].cout_p);
    HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, layer(plan->enc_b[0]), T, T, nb, count, base, A, nullptr, E[0], sm, nullptr, cf));
    HIP_TRY(stat(E[0], nb, T, 0, OMNISEG_ACT_ENC_E));
    for (int l = 1; l < L; ++l) {
      const int tl = T >> l;
      cf = layer_config(plan, 0, l, tl, tl, plan->enc_a[l].cout_p);
      HIP_TRY(launch_conv3x3(prec, LOAD_POOL, EPI_RELU, layer(plan->enc_a[l]), tl, tl, nb, count, base, E[l - 1], nullptr, A, sm, nullptr, cf));
      HIP_TRY(stat(A, nb, tl, l, OMNISEG_ACT_ENC_A));
      cf = layer_config(plan, 1, l, tl, tl, plan->enc_b[l].cout_p);
      HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, layer(plan->enc_b[l]), tl, tl, nb, count, base, A, nullptr, E[l], sm, nullptr, cf));
      HIP_TRY(stat(E[l], nb, tl, l, OMNISEG_ACT_ENC_E));
    }
    for (int l = L - 2; l >= 0; --l) {
      const int tl = T >> l;
      cf = layer_config(plan, 2, l, tl, tl, plan->dec_a[l].cout_p);
      HIP_TRY(launch_conv3x3(prec, LOAD_UPCAT, EPI_RELU, layer(plan->dec_a[l]), tl, tl, nb, count, base, E[l + 1], E[l], A, sm, nullptr, cf));
      HIP_TRY(stat(A, nb, tl, l, OMNISEG_ACT_DEC_A));
      cf = layer_config(plan, 3, l, tl, tl, plan->dec_b[l].cout_p);
      HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, layer(plan->dec_b[l]), tl, tl, nb, count, base, A, nullptr, E[l], sm, nullptr, cf));
      HIP_TRY(stat(E[l], nb, tl, l, OMNISEG_ACT_DEC_D));
    }
  }
  HIP_TRY(hipStreamSynchronize(sm));
  return OMNISEG_OK;
}

int32_t omniseg_workspace_bytes(const omniseg_plan* plan, const omniseg_slide* slides,
                                int32_t n_slides, const omniseg_pair* pairs, int32_t n_pairs,
                                int64_t* bytes) {
  if (!bytes) return fail(OMNISEG_ERR_ARG, "bytes is NULL");
  Layout lay;
  int32_t st = validate_call(plan, slides, n_slides, pairs, n_pairs, lay);
  if (st) return st;
  compute_layout(plan, slides, n_slides, lay);
  *bytes = lay.total;
  return OMNISEG_OK;
}

int32_t omniseg_workspace_region(const omniseg_plan* plan, const omniseg_slide* slides,
                                 int32_t n_slides, const omniseg_pair* pairs, int32_t n_pairs,
                                 int32_t region, int32_t index, int64_t* offset, int64_t* bytes) {
  if (!offset || !bytes) return fail(OMNISEG_ERR_ARG, "NULL argument");
  Layout lay;
  int32_t st = validate_call(plan, slides, n_slides, pairs, n_pairs, lay);
  if (st) return st;
  compute_layout(plan, slides, n_slides, lay);
  const int S = plan->cfg.n_scales;
  switch (region) {
    case OMNISEG_REGION_PAD:
      if (index < 0 || index >= n_slides) break;
      *offset = lay.off_pad[index];
      *bytes = 16;
      return OMNISEG_OK;
    case OMNISEG_REGION_PYRAMID:
      if (index < 0 || index >= n_slides * S) break;
      *offset = lay.off_pyr[index / S][index % S];
      *bytes = lay.sz_pyr[index / S][index % S];
      return OMNISEG_OK;
    case OMNISEG_REGION_TISSUE:
      if (index < 0 || index >= n_slides) break;
      *offset = lay.off_fg[index];
      *bytes = lay.sz_fg[index];
      return OMNISEG_OK;
    case OMNISEG_REGION_TILE_COUNT:
      *offset = lay.off_count;
      *bytes = 4;
      return OMNISEG_OK;
    case OMNISEG_REGION_TILE_LIST:
      *offset = lay.off_list;
      *bytes = (int64_t)lay.total_tiles * 16;
      return OMNISEG_OK;
    case OMNISEG_REGION_TILE_INDEX: {
      if (index < 0 || index >= n_slides * S) break;
      const int gi = index;  // groups are enumerated slide-major, slot-minor
      *offset = lay.off_index + (int64_t)lay.groups.base[gi] * 4;
      *bytes = (int64_t)(lay.groups.base[gi + 1] - lay.groups.base[gi]) * 4;
      return OMNISEG_OK;
    }
    case OMNISEG_REGION_TILE_LOGITS:
      *offset = lay.off_logits;
      *bytes = lay.sz_logits;
      return OMNISEG_OK;
    case OMNISEG_REGION_TISSUE_GRAY:
      if (index < 0 || index >= n_slides) break;
      *offset = lay.otsu ? lay.off_tgray[index] : 0;
      *bytes = lay.otsu ? lay.sz_fg[index] : 0;
      return OMNISEG_OK;
    case OMNISEG_REGION_TISSUE_STATS:
      if (index < 0 || index >= n_slides) break;
      *offset = lay.otsu ? lay.off_tstats[index] : 0;
      *bytes = lay.otsu ? 16 : 0;
      return OMNISEG_OK;
    default:
      return fail(OMNISEG_ERR_ARG, "unknown region %d", region);
  }
  return fail(OMNISEG_ERR_ARG, "region %d: index %d out of range", region, index);
}

int32_t omniseg_segment_slide(const omniseg_plan* plan, const void* packed,
                              const omniseg_slide* slides, int32_t n_slides,
                              const omniseg_pair* pairs, int32_t n_pairs,
                              const omniseg_output* outs, void* workspace, int64_t ws_bytes,
                              omniseg_stream stream) {
  Layout lay;
  int32_t st = validate_call(plan, slides, n_slides, pairs, n_pairs, lay);
  if (st) return st;
  if (!packed) return fail(OMNISEG_ERR_ARG, "packed weights are NULL");
  if (!outs) return fail(OMNISEG_ERR_ARG, "outs is NULL");
  if (!workspace) return fail(OMNISEG_ERR_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 || reinterpret_cast<uintptr_t>(packed) % 256)
    return fail(OMNISEG_ERR_ARG, "workspace and packed weights must be 256-byte aligned");
  const omniseg_config& c = plan->cfg;
  const bool emit = (c.flags & OMNISEG_FLAG_EMIT_LOGITS) != 0;
  for (int i = 0; i < n_slides; ++i) {
    for (int p = 0; p < n_pairs; ++p) {
      const omniseg_output& o = outs[(int64_t)i * n_pairs + p];
      const int Wk = ceil_div(slides[i].width, 1 << c.scale_log2[pairs[p].scale]);
      if (!o.mask) return fail(OMNISEG_ERR_ARG, "output (%d, %d): mask is NULL", i, p);
      if (o.mask_pitch < Wk) return fail(OMNISEG_ERR_ARG, "output (%d, %d): mask_pitch %lld < %d", i, p, (long long)o.mask_pitch, Wk);
      if (emit && !o.logit) return fail(OMNISEG_ERR_ARG, "output (%d, %d): logit is NULL with EMIT_LOGITS", i, p);
      if (emit && o.logit_pitch < Wk) return fail(OMNISEG_ERR_ARG, "output (%d, %d): logit_pitch %lld < %d", i, p, (long long)o.logit_pitch, Wk);
    }
  }
  compute_layout(plan, slides, n_slides, lay);
  if (ws_bytes < lay.total)
    return fail(OMNISEG_ERR_WORKSPACE, "workspace has %lld bytes, needs %lld", (long long)ws_bytes, (long long)lay.total);
  if ((c.flags & OMNISEG_FLAG_GRAPH) && stream == nullptr)
    return fail(OMNISEG_ERR_ARG, "OMNISEG_FLAG_GRAPH needs a created stream: the null stream cannot be captured");

  // ---- all checks passed: enqueue the work ----
  (void)hipGetLastError();  // launches below report their own errors, not stale ones
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const char* pk = static_cast<const char*>(packed);
  const int T = c.tile, s = c.stride, prec = c.precision;

  Prof prof = profile_start(plan, sm);
  const int B = lay.batch, L = plan->L;
  int32_t* index = reinterpret_cast<int32_t*>(ws + lay.off_index);
  int32_t* list = reinterpret_cast<int32_t*>(ws + lay.off_list);
  int32_t* count = reinterpret_cast<int32_t*>(ws + lay.off_count);
  float* logits = reinterpret_cast<float*>(ws + lay.off_logits);
  const int64_t tile_stride = (int64_t)lay.max_slots * T * T;

  // host tables of the streamed stitch: per group its tissue map, per
  // (slide, pair) its output planes, in the pairs' slot order within a scale
  std::vector<StreamGroup> groups = lay.sgroups;
  std::vector<StreamPlane> planes(std::max(1, lay.n_planes));
  for (int gi = 0; gi < lay.groups.n; ++gi) {
    const int i = lay.groups.slide[gi], si = lay.groups.slot[gi];
    StreamGroup& sg = groups[gi];
    sg.fg = c.mask_and_fg ? reinterpret_cast<const uint8_t*>(ws + lay.off_fg[i]) : nullptr;
    for (int p = 0; p < n_pairs; ++p) {
      if (pairs[p].scale != si) continue;
      const omniseg_output& o = outs[(int64_t)i * n_pairs + p];
      StreamPlane& pl = planes[sg.plane_first + lay.pair_slot[p]];
      pl.mask = o.mask;
      pl.mask_pitch = o.mask_pitch;
      pl.logit = emit ? o.logit : nullptr;
      pl.logit_pitch = emit ? o.logit_pitch : 0;
      pl.slot_off = (int64_t)lay.pair_slot[p] * T * T;
      pl.mode = stitch_mode(T, sg.s, tile_stride, pl.slot_off, logits, pl.logit);
      pl.pad_ = 0;
    }
  }
  StreamStitchArgs sargs{};
  sargs.groups = reinterpret_cast<const StreamGroup*>(ws + lay.off_sgroups);
  sargs.planes = reinterpret_cast<const StreamPlane*>(ws + lay.off_splanes);
  sargs.units = reinterpret_cast<StreamUnit*>(ws + lay.off_units);
  sargs.batch_first = reinterpret_cast<int32_t*>(ws + lay.off_bfirst);
  sargs.n_batches = lay.n_batches;
  sargs.n_groups = lay.groups.n;
  sargs.n_units = lay.n_units;
  sargs.pre = reinterpret_cast<const int32_t*>(ws + lay.off_pre);
  sargs.index = index;
  sargs.logits = logits;
  sargs.tile_stride = tile_stride;
  sargs.ring = lay.resident ? 0 : lay.ring;
  sargs.T = T;
  sargs.B = B;
  sargs.n_items = lay.n_items;

  // The whole call: tile list, then the backbone over batches of B list
  // positions, launched for every grid tile (a batch past the kept-tile
  // count exits at once), each batch followed by the stitch of the tile rows
  // it completed.  Nothing waits for the device unless profiling is on.
  // With OMNISEG_FLAG_GRAPH the sequence is captured once per distinct
  // argument set and replayed as one HIP graph.
  auto enqueue = [&]() -> int32_t {
    SlideDev* tab_dev = nullptr;
    int32_t est = enqueue_tile_list(plan, slides, n_slides, lay, ws, sm, prof, &tab_dev);
    if (est) return est;
    HIP_TRY(launch_put(ws + lay.off_sgroups, groups.data(), (int64_t)groups.size() * sizeof(StreamGroup), sm));
    HIP_TRY(launch_put(ws + lay.off_splanes, planes.data(), (int64_t)planes.size() * sizeof(StreamPlane), sm));
    HIP_TRY(launch_stream_units(sargs, sm));
    // profiling: the kept-tile count and the index grid make the per-launch
    // algorithmic work exact (the launches are the same as without profiling)
    int32_t n_kept = -1;
    std::vector<double> stitch_bytes;
    if (plan->profiling) {
      est = read_kept(lay, n_slides, ws, sm, &n_kept);
      if (est) return est;
      std::vector<int32_t> idx_host(lay.total_tiles);
      HIP_TRY(hipMemcpyAsync(idx_host.data(), index, sizeof(int32_t) * lay.total_tiles, hipMemcpyDeviceToHost, sm));
      HIP_TRY(hipStreamSynchronize(sm));
      stitch_bytes = stream_stitch_bytes(lay, idx_host, T, emit);
    }
    void* E[8];
    for (int l = 0; l < L; ++l) E[l] = ws + lay.off_E[l];
    void* A = ws + lay.off_A;
    float* g = reinterpret_cast<float*>(ws + lay.off_g);
    float* theta = reinterpret_cast<float*>(ws + lay.off_theta);
    auto layer = [&](const ConvDesc& d) { return make_layer(plan, pk, d); };
    const int es = elem_size(prec);
    FirstConvArgs fa{};
    fa.list = list;
    fa.count = count;
    fa.T = T;
    for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) fa.scale_s[si] = si < c.n_scales ? stride_of(c, si) : s;
    fa.w = reinterpret_cast<const float*>(pk + plan->pk_first_w);
    fa.b = reinterpret_cast<const float*>(pk + plan->pk_first_b);
    fa.c0 = plan->C[0];
    fa.c0_p = plan->Cp[0];
    fa.y = A;
    fa.slides = tab_dev;
    for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) fa.scale_k[si] = si < c.n_scales ? c.scale_log2[si] : 0;
    if (prec == OMNISEG_FP8)
      fa.oinv = reinterpret_cast<const float*>(pk + plan->pk_iscale) + plan->act_off[OMNISEG_ACT_ENC_A][0];
    for (int bi = 0; bi < lay.n_batches; ++bi) {
      const int base = bi * B;
      const int nb = std::min(B, lay.total_tiles - base);
      // tiles of this batch that are kept (known when profiling; records only)
      const int nk = n_kept >= 0 ? std::max(0, std::min(nb, n_kept - base)) : nb;
      // algorithmic work of one 3x3 conv launch over the batch's kept tiles at
      // h x h: input, output and weights once (a residual conv adds its own
      // input, so the residual costs no bytes of its own)
      auto conv_flops = [&](const ConvDesc& d, int h) { return 2.0 * 9 * d.cin * d.cout * (double)h * h * nk; };
      auto conv_bytes = [&](const ConvDesc& d, int h, double in_px_factor) {
        const double px = (double)h * h * nk;
        return nk == 0 ? 0.0 : px * in_px_factor * d.cin * es + px * d.cout * es + 9.0 * d.cin * d.cout * es;
      };
      fa.chunk_base = base;
      fa.batch = nb;
      HIP_TRY(prof.begin());
      HIP_TRY(launch_first_conv(prec, fa, sm));
      HIP_TRY(prof.end(OMNISEG_STAGE_FIRST_CONV, 0, nk, 2.0 * 27 * plan->C[0] * (double)T * T * nk,
                       (double)T * T * nk * (3.0 + plan->C[0] * es)));
      // encoder; with the fused pool, enc_b writes E_l and its pooled copy P
      // and the next conv_a reads P with the plain loader
      const bool fp = fuse_pool(plan);
      // BF16 with a 64-channel D_0 whose last conv runs weight-stationary
      // (configuration 10 with enough pixel blocks): that conv computes the
      // head's precls as well, and D_0 never reaches memory.  The precls
      // arithmetic is the head's own, so the logits are the same either way.
      auto fuse_precls = [&](int cf, int nbatch) {
        return prec == OMNISEG_BF16 && L >= 2 && plan->canon_pre_w >= 0 && plan->C[0] == 64 && plan->Cp[0] == 64 &&
               cf == CONV_CFG_ROWS8_16x16_64 && conv_precls_fusable(layer(plan->dec_b[0]), T, T, nbatch);
      };
      void* P = ws + lay.off_P;
      for (int l = 0; l < L; ++l) {
        const int tl = T >> l;
        int cf;
        if (l > 0) {
          HIP_TRY(prof.begin());
          cf = layer_config(plan, 0, l, tl, tl, plan->enc_a[l].cout_p);
          HIP_TRY(launch_conv3x3(prec, fp ? LOAD_PLAIN : LOAD_POOL, EPI_RELU, layer(plan->enc_a[l]), tl, tl, nb, count,
                                 base, fp ? P : E[l - 1], nullptr, A, sm, nullptr, cf));
          HIP_TRY(prof.end(OMNISEG_STAGE_ENC_A, l, nk, conv_flops(plan->enc_a[l], tl),
                           conv_bytes(plan->enc_a[l], tl, fp ? 1.0 : 4.0), cf));
        }
        HIP_TRY(prof.begin());
        ConvLayer lb = layer(plan->enc_b[l]);
        double pooled_bytes = 0.0;
        if (fp && l + 1 < L) {
          lb.pool_out = P;
          cf = pool_config(plan, l, tl, tl, plan->enc_b[l].cout_p);
          pooled_bytes = (double)nk * (tl / 2) * (tl / 2) * plan->enc_b[l].cout * es;
        } else {
          cf = layer_config(plan, 1, l, tl, tl, plan->enc_b[l].cout_p);
        }
        HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, lb, tl, tl, nb, count, base, A, nullptr, E[l], sm,
                               nullptr, cf));
        HIP_TRY(prof.end(OMNISEG_STAGE_ENC_B, l, nk, conv_flops(plan->enc_b[l], tl),
                         conv_bytes(plan->enc_b[l], tl, 1.0) + pooled_bytes, cf));
      }
      const int tb = T >> (L - 1);
      HIP_TRY(prof.begin());
      HIP_TRY(launch_gap(prec, E[L - 1], nb, tb * tb, plan->Cp[L - 1], plan->G, count, base, g, sm,
                         fp8_scale_of(plan, pk, OMNISEG_ACT_ENC_E, L - 1)));
      HIP_TRY(launch_controller(g, nb, plan->G, reinterpret_cast<const float*>(pk + plan->pk_ctrl_w),
                                reinterpret_cast<const float*>(pk + plan->pk_ctrl_b), plan->P, c.n_classes,
                                c.n_scales, lay.slots, lay.max_slots, list, count, base, theta, sm));
      HIP_TRY(prof.end(OMNISEG_STAGE_GAP_CTRL, L - 1, nk,
                       (double)nk * ((double)plan->G * tb * tb + 2.0 * plan->P * plan->G * lay.max_slots),
                       (double)nk * tb * tb * plan->G * es));
      for (int l = L - 2; l >= 0; --l) {
        const int tl = T >> l;
        // decoder level l: Z = [up2(D_{l+1}) ; E_l]; D_{l+1} lives in E[l+1]'s buffer
        HIP_TRY(prof.begin());
        int cf = layer_config(plan, 2, l, tl, tl, plan->dec_a[l].cout_p);
        HIP_TRY(launch_conv3x3(prec, LOAD_UPCAT, EPI_RELU, layer(plan->dec_a[l]), tl, tl, nb, count, base, E[l + 1],
                               E[l], A, sm, nullptr, cf));
        HIP_TRY(prof.end(OMNISEG_STAGE_DEC_A, l, nk, conv_flops(plan->dec_a[l], tl), conv_bytes(plan->dec_a[l], tl, 0.5),
                         cf));
        HIP_TRY(prof.begin());
        cf = layer_config(plan, 3, l, tl, tl, plan->dec_b[l].cout_p);
        if (l == 0 && fuse_precls(cf, nb)) {
          // the last decoder conv writes the head's precls output F (8 FP32
          // per pixel) into D_0's buffer instead of D_0
          HIP_TRY(launch_conv_ws_precls(layer(plan->dec_b[0]), T, T, nb, count, base, A,
                                        reinterpret_cast<const float*>(pk + plan->pk_pre_w),
                                        reinterpret_cast<const float*>(pk + plan->pk_pre_b),
                                        reinterpret_cast<float*>(E[0]), sm));
          const double px = (double)T * T * nk;
          HIP_TRY(prof.end(OMNISEG_STAGE_DEC_B, 0, nk, conv_flops(plan->dec_b[0], T) + px * 2.0 * 8 * plan->C[0],
                           conv_bytes(plan->dec_b[0], T, 1.0) - px * plan->dec_b[0].cout * es + px * 32.0, cf));
          continue;
        }
        HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, layer(plan->dec_b[l]), tl, tl, nb, count, base, A,
                               nullptr, E[l], sm, nullptr, cf));
        HIP_TRY(prof.end(OMNISEG_STAGE_DEC_B, l, nk, conv_flops(plan->dec_b[l], tl), conv_bytes(plan->dec_b[l], tl, 1.0),
                         cf));
      }
      const bool fused = L >= 2 && fuse_precls(layer_config(plan, 3, 0, T, T, plan->dec_b[0].cout_p), nb);
      HIP_TRY(prof.begin());
      HIP_TRY(launch_head(prec, E[0], nb, T, plan->C[0], plan->Cp[0],
                          plan->canon_pre_w >= 0 ? reinterpret_cast<const float*>(pk + plan->pk_pre_w) : nullptr,
                          plan->canon_pre_w >= 0 ? reinterpret_cast<const float*>(pk + plan->pk_pre_b) : nullptr,
                          theta, plan->P, c.head_out, lay.slots, lay.max_slots, list, count, base,
                          lay.resident ? base : base % lay.ring, logits, sm,
                          L >= 2 ? fp8_scale_of(plan, pk, OMNISEG_ACT_DEC_D, 0) : fp8_scale_of(plan, pk, OMNISEG_ACT_ENC_E, 0),
                          fused ? reinterpret_cast<const float*>(E[0]) : nullptr));
      {
        const double px = (double)T * T * nk;
        const double pre = plan->canon_pre_w >= 0 && !fused ? 2.0 * 8 * plan->C[0] : 0.0;
        // slots per tile vary with the tile's scale; count the largest
        const double head = lay.max_slots * (2.0 * 64 + 2.0 * 64 + 2.0 * 8 * c.head_out);
        HIP_TRY(prof.end(OMNISEG_STAGE_HEAD, 0, nk, px * (pre + head),
                         px * ((fused ? 32.0 : plan->C[0] * es) + 4.0 * lay.max_slots)));
      }
      // 4. stitch the tile rows this batch completed
      sargs.batch = bi;
      HIP_TRY(prof.begin());
      HIP_TRY(launch_stitch_stream(sargs, sm));
      HIP_TRY(prof.end(OMNISEG_STAGE_STITCH, -1, 0, 0.0, plan->profiling ? stitch_bytes[bi] : 0.0));
    }
    return OMNISEG_OK;
  };
  const bool use_graph = (c.flags & OMNISEG_FLAG_GRAPH) && !plan->profiling;
  if (!use_graph) return enqueue();
  uint64_t key = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) key = (key ^ b[i]) * 1099511628211ull;
  };
  mix(&packed, sizeof(packed));
  mix(&workspace, sizeof(workspace));
  mix(&ws_bytes, sizeof(ws_bytes));
  mix(slides, sizeof(omniseg_slide) * n_slides);
  mix(pairs, sizeof(omniseg_pair) * n_pairs);
  mix(outs, sizeof(omniseg_output) * (size_t)n_slides * n_pairs);
  mix(plan->tune, sizeof(plan->tune));  // the conv tile configurations are baked into the graph
  for (const auto& gc : plan->graphs) {
    if (gc.key == key) {
      HIP_TRY(hipGraphLaunch(gc.exec, sm));
      return OMNISEG_OK;
    }
  }
  HIP_TRY(hipStreamBeginCapture(sm, hipStreamCaptureModeThreadLocal));
  const int32_t est = enqueue();
  hipGraph_t graph = nullptr;
  const hipError_t cap = hipStreamEndCapture(sm, &graph);
  if (est != OMNISEG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return est;
  }
  if (cap != hipSuccess) return fail(OMNISEG_ERR_HIP, "stream capture failed: %s", hipGetErrorString(cap));
  hipGraphExec_t exec = nullptr;
  const hipError_t ins = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ins != hipSuccess) return fail(OMNISEG_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ins));
  if (plan->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(plan->graphs.front().exec);
    plan->graphs.erase(plan->graphs.begin());
  }
  plan->graphs.push_back({key, exec});
  HIP_TRY(hipGraphLaunch(exec, sm));
  return OMNISEG_OK;
}

static_assert(CONV_CFG_COUNT == OMNISEG_CONV_CONFIGS, "configuration count in the header");

int32_t omniseg_conv_config(int32_t config, int32_t* by, int32_t* bx, int32_t* bn, int32_t* wm, int32_t* wn,
                            int32_t* precisions) {
  if (config < 0 || config >= CONV_CFG_COUNT || !by || !bx || !bn || !wm || !wn || !precisions)
    return fail(OMNISEG_ERR_ARG, "unknown conv config %d", config);
  *precisions = conv_config_precisions(config);
  int a, b, c, d, e;
  conv_config_shape(config, &a, &b, &c, &d, &e);
  *by = a;
  *bx = b;
  *bn = c;
  *wm = d;
  *wn = e;
  return OMNISEG_OK;
}

int32_t omniseg_autotune(omniseg_plan* plan, const void* packed, const omniseg_slide* slides, int32_t n_slides,
                         const omniseg_pair* pairs, int32_t n_pairs, void* workspace, int64_t ws_bytes,
                         omniseg_stream stream) {
  Layout lay;
  int32_t st = validate_call(plan, slides, n_slides, pairs, n_pairs, lay);
  if (st) return st;
  if (!packed || !workspace) return fail(OMNISEG_ERR_ARG, "NULL packed weights or workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 || reinterpret_cast<uintptr_t>(packed) % 256)
    return fail(OMNISEG_ERR_ARG, "workspace and packed weights must be 256-byte aligned");
  compute_layout(plan, slides, n_slides, lay);
  if (ws_bytes < lay.total)
    return fail(OMNISEG_ERR_WORKSPACE, "workspace has %lld bytes, needs %lld", (long long)ws_bytes, (long long)lay.total);
  (void)hipGetLastError();
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const char* pk = static_cast<const char*>(packed);
  const int T = plan->cfg.tile, prec = plan->cfg.precision, L = plan->L, B = lay.batch;
  void* E[8];
  for (int l = 0; l < L; ++l) {
    E[l] = ws + lay.off_E[l];
    HIP_TRY(launch_zero(E[l], lay.sz_E[l], sm));
  }
  void* A = ws + lay.off_A;
  HIP_TRY(launch_zero(A, lay.sz_A, sm));
  const bool fp = fuse_pool(plan);
  void* P = ws + lay.off_P;
  if (fp) HIP_TRY(launch_zero(P, lay.sz_P, sm));
  int32_t* count = reinterpret_cast<int32_t*>(ws + lay.off_count);
  HIP_TRY(launch_set_i32(count, B, sm));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto layer = [&](const ConvDesc& d) { return make_layer(plan, pk, d); };
  int32_t result = OMNISEG_OK;
  for (int stg = 0; stg < 4 && result == OMNISEG_OK; ++stg) {
    for (int l = 0; l < L && result == OMNISEG_OK; ++l) {
      if ((stg == 0 && l == 0) || (stg >= 2 && l >= L - 1)) continue;
      const ConvDesc& d = stg == 0 ? plan->enc_a[l] : stg == 1 ? plan->enc_b[l] : stg == 2 ? plan->dec_a[l] : plan->dec_b[l];
      const int h = T >> l;
      // the launches segment_slide makes: with the fused pool, conv_a reads the
      // pooled tensor plainly and the residual conv also writes it
      const int loader = stg == 0 ? (fp ? LOAD_PLAIN : LOAD_POOL) : stg == 2 ? LOAD_UPCAT : LOAD_PLAIN;
      const int epi = (stg == 1 || stg == 3) ? EPI_RES_RELU : EPI_RELU;
      const void* x0 = stg == 0 ? (fp ? P : E[l - 1]) : stg == 2 ? E[l + 1] : A;
      const void* x1 = stg == 2 ? E[l] : nullptr;
      void* y = (stg == 1 || stg == 3) ? E[l] : A;
      const bool pooled = fp && stg == 1 && l + 1 < L;
      ConvLayer Ly = layer(d);
      if (pooled) Ly.pool_out = P;
      int best = -1;
      float best_ms = 1e30f;
      for (int cf = 0; cf < CONV_CFG_COUNT; ++cf) {
        if (!conv_config_valid(cf, prec, h, h, d.cout_p)) continue;
        if (pooled && cf < CONV_CFG_ROWS_16x16_64) continue;
        // one untimed launch, then five timed ones (near-equal configurations
        // otherwise swap places from run to run on timing noise)
        hipError_t e = launch_conv3x3(prec, loader, epi, Ly, h, h, B, count, 0, x0, x1, y, sm, nullptr, cf);
        if (e == hipSuccess) e = hipEventRecord(e0, sm);
        for (int r = 0; r < 5 && e == hipSuccess; ++r)
          e = launch_conv3x3(prec, loader, epi, Ly, h, h, B, count, 0, x0, x1, y, sm, nullptr, cf);
        if (e == hipSuccess) e = hipEventRecord(e1, sm);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          result = fail(OMNISEG_ERR_HIP, "autotune launch failed: %s", hipGetErrorString(e));
          break;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = cf;
        }
      }
      plan->tune[stg][l] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

int32_t omniseg_set_conv_tuning(omniseg_plan* plan, int32_t stage, int32_t level, int32_t config) {
  if (!plan) return fail(OMNISEG_ERR_ARG, "plan is NULL");
  if (stage < 0 || stage > 3 || level < 0 || level >= plan->L)
    return fail(OMNISEG_ERR_ARG, "no conv layer at stage %d, level %d", stage, level);
  if (config < -1 || config >= CONV_CFG_COUNT) return fail(OMNISEG_ERR_ARG, "unknown conv config %d", config);
  plan->tune[stage][level] = config;
  return OMNISEG_OK;
}

int32_t omniseg_get_conv_tuning(const omniseg_plan* plan, int32_t stage, int32_t level, int32_t* config) {
  if (!plan || !config) return fail(OMNISEG_ERR_ARG, "NULL argument");
  if (stage < 0 || stage > 3 || level < 0 || level >= plan->L)
    return fail(OMNISEG_ERR_ARG, "no conv layer at stage %d, level %d", stage, level);
  *config = plan->tune[stage][level];
  return OMNISEG_OK;
}

int32_t omniseg_set_profiling(omniseg_plan* plan, int32_t enable) {
  if (!plan) return fail(OMNISEG_ERR_ARG, "plan is NULL");
  plan->profiling = enable != 0;
  return OMNISEG_OK;
}

int32_t omniseg_read_profile(omniseg_plan* plan, omniseg_launch_record* recs, int32_t cap, int32_t* n) {
  if (!plan || !n || (cap > 0 && !recs)) return fail(OMNISEG_ERR_ARG, "NULL argument");
  plan->profile_read = true;  // the next profiled call starts a new list
  const int32_t total = (int32_t)plan->recs.size();
  for (int32_t i = 0; i < total; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventSynchronize(plan->events[2 * i + 1]));
    HIP_TRY(hipEventElapsedTime(&ms, plan->events[2 * i], plan->events[2 * i + 1]));
    plan->recs[i].ms = ms;
    if (i < cap) recs[i] = plan->recs[i];
  }
  *n = total;
  return OMNISEG_OK;
}

int32_t omniseg_conv3x3_workspace_bytes(int32_t precision, int32_t cin, int32_t cu, int32_t cout,
                                        int64_t* bytes) {
  if (!bytes) return fail(OMNISEG_ERR_ARG, "bytes is NULL");
  if (precision != OMNISEG_FP32 && precision != OMNISEG_BF16) return fail(OMNISEG_ERR_UNSUPPORTED, "unknown precision");
  if (cin < 1 || cout < 1 || cu < 1 || cu > cin || cin > 8192 || cout > 8192) return fail(OMNISEG_ERR_ARG, "bad channel counts");
  const int cin_p = cu < cin ? pad_ch(cu) + pad_ch(cin - cu) : pad_ch(cin);
  *bytes = 256 + align256((int64_t)cin_p * 9 * pad_ch(cout) * elem_size(precision)) + align256((int64_t)pad_ch(cout) * 4);
  return OMNISEG_OK;
}

// Row-reuse configuration for a stand-alone conv with a pooled output: the
// requested one (which must be row-reuse), or the first that fits.
static int32_t pooled_conv_config(int precision, int config, int H, int W, int cout_p, int* out) {
  if (config != -1) {
    if (config < CONV_CFG_ROWS_16x16_64) return fail(OMNISEG_ERR_ARG, "a pooled output needs a row-reuse configuration");
    *out = config;
    return OMNISEG_OK;
  }
  for (int c : {CONV_CFG_ROWS_16x16_64, CONV_CFG_ROWS_16x16_32, CONV_CFG_ROWS_32x16_32, CONV_CFG_ROWS_16x16_128})
    if (conv_config_valid(c, precision, H, W, cout_p)) {
      *out = c;
      return OMNISEG_OK;
    }
  return fail(OMNISEG_ERR_UNSUPPORTED, "no row-reuse configuration fits %dx%d", H, W);
}

int32_t omniseg_conv3x3(int32_t precision, int32_t mode, int32_t n, int32_t height, int32_t width, int32_t cin,
                        int32_t cu, int32_t cout, const float* weights, const float* bias, const void* x0,
                        const void* x1, const void* aux, void* y, void* y_pool, int32_t config, void* workspace,
                        int64_t ws_bytes, omniseg_stream stream) {
  int64_t need = 0;
  int32_t st = omniseg_conv3x3_workspace_bytes(precision, cin, cu, cout, &need);
  if (st) return st;
  if (mode < OMNISEG_CONV_RELU || mode > OMNISEG_CONV_DGRAD_RES_MASK) return fail(OMNISEG_ERR_ARG, "unknown mode %d", mode);
  if (n < 1 || height < 8 || width < 8 || height % 8 || width % 8 || height > 4096 || width > 4096)
    return fail(OMNISEG_ERR_ARG, "n >= 1 and H, W multiples of 8 in [8, 4096] required");
  if (!weights || !x0 || !y || !workspace) return fail(OMNISEG_ERR_ARG, "NULL argument");
  const bool dgrad = mode >= OMNISEG_CONV_DGRAD;
  if (!dgrad && !bias) return fail(OMNISEG_ERR_ARG, "bias is NULL");
  if (mode == OMNISEG_CONV_UPCAT_RELU) {
    if (!x1 || cu >= cin || height % 2 || width % 2) return fail(OMNISEG_ERR_ARG, "UPCAT needs x1, cu < cin and even H, W");
  } else if (cu != cin && mode != OMNISEG_CONV_DGRAD) {
    return fail(OMNISEG_ERR_ARG, "cu must equal cin outside UPCAT / DGRAD");
  }
  if ((mode == OMNISEG_CONV_RES_RELU || mode == OMNISEG_CONV_DGRAD_RES_MASK) && cin != cout)
    return fail(OMNISEG_ERR_ARG, "residual modes need cin == cout");
  if (mode == OMNISEG_CONV_DGRAD_RES_MASK && !aux) return fail(OMNISEG_ERR_ARG, "aux is NULL");
  {
    const int out_p = dgrad ? (cu < cin ? pad_ch(cu) + pad_ch(cin - cu) : pad_ch(cin)) : pad_ch(cout);
    if (config != -1 && !conv_config_valid(config, precision, height, width, out_p))
      return fail(OMNISEG_ERR_ARG, "conv config %d does not fit %dx%d with %d output channels", config, height, width, out_p);
    if (y_pool) {
      if (precision == OMNISEG_FP32) return fail(OMNISEG_ERR_UNSUPPORTED, "a pooled output needs BF16 or FP8");
      if (mode != OMNISEG_CONV_RES_RELU) return fail(OMNISEG_ERR_ARG, "a pooled output needs mode RES_RELU");
      const int32_t pst = pooled_conv_config(precision, config, height, width, out_p, &config);
      if (pst) return pst;
    }
  }
  if (per_image_bytes_too_big(mode, height, width, cin, precision))
    return fail(OMNISEG_ERR_UNSUPPORTED, "one image's input exceeds 2^31 bytes");
  if (ws_bytes < need) return fail(OMNISEG_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(OMNISEG_ERR_ARG, "workspace not 256-byte aligned");
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  char* ws = static_cast<char*>(workspace);
  int32_t* count = reinterpret_cast<int32_t*>(ws);
  const int cu_p = pad_ch(cu), cin_p = cu < cin ? cu_p + pad_ch(cin - cu) : pad_ch(cin), cout_p = pad_ch(cout);
  PackConv pc;
  pc.src = 0;
  pc.src_b = 0;
  pc.cout = cout;
  pc.cin = cin;
  pc.cu = cu;
  pc.cu_p = cu < cin ? cu_p : cin_p;
  pc.cin_p = cin_p;
  pc.cout_p = cout_p;
  pc.dst = 256;
  pc.dst_b = -1;  // the bias is copied separately below
  pc.transpose = dgrad ? 1 : 0;
  const int64_t off_b = 256 + align256((int64_t)cin_p * 9 * cout_p * elem_size(precision));
  HIP_TRY(launch_set_i32(count, n, sm));
  HIP_TRY(launch_pack_conv(precision, weights, ws, pc, sm));
  float* pb = reinterpret_cast<float*>(ws + off_b);
  if (!dgrad) {
    HIP_TRY(launch_zero(pb, (int64_t)cout_p * 4, sm));
    HIP_TRY(launch_copy_f32(bias, pb, cout, sm));
  }
  ConvLayer L;
  L.w = ws + 256;
  L.b = pb;
  if (dgrad) {
    L.cin_p = cout_p;
    L.cu_p = cout_p;
    L.cout_p = cin_p;
  } else {
    L.cin_p = cin_p;
    L.cu_p = pc.cu_p;
    L.cout_p = cout_p;
  }
  L.pool_out = y_pool;
  static const int loader_of[] = {LOAD_PLAIN, LOAD_PLAIN, LOAD_POOL, LOAD_UPCAT, LOAD_PLAIN, LOAD_PLAIN};
  static const int epi_of[] = {EPI_RELU, EPI_RES_RELU, EPI_RELU, EPI_RELU, EPI_NONE, EPI_RES_MASK};
  HIP_TRY(launch_conv3x3(precision, loader_of[mode], epi_of[mode], L, height, width, n, count, 0, x0, x1, y, sm, aux,
                         config));
  return OMNISEG_OK;
}

namespace {
struct Fp8ConvLayout {
  int cu_p, cin_p, cout_p, nch;
  int64_t w, b, ws, sin, oinv, total;
};
Fp8ConvLayout fp8_conv_layout(int cin, int cu, int cout) {
  Fp8ConvLayout f;
  f.cu_p = pad_ch(cu);
  f.cin_p = cu < cin ? f.cu_p + pad_ch(cin - cu) : pad_ch(cin);
  f.cout_p = pad_ch(cout);
  f.nch = ceil_div(f.cin_p, kFp8Chunk);
  f.w = 256;
  f.b = f.w + align256((int64_t)f.nch * kFp8Chunk * 9 * f.cout_p);
  f.ws = f.b + align256((int64_t)f.cout_p * 4);
  f.sin = f.ws + align256((int64_t)f.cout_p * 4);
  f.oinv = f.sin + align256((int64_t)f.cin_p * 4);
  f.total = f.oinv + align256((int64_t)f.cout_p * 4);
  return f;
}
}  // namespace

int32_t omniseg_conv3x3_fp8_workspace_bytes(int32_t cin, int32_t cu, int32_t cout, int64_t* bytes) {
  if (!bytes) return fail(OMNISEG_ERR_ARG, "bytes is NULL");
  if (cin < 1 || cout < 1 || cu < 1 || cu > cin || cin > 8192 || cout > 8192) return fail(OMNISEG_ERR_ARG, "bad channel counts");
  *bytes = fp8_conv_layout(cin, cu, cout).total;
  return OMNISEG_OK;
}

int32_t omniseg_conv3x3_fp8(int32_t mode, int32_t n, int32_t height, int32_t width, int32_t cin, int32_t cu,
                            int32_t cout, const float* weights, const float* bias, const float* in_scale,
                            const float* out_scale, const void* x0, const void* x1, void* y, void* y_pool,
                            int32_t config, void* workspace, int64_t ws_bytes, omniseg_stream stream) {
  int64_t need = 0;
  int32_t st = omniseg_conv3x3_fp8_workspace_bytes(cin, cu, cout, &need);
  if (st) return st;
  if (mode < OMNISEG_CONV_RELU || mode > OMNISEG_CONV_UPCAT_RELU)
    return fail(OMNISEG_ERR_UNSUPPORTED, "FP8 conv modes are RELU, RES_RELU, POOL_RELU and UPCAT_RELU");
  if (n < 1 || height < 16 || width < 16 || height % 16 || width % 16 || height > 4096 || width > 4096)
    return fail(OMNISEG_ERR_ARG, "n >= 1 and H, W multiples of 16 in [16, 4096] required");
  if (!weights || !bias || !in_scale || !out_scale || !x0 || !y || !workspace) return fail(OMNISEG_ERR_ARG, "NULL argument");
  if (mode == OMNISEG_CONV_UPCAT_RELU) {
    if (!x1 || cu >= cin) return fail(OMNISEG_ERR_ARG, "UPCAT needs x1 and cu < cin");
  } else if (cu != cin) {
    return fail(OMNISEG_ERR_ARG, "cu must equal cin outside UPCAT");
  }
  if (mode == OMNISEG_CONV_RES_RELU && cin != cout) return fail(OMNISEG_ERR_ARG, "RES_RELU needs cin == cout");
  const Fp8ConvLayout f = fp8_conv_layout(cin, cu, cout);
  if (config != -1 && !conv_config_valid(config, OMNISEG_FP8, height, width, f.cout_p))
    return fail(OMNISEG_ERR_ARG, "conv config %d does not run FP8 at %dx%d with %d output channels", config, height,
                width, f.cout_p);
  if (conv_default_config(OMNISEG_FP8, height, width, f.cout_p) < 0)
    return fail(OMNISEG_ERR_UNSUPPORTED, "no FP8 configuration fits %dx%d", height, width);
  if (y_pool && mode != OMNISEG_CONV_RES_RELU) return fail(OMNISEG_ERR_ARG, "a pooled output needs mode RES_RELU");
  if (per_image_bytes_too_big(mode, height, width, cin, OMNISEG_FP8))
    return fail(OMNISEG_ERR_UNSUPPORTED, "one image's input exceeds 2^31 bytes");
  if (ws_bytes < need) return fail(OMNISEG_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(OMNISEG_ERR_ARG, "workspace not 256-byte aligned");
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  char* ws = static_cast<char*>(workspace);
  int32_t* count = reinterpret_cast<int32_t*>(ws);
  float* s_in = reinterpret_cast<float*>(ws + f.sin);
  float* oinv = reinterpret_cast<float*>(ws + f.oinv);
  float* wscale = reinterpret_cast<float*>(ws + f.ws);
  HIP_TRY(launch_set_i32(count, n, sm));
  HIP_TRY(launch_fp8_conv_scales(in_scale, cin, cu, cu < cin ? f.cu_p : f.cin_p, f.cin_p, out_scale, cout, f.cout_p,
                                 s_in, oinv, sm));
  PackConv pc;
  pc.src = 0;
  pc.src_b = 0;
  pc.cout = cout;
  pc.cin = cin;
  pc.cu = cu;
  pc.cu_p = cu < cin ? f.cu_p : f.cin_p;
  pc.cin_p = f.cin_p;
  pc.cout_p = f.cout_p;
  pc.dst = f.w;
  pc.dst_b = -1;
  pc.transpose = 0;
  HIP_TRY(launch_pack_conv_fp8(weights, ws, pc, s_in, s_in + pc.cu_p, wscale, sm));
  HIP_TRY(launch_copy_f32(bias, reinterpret_cast<float*>(ws + f.b), cout, sm));
  if (f.cout_p > cout) HIP_TRY(launch_zero(ws + f.b + (int64_t)cout * 4, (int64_t)(f.cout_p - cout) * 4, sm));
  ConvLayer L;
  L.cin_p = f.cin_p;
  L.cu_p = pc.cu_p;
  L.cout_p = f.cout_p;
  L.w = ws + f.w;
  L.b = reinterpret_cast<const float*>(ws + f.b);
  L.wscale = wscale;
  L.rscale = s_in;
  L.oinv = oinv;
  L.pool_out = y_pool;
  static const int loader_of[] = {LOAD_PLAIN, LOAD_PLAIN, LOAD_POOL, LOAD_UPCAT};
  static const int epi_of[] = {EPI_RELU, EPI_RES_RELU, EPI_RELU, EPI_RELU};
  HIP_TRY(launch_conv3x3(OMNISEG_FP8, loader_of[mode], epi_of[mode], L, height, width, n, count, 0, x0, x1, y, sm,
                         nullptr, config));
  return OMNISEG_OK;
}

int32_t omniseg_stitch_workspace_bytes(int32_t tile, int32_t stride, int32_t height, int32_t width,
                                       int64_t* bytes) {
  if (!bytes) return fail(OMNISEG_ERR_ARG, "bytes is NULL");
  if (tile < 1 || tile > 4096 || stride < 1 || stride > tile || height < 1 || width < 1)
    return fail(OMNISEG_ERR_ARG, "bad stitch geometry");
  const int64_t ny = grid_count(height, tile, stride), nx = grid_count(width, tile, stride);
  if (ny * nx > (1LL << 30)) return fail(OMNISEG_ERR_UNSUPPORTED, "stitch grid of %lld tiles above 2^30", (long long)(ny * nx));
  *bytes = align256(ny * nx * 4);
  return OMNISEG_OK;
}

int32_t omniseg_stitch_tiles(int32_t tile, int32_t stride, int32_t height, int32_t width,
                             int32_t vote_threshold, const float* tile_logits, const int32_t* tile_yx, int32_t n_tiles,
                             uint8_t* mask, int64_t mask_pitch, float* logit, int64_t logit_pitch,
                             void* workspace, int64_t ws_bytes, omniseg_stream stream) {
  int64_t need = 0;
  int32_t st = omniseg_stitch_workspace_bytes(tile, stride, height, width, &need);
  if (st) return st;
  if (n_tiles < 0) return fail(OMNISEG_ERR_ARG, "n_tiles < 0");
  if (vote_threshold < 0) return fail(OMNISEG_ERR_ARG, "vote_threshold %d < 0", vote_threshold);
  if (n_tiles > 0 && (!tile_logits || !tile_yx)) return fail(OMNISEG_ERR_ARG, "tile arrays are NULL");
  if (!mask || mask_pitch < width) return fail(OMNISEG_ERR_ARG, "bad mask buffer");
  if (logit && logit_pitch < width) return fail(OMNISEG_ERR_ARG, "bad logit pitch");
  if (!workspace || ws_bytes < need) return fail(OMNISEG_ERR_WORKSPACE, "stitch workspace needs %lld bytes", (long long)need);
  const int ny = grid_count(height, tile, stride), nx = grid_count(width, tile, stride);
  if ((int64_t)n_tiles > (int64_t)ny * nx) return fail(OMNISEG_ERR_ARG, "more tiles than grid positions");
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  int32_t* grid = static_cast<int32_t*>(workspace);
  HIP_TRY(launch_grid_from_list(tile_yx, n_tiles, ny, nx, grid, sm));
  StitchArgs sa{};
  sa.logits = tile_logits;
  sa.tile_stride = (int64_t)tile * tile;
  sa.slot_off = 0;
  sa.index = grid;
  sa.ny = ny;
  sa.nx = nx;
  sa.T = tile;
  sa.s = stride;
  sa.Hk = height;
  sa.Wk = width;
  sa.mask = mask;
  sa.mask_pitch = mask_pitch;
  sa.logit = logit;
  sa.logit_pitch = logit_pitch;
  sa.fg = nullptr;
  sa.fg_shift = 0;
  sa.Hc = 0;
  sa.Wc = 0;
  sa.coverage = 0;
  sa.vote = vote_threshold;
  HIP_TRY(launch_stitch(sa, sm));
  return OMNISEG_OK;
}

}  // extern "C"

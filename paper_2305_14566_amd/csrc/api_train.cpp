// C ABI of the training path: forward over a tile batch with per-level
// checkpoints, the BCE loss, and the hand-written backward pass.
//
// Gradient flow (reverse of the forward):
//   stitch: dl_t = dLambda * w / D            head + precls: dtheta, dD_0
//   controller: dW_c, db_c, dg                bottleneck mean: dE_{L-1} += dg / hw
//   decoder level l = 0 .. L-2, encoder level l = L-1 .. 0, each:
//     recompute A = ReLU(conv_a(input))       (activation checkpointing)
//     dpre_b = dOut * [Out > 0]               dW_b, db_b from (A, dpre_b)
//     dpre_a = (conv_b^T dpre_b + dpre_b) * [A > 0]
//     dW_a, db_a from (input, dpre_a)         dInput = conv_a^T dpre_a
//   decoder dInput splits into the skip (dE_l) and the 2x2-summed upsampled
//   part (dD_{l+1}); encoder dInput goes through the max-pool to dE_{l-1}.
#include <algorithm>
#include <cstring>
#include <vector>

#include <climits>

#include "plan.h"

using namespace omniseg;

namespace {

struct TrainLayout {
  ScaleGeom geom[OMNISEG_MAX_SCALES];
  SlotTable slots;
  int max_slots = 0;
  int pair_slot[OMNISEG_MAX_CLASSES * OMNISEG_MAX_SCALES];
  int64_t plane_off[OMNISEG_MAX_CLASSES * OMNISEG_MAX_SCALES + 1];
  int n = 0;  // tiles
  int64_t off_tab, off_pad, off_pyr[OMNISEG_MAX_SCALES], off_list, off_count, off_grid[OMNISEG_MAX_SCALES];
  int64_t off_x, off_E[8], off_D[8], off_A, off_g, off_theta, off_logits;
  int64_t off_dl, off_dth_part, off_dth, off_dwp_part, off_sum_part, off_dg, off_dE[8], off_P, off_Q, off_Z, off_Dg[2];
  int64_t off_wpart, off_bpart, off_dd0;
  int64_t sz_level0, sz_wpart;
  int64_t total = 0;
};

constexpr int64_t kWgradPartBudget = 64LL << 20;  // bytes of split-K partials per conv

// Split count of the first conv's weight gradient over the batch's tile
// rows (a few rows per split).
int first_wgrad_splits(int64_t rows) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, rows / 4)); }

int wgrad_splits(int cout_p, int cin_p, int n_chunks) {
  const int blocks = (cout_p / wgrad_bo(cout_p)) * (cin_p / 32);
  int s = std::max(1, (1024 + blocks - 1) / blocks);
  const int64_t per = (int64_t)cout_p * 9 * cin_p * 4;
  s = (int)std::min<int64_t>(s, std::max<int64_t>(1, kWgradPartBudget / per));
  return std::min(s, std::max(1, n_chunks));
}

int32_t validate_train(const omniseg_plan* plan, const omniseg_slide* slide, const omniseg_tile* tiles,
                       int32_t n_tiles, const omniseg_pair* pairs, int32_t n_pairs, TrainLayout& lay) {
  if (!plan || !slide || !tiles || !pairs) return fail(OMNISEG_ERR_ARG, "NULL argument");
  const omniseg_config& c = plan->cfg;
  if (!(c.flags & OMNISEG_FLAG_TRAINING)) return fail(OMNISEG_ERR_ARG, "plan was created without OMNISEG_FLAG_TRAINING");
  if (plan->L < 2) return fail(OMNISEG_ERR_UNSUPPORTED, "training needs at least 2 U-Net levels");
  if (!slide->rgb || slide->height < 2 || slide->width < 2 || slide->row_pitch < 3LL * slide->width)
    return fail(OMNISEG_ERR_ARG, "bad slide");
  if (slide->height > (1 << 20) || slide->width > (1 << 20)) return fail(OMNISEG_ERR_UNSUPPORTED, "slide side above 2^20");
  if (n_tiles < 1 || n_tiles > OMNISEG_MAX_TRAIN_TILES)
    return fail(OMNISEG_ERR_ARG, "n_tiles %d outside [1, %d]", n_tiles, OMNISEG_MAX_TRAIN_TILES);
  if (n_pairs < 1 || n_pairs > c.n_classes * c.n_scales) return fail(OMNISEG_ERR_ARG, "bad n_pairs %d", n_pairs);
  for (int si = 0; si < c.n_scales; ++si)
    lay.geom[si] = make_geom(slide->height, slide->width, c.scale_log2[si], c.tile, c.stride);
  bool seen[OMNISEG_MAX_CLASSES][OMNISEG_MAX_SCALES] = {};
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) lay.slots.n_slots[si] = 0;
  lay.plane_off[0] = 0;
  for (int p = 0; p < n_pairs; ++p) {
    const int cl = pairs[p].cls, sc = pairs[p].scale;
    if (cl < 0 || cl >= c.n_classes || sc < 0 || sc >= c.n_scales) return fail(OMNISEG_ERR_ARG, "pair %d out of range", p);
    if (seen[cl][sc]) return fail(OMNISEG_ERR_ARG, "pair %d repeated", p);
    seen[cl][sc] = true;
    lay.pair_slot[p] = lay.slots.n_slots[sc];
    lay.slots.cls[sc][lay.slots.n_slots[sc]++] = cl;
    lay.plane_off[p + 1] = lay.plane_off[p] + (int64_t)lay.geom[sc].Hk * lay.geom[sc].Wk;
  }
  lay.max_slots = 0;
  for (int si = 0; si < c.n_scales; ++si) lay.max_slots = std::max(lay.max_slots, lay.slots.n_slots[si]);
  std::vector<char> used;
  for (int i = 0; i < n_tiles; ++i) {
    const omniseg_tile& t = tiles[i];
    if (t.scale < 0 || t.scale >= c.n_scales) return fail(OMNISEG_ERR_ARG, "tile %d: scale %d out of range", i, t.scale);
    const ScaleGeom& g = lay.geom[t.scale];
    if (t.jy < 0 || t.jy >= g.ny || t.jx < 0 || t.jx >= g.nx)
      return fail(OMNISEG_ERR_ARG, "tile %d: (%d, %d) outside the %dx%d grid", i, t.jy, t.jx, g.ny, g.nx);
    for (int j = 0; j < i; ++j)
      if (tiles[j].scale == t.scale && tiles[j].jy == t.jy && tiles[j].jx == t.jx)
        return fail(OMNISEG_ERR_ARG, "tile %d repeats tile %d", i, j);
  }
  lay.n = n_tiles;
  return OMNISEG_OK;
}

void train_layout(const omniseg_plan* plan, TrainLayout& lay) {
  const omniseg_config& c = plan->cfg;
  const int T = c.tile, n = lay.n, L = plan->L, es = elem_size(c.precision);
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off += align256(std::max<int64_t>(bytes, 1));
    return o;
  };
  lay.off_tab = take(sizeof(SlideDev));
  lay.off_pad = take(16);
  for (int si = 0; si < c.n_scales; ++si)
    lay.off_pyr[si] = lay.geom[si].k >= 1 ? take((int64_t)lay.geom[si].Ey * lay.geom[si].Ex * 8) : -1;
  lay.off_list = take((int64_t)n * 16);
  lay.off_count = take(4);
  for (int si = 0; si < c.n_scales; ++si) lay.off_grid[si] = take((int64_t)lay.geom[si].ny * lay.geom[si].nx * 4);
  const int64_t px0 = (int64_t)n * T * T;
  lay.off_x = take(px0 * 32 * 4);
  for (int l = 0; l < L; ++l) lay.off_E[l] = take(px0 / (1LL << (2 * l)) * plan->Cp[l] * es);
  for (int l = 0; l + 1 < L; ++l) lay.off_D[l] = take(px0 / (1LL << (2 * l)) * plan->Cp[l] * es);
  lay.sz_level0 = px0 * plan->Cp[0] * es;
  lay.off_A = take(lay.sz_level0);
  lay.off_g = take((int64_t)n * plan->Cp[L - 1] * 4);
  lay.off_theta = take((int64_t)n * lay.max_slots * plan->P * 4);
  lay.off_logits = take(px0 * lay.max_slots * 4);
  // backward
  const int per = T * T / 256;
  lay.off_dl = take(px0 * lay.max_slots * 4);
  lay.off_dth_part = take((int64_t)n * lay.max_slots * per * plan->P * 4);
  lay.off_dth = take((int64_t)n * lay.max_slots * plan->P * 4);
  lay.off_dwp_part = take((int64_t)n * per * (8 * plan->C[0] + 8) * 4);
  lay.off_sum_part = take(4 * std::max(sum_mid_part_floats(n * lay.max_slots, per, plan->P),
                                       sum_mid_part_floats(1, n * per, 8 * plan->C[0] + 8)));
  lay.off_dg = take((int64_t)n * plan->Cp[L - 1] * 4);
  lay.off_dd0 = take(lay.sz_level0);
  for (int l = 0; l < L; ++l) lay.off_dE[l] = take(px0 / (1LL << (2 * l)) * plan->Cp[l] * es);
  lay.off_P = take(lay.sz_level0);
  lay.off_Q = take(lay.sz_level0);
  // dZ of the decoder's first conv (2 C_l + C_l channels) or the encoder's dX
  int64_t zmax = 0;
  for (int l = 0; l + 1 < L; ++l) zmax = std::max<int64_t>(zmax, px0 / (1LL << (2 * l)) * (plan->Cp[l + 1] + plan->Cp[l]) * es);
  lay.off_Z = take(std::max(zmax, lay.sz_level0));
  lay.off_Dg[0] = take(lay.sz_level0);
  lay.off_Dg[1] = take(lay.sz_level0);
  // split-K partials of the largest weight gradient
  int64_t wmax = 0;
  auto acc_w = [&](const ConvDesc& d, int h) {
    const int chunks = n * (h / 8) * (h / (h % 16 == 0 ? 16 : 8));
    const int s = wgrad_splits(d.cout_p, d.cin_p, chunks);
    wmax = std::max(wmax, (int64_t)s * d.cout_p * 9 * d.cin_p * 4);
  };
  // the first conv: splits x cout_p x 9 taps x 4 (3 channels padded)
  wmax = std::max(wmax, (int64_t)first_wgrad_splits((int64_t)n * T) * plan->Cp[0] * 9 * 4 * 4);
  for (int l = 0; l < L; ++l) {
    if (l > 0) acc_w(plan->enc_a[l], T >> l);
    acc_w(plan->enc_b[l], T >> l);
  }
  for (int l = 0; l + 1 < L; ++l) {
    acc_w(plan->dec_a[l], T >> l);
    acc_w(plan->dec_b[l], T >> l);
  }
  lay.sz_wpart = wmax;
  lay.off_wpart = take(wmax);
  lay.off_bpart = take((int64_t)kBiasGradSplits * 4096 * 4);
  lay.total = off;
}

ConvLayer fwd_layer(const char* pk, const ConvDesc& d) {
  ConvLayer L;
  L.cin_p = d.cin_p;
  L.cu_p = d.cu_p;
  L.cout_p = d.cout_p;
  L.w = pk + d.pk_w;
  L.b = reinterpret_cast<const float*>(pk + d.pk_b);
  return L;
}

// the data-gradient conv: input = forward output channels, output = forward input channels
ConvLayer bwd_layer(const char* pk, const ConvDesc& d) {
  ConvLayer L;
  L.cin_p = d.cout_p;
  L.cu_p = d.cout_p;
  L.cout_p = d.cin_p;
  L.w = pk + d.pk_wt;
  L.b = reinterpret_cast<const float*>(pk + d.pk_b);  // not read by the gradient epilogues
  return L;
}

// Shared set-up of both calls: slide table, tile list, grids.
int32_t upload_tables(const omniseg_plan* plan, const omniseg_slide* slide, const omniseg_tile* tiles,
                      const TrainLayout& lay, char* ws, hipStream_t sm) {
  const omniseg_config& c = plan->cfg;
  plan->slide_tab.assign(1, SlideDev());
  SlideDev& d = plan->slide_tab[0];
  d.rgb = slide->rgb;
  d.pitch = slide->row_pitch;
  d.H = slide->height;
  d.W = slide->width;
  d.pad = reinterpret_cast<const int32_t*>(ws + lay.off_pad);
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) {
    d.pyr[si] = (si < c.n_scales && lay.off_pyr[si] >= 0) ? reinterpret_cast<const uint16_t*>(ws + lay.off_pyr[si]) : nullptr;
    d.pyr_ex[si] = si < c.n_scales ? lay.geom[si].Ex : 0;
  }
  d.fg = nullptr;
  d.Hc = d.Wc = 0;
  HIP_TRY(hipMemcpyAsync(ws + lay.off_tab, plan->slide_tab.data(), sizeof(SlideDev), hipMemcpyHostToDevice, sm));
  // tile list (slide 0, slot, jy, jx), count, then one grid per slot
  std::vector<int32_t>& h = plan->host_tab;
  int64_t words = 4LL * lay.n + 1;
  for (int si = 0; si < c.n_scales; ++si) words += (int64_t)lay.geom[si].ny * lay.geom[si].nx;
  h.assign(words, -1);
  for (int i = 0; i < lay.n; ++i) {
    h[4 * i] = 0;
    h[4 * i + 1] = tiles[i].scale;
    h[4 * i + 2] = tiles[i].jy;
    h[4 * i + 3] = tiles[i].jx;
  }
  h[4 * lay.n] = lay.n;
  int64_t pos = 4LL * lay.n + 1;
  int64_t gpos[OMNISEG_MAX_SCALES];
  for (int si = 0; si < c.n_scales; ++si) {
    gpos[si] = pos;
    pos += (int64_t)lay.geom[si].ny * lay.geom[si].nx;
  }
  for (int i = 0; i < lay.n; ++i) {
    const omniseg_tile& t = tiles[i];
    h[gpos[t.scale] + (int64_t)t.jy * lay.geom[t.scale].nx + t.jx] = i;
  }
  HIP_TRY(hipMemcpyAsync(ws + lay.off_list, h.data(), 16LL * lay.n, hipMemcpyHostToDevice, sm));
  HIP_TRY(hipMemcpyAsync(ws + lay.off_count, h.data() + 4 * lay.n, 4, hipMemcpyHostToDevice, sm));
  for (int si = 0; si < c.n_scales; ++si)
    HIP_TRY(hipMemcpyAsync(ws + lay.off_grid[si], h.data() + gpos[si], 4LL * lay.geom[si].ny * lay.geom[si].nx,
                           hipMemcpyHostToDevice, sm));
  return OMNISEG_OK;
}

FirstConvArgs first_args(const omniseg_plan* plan, const char* pk, const TrainLayout& lay, char* ws, void* y) {
  const omniseg_config& c = plan->cfg;
  FirstConvArgs fa{};
  fa.list = reinterpret_cast<const int32_t*>(ws + lay.off_list);
  fa.count = reinterpret_cast<const int32_t*>(ws + lay.off_count);
  fa.chunk_base = 0;
  fa.batch = lay.n;
  fa.T = c.tile;
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) fa.scale_s[si] = c.stride;  // training plans: one stride
  fa.w = reinterpret_cast<const float*>(pk + plan->pk_first_w);
  fa.b = reinterpret_cast<const float*>(pk + plan->pk_first_b);
  fa.c0 = plan->C[0];
  fa.c0_p = plan->Cp[0];
  fa.y = y;
  fa.slides = reinterpret_cast<const SlideDev*>(ws + lay.off_tab);
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) fa.scale_k[si] = si < c.n_scales ? c.scale_log2[si] : 0;
  return fa;
}

int32_t check_common(const omniseg_plan* plan, const void* packed, void* workspace, int64_t ws_bytes,
                     const TrainLayout& lay) {
  if (!packed || !workspace) return fail(OMNISEG_ERR_ARG, "NULL packed weights or workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 || reinterpret_cast<uintptr_t>(packed) % 256)
    return fail(OMNISEG_ERR_ARG, "workspace and packed weights must be 256-byte aligned");
  if (ws_bytes < lay.total)
    return fail(OMNISEG_ERR_WORKSPACE, "workspace has %lld bytes, needs %lld", (long long)ws_bytes, (long long)lay.total);
  (void)plan;
  return OMNISEG_OK;
}

}  // namespace

extern "C" {

int32_t omniseg_plane_offsets(const omniseg_plan* plan, const omniseg_slide* slide, const omniseg_pair* pairs,
                              int32_t n_pairs, int64_t* offsets) {
  if (!plan || !slide || !pairs || !offsets) return fail(OMNISEG_ERR_ARG, "NULL argument");
  const omniseg_config& c = plan->cfg;
  if (n_pairs < 1 || n_pairs > c.n_classes * c.n_scales) return fail(OMNISEG_ERR_ARG, "bad n_pairs %d", n_pairs);
  if (slide->height < 1 || slide->width < 1) return fail(OMNISEG_ERR_ARG, "bad slide size");
  offsets[0] = 0;
  for (int p = 0; p < n_pairs; ++p) {
    if (pairs[p].scale < 0 || pairs[p].scale >= c.n_scales) return fail(OMNISEG_ERR_ARG, "pair %d: bad scale", p);
    const int k = c.scale_log2[pairs[p].scale];
    offsets[p + 1] = offsets[p] + (int64_t)ceil_div(slide->height, 1 << k) * ceil_div(slide->width, 1 << k);
  }
  return OMNISEG_OK;
}

int32_t omniseg_train_workspace_bytes(const omniseg_plan* plan, const omniseg_slide* slide,
                                      const omniseg_tile* tiles, int32_t n_tiles, const omniseg_pair* pairs,
                                      int32_t n_pairs, int64_t* bytes) {
  if (!bytes) return fail(OMNISEG_ERR_ARG, "bytes is NULL");
  TrainLayout lay;
  int32_t st = validate_train(plan, slide, tiles, n_tiles, pairs, n_pairs, lay);
  if (st) return st;
  train_layout(plan, lay);
  *bytes = lay.total;
  return OMNISEG_OK;
}

int32_t omniseg_train_forward(const omniseg_plan* plan, const void* packed, const omniseg_slide* slide,
                              const omniseg_tile* tiles, int32_t n_tiles, const omniseg_pair* pairs,
                              int32_t n_pairs, float* logit, uint8_t* covered, void* workspace,
                              int64_t ws_bytes, omniseg_stream stream) {
  TrainLayout lay;
  int32_t st = validate_train(plan, slide, tiles, n_tiles, pairs, n_pairs, lay);
  if (st) return st;
  if (!logit || !covered) return fail(OMNISEG_ERR_ARG, "NULL output planes");
  train_layout(plan, lay);
  st = check_common(plan, packed, workspace, ws_bytes, lay);
  if (st) return st;

  const omniseg_config& c = plan->cfg;
  (void)hipGetLastError();  // launches below report their own errors, not stale ones
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const char* pk = static_cast<const char*>(packed);
  const int T = c.tile, s = c.stride, prec = c.precision, L = plan->L, n = lay.n;
  st = upload_tables(plan, slide, tiles, lay, ws, sm);
  if (st) return st;
  int32_t* pad = reinterpret_cast<int32_t*>(ws + lay.off_pad);
  HIP_TRY(launch_pad_colour(slide->rgb, slide->row_pitch, pad, sm));
  {
    uint16_t* lvl[4] = {nullptr, nullptr, nullptr, nullptr};
    int Ey[4] = {0, 0, 0, 0}, Ex[4] = {0, 0, 0, 0};
    int kmax = 0;
    for (int si = 0; si < c.n_scales; ++si) {
      const ScaleGeom& g = lay.geom[si];
      kmax = std::max(kmax, g.k);
      if (g.k >= 1) {
        lvl[g.k] = reinterpret_cast<uint16_t*>(ws + lay.off_pyr[si]);
        Ey[g.k] = g.Ey;
        Ex[g.k] = g.Ex;
      }
    }
    HIP_TRY(launch_pyramid(slide->rgb, slide->row_pitch, slide->height, slide->width, pad, kmax, lvl, Ey, Ex, sm));
  }
  const int32_t* list = reinterpret_cast<const int32_t*>(ws + lay.off_list);
  const int32_t* count = reinterpret_cast<const int32_t*>(ws + lay.off_count);
  void* A = ws + lay.off_A;
  void* E[8];
  void* D[8];
  for (int l = 0; l < L; ++l) E[l] = ws + lay.off_E[l];
  for (int l = 0; l + 1 < L; ++l) D[l] = ws + lay.off_D[l];
  float* g = reinterpret_cast<float*>(ws + lay.off_g);
  float* theta = reinterpret_cast<float*>(ws + lay.off_theta);
  float* tlog = reinterpret_cast<float*>(ws + lay.off_logits);

  FirstConvArgs fa = first_args(plan, pk, lay, ws, A);
  HIP_TRY(launch_input_x(fa, reinterpret_cast<float*>(ws + lay.off_x), sm));
  HIP_TRY(launch_first_conv(prec, fa, sm));
  HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, fwd_layer(pk, plan->enc_b[0]), T, T, n, count, 0, A, nullptr, E[0], sm,
                         nullptr, layer_config(plan, 1, 0, T, T, plan->enc_b[0].cout_p)));
  for (int l = 1; l < L; ++l) {
    const int tl = T >> l;
    HIP_TRY(launch_conv3x3(prec, LOAD_POOL, EPI_RELU, fwd_layer(pk, plan->enc_a[l]), tl, tl, n, count, 0, E[l - 1], nullptr, A, sm,
                           nullptr, layer_config(plan, 0, l, tl, tl, plan->enc_a[l].cout_p)));
    HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, fwd_layer(pk, plan->enc_b[l]), tl, tl, n, count, 0, A, nullptr, E[l], sm,
                           nullptr, layer_config(plan, 1, l, tl, tl, plan->enc_b[l].cout_p)));
  }
  const int tb = T >> (L - 1);
  HIP_TRY(launch_gap(prec, E[L - 1], n, tb * tb, plan->Cp[L - 1], plan->G, count, 0, g, sm));
  HIP_TRY(launch_controller(g, n, plan->G, reinterpret_cast<const float*>(pk + plan->pk_ctrl_w),
                            reinterpret_cast<const float*>(pk + plan->pk_ctrl_b), plan->P, c.n_classes, c.n_scales,
                            lay.slots, lay.max_slots, list, count, 0, theta, sm));
  for (int l = L - 2; l >= 0; --l) {
    const int tl = T >> l;
    const void* below = (l + 1 == L - 1) ? E[L - 1] : D[l + 1];
    HIP_TRY(launch_conv3x3(prec, LOAD_UPCAT, EPI_RELU, fwd_layer(pk, plan->dec_a[l]), tl, tl, n, count, 0, below, E[l], A, sm,
                           nullptr, layer_config(plan, 2, l, tl, tl, plan->dec_a[l].cout_p)));
    HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_RELU, fwd_layer(pk, plan->dec_b[l]), tl, tl, n, count, 0, A, nullptr, D[l], sm,
                           nullptr, layer_config(plan, 3, l, tl, tl, plan->dec_b[l].cout_p)));
  }
  const void* d0 = L >= 2 ? D[0] : E[0];
  HIP_TRY(launch_head(prec, d0, n, T, plan->C[0], plan->Cp[0],
                      plan->canon_pre_w >= 0 ? reinterpret_cast<const float*>(pk + plan->pk_pre_w) : nullptr,
                      plan->canon_pre_w >= 0 ? reinterpret_cast<const float*>(pk + plan->pk_pre_b) : nullptr, theta,
                      plan->P, c.head_out, lay.slots, lay.max_slots, list, count, 0, 0, tlog, sm));
  for (int p = 0; p < n_pairs; ++p) {
    const int si = pairs[p].scale;
    const ScaleGeom& gm = lay.geom[si];
    StitchArgs sa{};
    sa.logits = tlog;
    sa.tile_stride = (int64_t)lay.max_slots * T * T;
    sa.slot_off = (int64_t)lay.pair_slot[p] * T * T;
    sa.index = reinterpret_cast<const int32_t*>(ws + lay.off_grid[si]);
    sa.ny = gm.ny;
    sa.nx = gm.nx;
    sa.T = T;
    sa.s = s;
    sa.Hk = gm.Hk;
    sa.Wk = gm.Wk;
    sa.mask = covered + lay.plane_off[p];
    sa.mask_pitch = gm.Wk;
    sa.logit = logit + lay.plane_off[p];
    sa.logit_pitch = gm.Wk;
    sa.fg = nullptr;
    sa.fg_shift = 0;
    sa.Hc = sa.Wc = 0;
    sa.coverage = 1;
    HIP_TRY(launch_stitch(sa, sm));
  }
  return OMNISEG_OK;
}

int32_t omniseg_backward(const omniseg_plan* plan, const void* packed, const omniseg_slide* slide,
                         const omniseg_tile* tiles, int32_t n_tiles, const omniseg_pair* pairs, int32_t n_pairs,
                         const float* grad_logit, float* grad_weights, void* workspace, int64_t ws_bytes,
                         omniseg_stream stream) {
  TrainLayout lay;
  int32_t st = validate_train(plan, slide, tiles, n_tiles, pairs, n_pairs, lay);
  if (st) return st;
  if (!grad_logit || !grad_weights) return fail(OMNISEG_ERR_ARG, "NULL gradient buffer");
  train_layout(plan, lay);
  st = check_common(plan, packed, workspace, ws_bytes, lay);
  if (st) return st;

  const omniseg_config& c = plan->cfg;
  (void)hipGetLastError();  // launches below report their own errors, not stale ones
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const char* pk = static_cast<const char*>(packed);
  const int T = c.tile, s = c.stride, prec = c.precision, L = plan->L, n = lay.n, es = elem_size(prec);
  const int per = T * T / 256;
  // the slide table, tile list and grids are still in the workspace from the forward
  const int32_t* list = reinterpret_cast<const int32_t*>(ws + lay.off_list);
  const int32_t* count = reinterpret_cast<const int32_t*>(ws + lay.off_count);
  void* A = ws + lay.off_A;
  void* E[8];
  void* D[8];
  void* dE[8];
  for (int l = 0; l < L; ++l) {
    E[l] = ws + lay.off_E[l];
    dE[l] = ws + lay.off_dE[l];
  }
  for (int l = 0; l + 1 < L; ++l) D[l] = ws + lay.off_D[l];
  void* bufP = ws + lay.off_P;
  void* bufQ = ws + lay.off_Q;
  void* bufZ = ws + lay.off_Z;
  void* bufD[2] = {ws + lay.off_Dg[0], ws + lay.off_Dg[1]};
  float* wpart = reinterpret_cast<float*>(ws + lay.off_wpart);
  float* bpart = reinterpret_cast<float*>(ws + lay.off_bpart);
  float* gw = grad_weights;

  // 1. stitch backward
  StitchBwdArgs sb{};
  sb.dlam = grad_logit;
  sb.dl = reinterpret_cast<float*>(ws + lay.off_dl);
  sb.list = list;
  sb.n_tiles = n;
  sb.T = T;
  sb.s = s;
  sb.max_slots = lay.max_slots;
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) {
    const bool u = si < c.n_scales;
    sb.ny[si] = u ? lay.geom[si].ny : 0;
    sb.nx[si] = u ? lay.geom[si].nx : 0;
    sb.Hk[si] = u ? lay.geom[si].Hk : 0;
    sb.Wk[si] = u ? lay.geom[si].Wk : 0;
    sb.grid[si] = u ? reinterpret_cast<const int32_t*>(ws + lay.off_grid[si]) : nullptr;
    sb.n_slots[si] = lay.slots.n_slots[si];
    for (int j = 0; j < OMNISEG_MAX_CLASSES; ++j) sb.plane_off[si][j] = 0;
  }
  for (int p = 0; p < n_pairs; ++p) sb.plane_off[pairs[p].scale][lay.pair_slot[p]] = lay.plane_off[p];
  HIP_TRY(launch_stitch_bwd(sb, sm));

  // 2. head and precls backward
  HeadBwdArgs hb{};
  hb.d0 = L >= 2 ? D[0] : E[0];
  hb.theta = reinterpret_cast<const float*>(ws + lay.off_theta);
  hb.dl = sb.dl;
  hb.wp = plan->canon_pre_w >= 0 ? reinterpret_cast<const float*>(pk + plan->pk_pre_w) : nullptr;
  hb.bp = plan->canon_pre_w >= 0 ? reinterpret_cast<const float*>(pk + plan->pk_pre_b) : nullptr;
  hb.list = list;
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) hb.n_slots[si] = lay.slots.n_slots[si];
  hb.n_tiles = n;
  hb.T = T;
  hb.c0 = plan->C[0];
  hb.c0_p = plan->Cp[0];
  hb.o = c.head_out;
  hb.max_slots = lay.max_slots;
  hb.dtheta_part = reinterpret_cast<float*>(ws + lay.off_dth_part);
  hb.dwp_part = reinterpret_cast<float*>(ws + lay.off_dwp_part);
  hb.dd0 = ws + lay.off_dd0;
  hb.mask_d0 = L >= 2 ? 1 : 0;  // D_0 is the decoder's ReLU output: its gradient leaves masked
  HIP_TRY(launch_head_bwd(prec, hb, sm));
  float* dtheta = reinterpret_cast<float*>(ws + lay.off_dth);
  float* sum_part = reinterpret_cast<float*>(ws + lay.off_sum_part);
  HIP_TRY(launch_sum_mid(hb.dtheta_part, n * lay.max_slots, per, plan->P, dtheta, sum_part, sm));
  if (plan->canon_pre_w >= 0)  // precls W then b are contiguous in canonical order
    HIP_TRY(launch_sum_mid(hb.dwp_part, 1, n * per, 8 * plan->C[0] + 8, gw + plan->canon_pre_w, sum_part, sm));

  // 3. controller backward
  CtrlBwdArgs cb{};
  cb.dtheta = dtheta;
  cb.g = reinterpret_cast<const float*>(ws + lay.off_g);
  cb.wc = reinterpret_cast<const float*>(pk + plan->pk_ctrl_w);
  cb.list = list;
  for (int si = 0; si < OMNISEG_MAX_SCALES; ++si) {
    cb.n_slots[si] = lay.slots.n_slots[si];
    for (int j = 0; j < OMNISEG_MAX_CLASSES; ++j) cb.cls[si][j] = lay.slots.cls[si][j];
  }
  cb.n_tiles = n;
  cb.max_slots = lay.max_slots;
  cb.P = plan->P;
  cb.G = plan->G;
  cb.g_stride = plan->Cp[L - 1];
  cb.n_classes = c.n_classes;
  cb.row_len = plan->G + c.n_classes + c.n_scales;
  cb.dwc = gw + plan->canon_ctrl_w;
  cb.dbc = gw + plan->canon_ctrl_b;
  cb.dg = reinterpret_cast<float*>(ws + lay.off_dg);
  HIP_TRY(launch_ctrl_bwd(cb, sm));

  // 4. level gradients start at zero; the bottleneck gets the mean's gradient
  for (int l = 0; l + 1 < L; ++l)
    HIP_TRY(launch_zero(dE[l], (int64_t)n * (T >> l) * (T >> l) * plan->Cp[l] * es, sm));
  const int tb = T >> (L - 1);
  HIP_TRY(launch_gap_bwd(prec, cb.dg, plan->Cp[L - 1], plan->G, tb * tb, plan->Cp[L - 1], n, dE[L - 1], sm));

  auto wgrad = [&](const ConvDesc& d, int loader, int px, const void* x0, const void* x1, const void* dy, int h,
                   int cin_real, int cin_p, int cu, int cu_p, float* dst) -> int32_t {
    WgradArgs wa{};
    wa.x0 = x0;
    wa.x1 = x1;
    wa.dy = dy;
    wa.part = wpart;
    wa.H = h;
    wa.W = h;
    wa.cin_p = cin_p;
    wa.cu_p = cu_p;
    wa.cout_p = d.cout_p;
    wa.n_tiles = n;
    const int chunks = n * (h / 8) * (h / (h % 16 == 0 ? 16 : 8));
    wa.splits = wgrad_splits(d.cout_p, cin_p, chunks);
    HIP_TRY(launch_wgrad(px, prec, loader, wa, d.cout, cin_real, cu, dst, sm));
    return OMNISEG_OK;
  };
  auto bias = [&](const ConvDesc& d, const void* dy, int h, float* dst) -> int32_t {
    HIP_TRY(launch_bias_grad(prec, dy, (int64_t)n * h * h, d.cout_p, d.cout, bpart,
                             bias_grad_splits((int64_t)n * h * h), dst, sm));
    return OMNISEG_OK;
  };
#define OMNISEG_CALL(x)      \
  do {                       \
    int32_t r_ = (x);        \
    if (r_) return r_;       \
  } while (0)

  // 5. decoder levels, from the output inwards
  const void* dcur = ws + lay.off_dd0;
  for (int l = 0; l + 1 < L; ++l) {
    const int tl = T >> l;
    const ConvDesc& da = plan->dec_a[l];
    const ConvDesc& db = plan->dec_b[l];
    const void* below = (l + 1 == L - 1) ? E[L - 1] : D[l + 1];
    HIP_TRY(launch_conv3x3(prec, LOAD_UPCAT, EPI_RELU, fwd_layer(pk, da), tl, tl, n, count, 0, below, E[l], A, sm));
    // dcur is already the gradient through the ReLU of D_l (the head's
    // backward or the level below's concat backward applied the mask)
    const void* gD = dcur;
    OMNISEG_CALL(wgrad(db, LOAD_PLAIN, prec, A, nullptr, gD, tl, db.cin, db.cin_p, db.cu, db.cu_p, gw + db.canon_w));
    OMNISEG_CALL(bias(db, gD, tl, gw + db.canon_b));
    HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_MASK, bwd_layer(pk, db), tl, tl, n, count, 0, gD, nullptr, bufQ, sm, A));
    OMNISEG_CALL(wgrad(da, LOAD_UPCAT, prec, below, E[l], bufQ, tl, da.cin, da.cin_p, da.cu, da.cu_p, gw + da.canon_w));
    OMNISEG_CALL(bias(da, bufQ, tl, gw + da.canon_b));
    HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_NONE, bwd_layer(pk, da), tl, tl, n, count, 0, bufQ, nullptr, bufZ, sm));
    const bool last = (l + 1 == L - 1);
    void* dnext = last ? dE[L - 1] : bufD[(l + 1) & 1];
    HIP_TRY(launch_concat_bwd(prec, bufZ, n, tl, tl, da.cu_p, plan->Cp[l], dE[l], dnext, last ? 1 : 0,
                              last ? nullptr : D[l + 1], sm));
    dcur = dnext;
  }
  // 6. encoder levels, from the bottleneck outwards
  for (int l = L - 1; l >= 0; --l) {
    const int tl = T >> l;
    const int64_t npx = (int64_t)n * tl * tl;
    const ConvDesc& eb = plan->enc_b[l];
    if (l == 0) {
      FirstConvArgs fa = first_args(plan, pk, lay, ws, A);
      HIP_TRY(launch_first_conv(prec, fa, sm));
    } else {
      HIP_TRY(launch_conv3x3(prec, LOAD_POOL, EPI_RELU, fwd_layer(pk, plan->enc_a[l]), tl, tl, n, count, 0, E[l - 1], nullptr, A, sm));
    }
    // below the bottleneck the max-pool backward of level l + 1 stored dE_l
    // through the ReLU of E_l already
    const void* gE = dE[l];
    if (l == L - 1) {
      HIP_TRY(launch_relu_mask(prec, dE[l], E[l], npx * plan->Cp[l], bufP, sm));
      gE = bufP;
    }
    OMNISEG_CALL(wgrad(eb, LOAD_PLAIN, prec, A, nullptr, gE, tl, eb.cin, eb.cin_p, eb.cu, eb.cu_p, gw + eb.canon_w));
    OMNISEG_CALL(bias(eb, gE, tl, gw + eb.canon_b));
    HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_RES_MASK, bwd_layer(pk, eb), tl, tl, n, count, 0, gE, nullptr, bufQ, sm, A));
    if (l == 0) {
      ConvDesc d0{};
      d0.cout = plan->C[0];
      d0.cout_p = plan->Cp[0];
      // 3 input channels: a kernel of its own rather than the 32-channel one
      HIP_TRY(launch_wgrad_first(prec, reinterpret_cast<const float*>(ws + lay.off_x), 32, bufQ, n, T, d0.cout,
                                 d0.cout_p, wpart, first_wgrad_splits((int64_t)n * T),
                                 gw + plan->canon_first_w, sm));
      OMNISEG_CALL(bias(d0, bufQ, T, gw + plan->canon_first_b));
    } else {
      const ConvDesc& ea = plan->enc_a[l];
      OMNISEG_CALL(wgrad(ea, LOAD_POOL, prec, E[l - 1], nullptr, bufQ, tl, ea.cin, ea.cin_p, ea.cu, ea.cu_p, gw + ea.canon_w));
      OMNISEG_CALL(bias(ea, bufQ, tl, gw + ea.canon_b));
      HIP_TRY(launch_conv3x3(prec, LOAD_PLAIN, EPI_NONE, bwd_layer(pk, ea), tl, tl, n, count, 0, bufQ, nullptr, bufZ, sm));
      HIP_TRY(launch_maxpool_bwd(prec, E[l - 1], bufZ, n, 2 * tl, 2 * tl, plan->Cp[l - 1], dE[l - 1], sm, 1));
    }
  }
#undef OMNISEG_CALL
  return OMNISEG_OK;
}

namespace {
struct WgradGeom {
  int cin_p, cu_p, cout_p, chunks, splits;
};
int32_t wgrad_geom(int32_t n, int32_t height, int32_t width, int32_t cin, int32_t cu, int32_t cout, WgradGeom* g) {
  if (n < 1 || height < 8 || width < 8 || height % 8 || width % 8 || height > 4096 || width > 4096)
    return fail(OMNISEG_ERR_ARG, "n >= 1 and H, W multiples of 8 in [8, 4096] required");
  if (cin < 1 || cout < 1 || cu < 1 || cu > cin || cin > 8192 || cout > 8192) return fail(OMNISEG_ERR_ARG, "bad channel counts");
  g->cu_p = pad_ch(cu);
  g->cin_p = cu < cin ? g->cu_p + pad_ch(cin - cu) : pad_ch(cin);
  g->cout_p = pad_ch(cout);
  const int64_t chunks = (int64_t)n * (height / 8) * (width / (width % 16 == 0 ? 16 : 8));
  if (chunks > INT32_MAX) return fail(OMNISEG_ERR_UNSUPPORTED, "too many pixel blocks");
  g->chunks = (int)chunks;
  g->splits = wgrad_splits(g->cout_p, g->cin_p, g->chunks);
  return OMNISEG_OK;
}
}  // namespace

int32_t omniseg_conv3x3_wgrad_workspace_bytes(int32_t n, int32_t height, int32_t width, int32_t cin, int32_t cu,
                                              int32_t cout, int64_t* bytes) {
  if (!bytes) return fail(OMNISEG_ERR_ARG, "bytes is NULL");
  WgradGeom g;
  const int32_t st = wgrad_geom(n, height, width, cin, cu, cout, &g);
  if (st) return st;
  *bytes = align256((int64_t)g.splits * g.cout_p * 9 * g.cin_p * 4);
  return OMNISEG_OK;
}

int32_t omniseg_conv3x3_wgrad(int32_t precision, int32_t mode, int32_t n, int32_t height, int32_t width, int32_t cin,
                              int32_t cu, int32_t cout, const void* x0, const void* x1, const void* dy, float* dw,
                              void* workspace, int64_t ws_bytes, omniseg_stream stream) {
  if (precision != OMNISEG_FP32 && precision != OMNISEG_BF16) return fail(OMNISEG_ERR_UNSUPPORTED, "precision %d", precision);
  int loader;
  if (mode == OMNISEG_CONV_RELU) loader = LOAD_PLAIN;
  else if (mode == OMNISEG_CONV_POOL_RELU) loader = LOAD_POOL;
  else if (mode == OMNISEG_CONV_UPCAT_RELU) loader = LOAD_UPCAT;
  else return fail(OMNISEG_ERR_ARG, "mode %d: RELU, POOL_RELU or UPCAT_RELU", mode);
  WgradGeom g;
  int32_t st = wgrad_geom(n, height, width, cin, cu, cout, &g);
  if (st) return st;
  if (loader == LOAD_UPCAT) {
    if (!x1 || cu >= cin || height % 2 || width % 2) return fail(OMNISEG_ERR_ARG, "UPCAT needs x1, cu < cin and even H, W");
  } else if (cu != cin) {
    return fail(OMNISEG_ERR_ARG, "cu must equal cin outside UPCAT");
  }
  if (!x0 || !dy || !dw || !workspace) return fail(OMNISEG_ERR_ARG, "NULL argument");
  if (ws_bytes < (int64_t)g.splits * g.cout_p * 9 * g.cin_p * 4) return fail(OMNISEG_ERR_WORKSPACE, "workspace too small");
  (void)hipGetLastError();
  WgradArgs wa{};
  wa.x0 = x0;
  wa.x1 = x1;
  wa.dy = dy;
  wa.part = static_cast<float*>(workspace);
  wa.H = height;
  wa.W = width;
  wa.cin_p = g.cin_p;
  wa.cu_p = loader == LOAD_UPCAT ? g.cu_p : g.cin_p;
  wa.cout_p = g.cout_p;
  wa.n_tiles = n;
  wa.splits = g.splits;
  HIP_TRY(launch_wgrad(precision, precision, loader, wa, cout, cin, loader == LOAD_UPCAT ? cu : cin, dw,
                       reinterpret_cast<hipStream_t>(stream)));
  return OMNISEG_OK;
}

int32_t omniseg_bce_loss(const float* logit, const float* target, const uint8_t* valid, int64_t n, double* loss,
                         float* grad, void* workspace, int64_t ws_bytes, omniseg_stream stream) {
  if (!logit || !target || !valid || !loss || !workspace) return fail(OMNISEG_ERR_ARG, "NULL argument");
  if (n < 1) return fail(OMNISEG_ERR_ARG, "n < 1");
  if (ws_bytes < 16384) return fail(OMNISEG_ERR_WORKSPACE, "bce workspace needs 16384 bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(OMNISEG_ERR_ARG, "workspace not 256-byte aligned");
  const int nb = 1024;
  (void)hipGetLastError();
  char* ws = static_cast<char*>(workspace);
  double* psum = reinterpret_cast<double*>(ws);
  int* pcnt = reinterpret_cast<int*>(ws + 8 * nb);
  int* cnt = reinterpret_cast<int*>(ws + 12 * nb);
  HIP_TRY(launch_bce(logit, target, valid, n, psum, pcnt, nb, loss, cnt, grad, reinterpret_cast<hipStream_t>(stream)));
  return OMNISEG_OK;
}

}  // extern "C"

// C ABI of the aggregation and mapping steps: per-class merge to the 40x
// base and the colour overlay (k_map.hip).  Validation happens on the host
// before any launch.
#include <algorithm>

#include "plan.h"

using namespace omniseg;

extern "C" {

int32_t omniseg_merge_to_base(int32_t height, int32_t width, const omniseg_base_plane* planes,
                              int32_t n_planes, omniseg_stream stream) {
  if (!planes) return fail(OMNISEG_ERR_ARG, "planes is NULL");
  if (height < 1 || width < 1 || height > (1 << 20) || width > (1 << 20))
    return fail(OMNISEG_ERR_ARG, "size %dx%d outside [1, 2^20]", height, width);
  if (n_planes < 1 || n_planes > OMNISEG_MAX_CLASSES)
    return fail(OMNISEG_ERR_ARG, "n_planes %d outside [1, %d]", n_planes, OMNISEG_MAX_CLASSES);
  MergeArgs a{};
  a.H = height;
  a.W = width;
  for (int i = 0; i < n_planes; ++i) {
    const omniseg_base_plane& p = planes[i];
    const int k = p.scale_log2;
    if (k < 0 || k > 3) return fail(OMNISEG_ERR_ARG, "plane %d: scale_log2 %d outside [0, 3]", i, k);
    if (p.mode != OMNISEG_UPSAMPLE_NEAREST && p.mode != OMNISEG_UPSAMPLE_BILINEAR)
      return fail(OMNISEG_ERR_ARG, "plane %d: unknown mode %d", i, p.mode);
    const int Hk = ceil_div(height, 1 << k), Wk = ceil_div(width, 1 << k);
    const bool bil = p.mode == OMNISEG_UPSAMPLE_BILINEAR;
    if (bil ? !p.logit : !p.mask) return fail(OMNISEG_ERR_ARG, "plane %d: source is NULL", i);
    if (p.pitch < Wk) return fail(OMNISEG_ERR_ARG, "plane %d: pitch %lld < %d", i, (long long)p.pitch, Wk);
    if (!p.out || p.out_pitch < width) return fail(OMNISEG_ERR_ARG, "plane %d: bad output", i);
    MergePlane& m = a.plane[i];
    m.mask = p.mask;
    m.logit = p.logit;
    m.pitch = p.pitch;
    m.k = k;
    m.Hk = Hk;
    m.Wk = Wk;
    m.bilinear = bil ? 1 : 0;
    m.out = p.out;
    m.out_pitch = p.out_pitch;
    m.vec4 = (reinterpret_cast<uintptr_t>(p.out) % 4 == 0 && p.out_pitch % 4 == 0) ? 1 : 0;
    m.vec16 = (reinterpret_cast<uintptr_t>(p.out) % 16 == 0 && p.out_pitch % 16 == 0) ? 1 : 0;
    const uintptr_t src = bil ? reinterpret_cast<uintptr_t>(p.logit) : reinterpret_cast<uintptr_t>(p.mask);
    const int64_t row_bytes = bil ? p.pitch * 4 : p.pitch;
    m.vec_src = (src % 16 == 0 && row_bytes % 16 == 0) ? 1 : 0;
  }
  (void)hipGetLastError();
  HIP_TRY(launch_merge_base(a, n_planes, reinterpret_cast<hipStream_t>(stream)));
  return OMNISEG_OK;
}

int32_t omniseg_overlay(const omniseg_slide* slide, const omniseg_overlay_class* classes, int32_t n_classes,
                        uint8_t* out, int64_t out_pitch, uint8_t* out10, int64_t out10_pitch,
                        omniseg_stream stream) {
  if (!slide || !slide->rgb) return fail(OMNISEG_ERR_ARG, "slide is NULL");
  const int H = slide->height, W = slide->width;
  if (H < 1 || W < 1 || H > (1 << 20) || W > (1 << 20))
    return fail(OMNISEG_ERR_ARG, "size %dx%d outside [1, 2^20]", H, W);
  if (slide->row_pitch < 3LL * W) return fail(OMNISEG_ERR_ARG, "slide row_pitch < 3 * width");
  if (n_classes < 0 || n_classes > OMNISEG_MAX_CLASSES)
    return fail(OMNISEG_ERR_ARG, "n_classes %d outside [0, %d]", n_classes, OMNISEG_MAX_CLASSES);
  if (n_classes > 0 && !classes) return fail(OMNISEG_ERR_ARG, "classes is NULL");
  if (!out || out_pitch < 3LL * W) return fail(OMNISEG_ERR_ARG, "bad output buffer");
  if (out10 && out10_pitch < 3LL * ceil_div(W, 4)) return fail(OMNISEG_ERR_ARG, "bad 10x output pitch");
  OverlayArgs a{};
  a.rgb = slide->rgb;
  a.pitch = slide->row_pitch;
  a.H = H;
  a.W = W;
  a.n = n_classes;
  for (int i = 0; i < n_classes; ++i) {
    const omniseg_overlay_class& c = classes[i];
    if (!c.mask) return fail(OMNISEG_ERR_ARG, "class %d: mask is NULL", i);
    if (c.scale_log2 < 0 || c.scale_log2 > 3)
      return fail(OMNISEG_ERR_ARG, "class %d: scale_log2 %d outside [0, 3]", i, c.scale_log2);
    if (c.pitch < ceil_div(W, 1 << c.scale_log2)) return fail(OMNISEG_ERR_ARG, "class %d: pitch too small", i);
    if (c.alpha < 0 || c.alpha > 256) return fail(OMNISEG_ERR_ARG, "class %d: alpha %d outside [0, 256]", i, c.alpha);
    OverlayClass& o = a.cls[i];
    o.mask = c.mask;
    o.pitch = c.pitch;
    o.k = c.scale_log2;
    o.alpha = c.alpha;
    for (int ch = 0; ch < 3; ++ch) o.rgb[ch] = c.rgb[ch];
    o.vec4 = (reinterpret_cast<uintptr_t>(c.mask) % 4 == 0 && c.pitch % 4 == 0) ? 1 : 0;
  }
  a.out = out;
  a.out_pitch = out_pitch;
  a.out10 = out10;
  a.out10_pitch = out10_pitch;
  a.vec = (reinterpret_cast<uintptr_t>(slide->rgb) % 4 == 0 && slide->row_pitch % 4 == 0 &&
           reinterpret_cast<uintptr_t>(out) % 4 == 0 && out_pitch % 4 == 0)
              ? 1
              : 0;
  (void)hipGetLastError();
  HIP_TRY(launch_overlay(a, reinterpret_cast<hipStream_t>(stream)));
  return OMNISEG_OK;
}

}  // extern "C"

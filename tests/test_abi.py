"""C-ABI library tests that need no GPU: it loads, exports every declared
symbol, shares torch's HIP runtime, and rejects bad arguments before any
HIP call (so no compute happens here)."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from paper_2305_14566_amd import omniseg as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "omniseg.h")
FAKE = 1 << 20  # never dereferenced: every call below fails validation first


def declared_functions():
    src = open(HEADER).read()
    decl = r"^(?:const\s+)?\w+\s*\*?\s*(omniseg_\w+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    lib = om.lib()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", om.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (omniseg_\w+)", out))
    assert set(names) <= exported


def test_library_uses_torchs_hip_runtime():
    """The library's HIP dependency resolves to the runtime torch loads."""
    import torch
    tlib = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
    need = subprocess.run(["readelf", "-d", om.LIB_PATH], capture_output=True, text=True).stdout
    son = subprocess.run(["readelf", "-d", tlib], capture_output=True, text=True).stdout
    needed = re.findall(r"NEEDED.*\[(libamdhip64[^\]]*)\]", need)
    soname = re.findall(r"SONAME.*\[([^\]]*)\]", son)
    assert needed and soname and needed[0] == soname[0]


def test_status_strings():
    lib = om.lib()
    assert lib.omniseg_status_string(0) == b"ok"
    assert b"workspace" in lib.omniseg_status_string(3)


def _cfg(**kw):
    c = om.Config()
    c.abi_version = om.ABI_VERSION
    c.base_channels = 8
    c.levels = 3
    c.head_out = 1
    c.n_classes = 1
    c.n_scales = 1
    c.tile = 128
    c.stride = 64
    c.fg_filter = 0
    c.fg_threshold = 220
    c.mask_and_fg = 0
    c.precision = om.FP32
    c.flags = 0
    c.batch_tiles = 0
    c.logit_ring_tiles = 0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("field,value,status", [
    ("abi_version", 99, 1), ("base_channels", 0, 1), ("base_channels", 129, 1),
    ("levels", 0, 1), ("head_out", 3, 1), ("n_classes", 0, 1), ("n_classes", 17, 1),
    ("n_scales", 5, 1), ("tile", 100, 1), ("tile", 1024, 1), ("stride", 0, 1), ("stride", 129, 1),
    ("levels", 6, 2), ("fg_threshold", 0, 1), ("precision", 7, 2), ("flags", 8, 1),
    ("batch_tiles", -1, 1), ("fg_filter", 2, 1), ("logit_ring_tiles", -1, 1),
])
def test_plan_create_rejects(field, value, status):
    lib = om.lib()
    h = ctypes.c_void_p()
    c = _cfg(**{field: value})
    assert lib.omniseg_plan_create(ctypes.byref(c), ctypes.byref(h)) == status
    assert lib.omniseg_last_error() != b""
    assert not h.value


@pytest.mark.parametrize("base,L,C,scales,o", [(8, 3, 1, (0,), 1), (64, 5, 6, (0, 1, 2, 3), 2),
                                                (4, 3, 6, (0, 1), 2), (16, 4, 3, (0, 2, 3), 2)])
def test_weight_count_matches_canonical_layout(base, L, C, scales, o):
    p = om.Plan(base=base, levels=L, head_out=o, n_classes=C, scales=scales, tile=256, stride=128)
    n = sum(int(np.prod(sh)) for _, sh, _ in synth.weight_layout(base, L, C, len(scales), o))
    assert p.weight_count == n
    assert p.packed_bytes > 0 and p.packed_bytes % 256 == 0


def test_config2_parameter_count():
    """Base 64, 5 levels, 6 classes, 4 scales, 8-8-8-2 head."""
    p = om.Plan(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 1, 2, 3), tile=256, stride=128)
    ctrl = 162 * (1024 + 10) + 162
    assert p.weight_count - ctrl == 31_378_880 + 8 * 64 + 8


def _slides(shapes):
    arr = (om.Slide * len(shapes))()
    for i, (h, w) in enumerate(shapes):
        arr[i].rgb = FAKE
        arr[i].height = h
        arr[i].width = w
        arr[i].row_pitch = 3 * w
    return arr


def _pairs(pairs):
    arr = (om.Pair * len(pairs))()
    for i, (c, s) in enumerate(pairs):
        arr[i].cls = c
        arr[i].scale = s
    return arr


def test_workspace_layout_and_regions():
    p = om.Plan(base=8, levels=3, head_out=2, n_classes=2, scales=(0, 1), tile=64, stride=32,
                fg_filter=True)
    lib = om.lib()
    sl = _slides([(300, 517), (129, 64)])
    pr = _pairs([(0, 0), (1, 1), (1, 0)])
    n = ctypes.c_int64()
    assert lib.omniseg_workspace_bytes(p._h, sl, 2, pr, 3, ctypes.byref(n)) == 0
    total = n.value
    assert total > 0 and total % 256 == 0
    seen = []
    for region, count in [(0, 2), (1, 4), (2, 2), (3, 1), (4, 1), (5, 4), (6, 1)]:
        for idx in range(count):
            off, nb = ctypes.c_int64(), ctypes.c_int64()
            assert lib.omniseg_workspace_region(p._h, sl, 2, pr, 3, region, idx, ctypes.byref(off),
                                                ctypes.byref(nb)) == 0
            if nb.value > 0 and off.value >= 0:
                assert off.value + nb.value <= total
                seen.append((off.value, nb.value))
    # tile index regions follow the grid sizes: 300x517 at 40x -> 9 x 16 tiles
    off, nb = ctypes.c_int64(), ctypes.c_int64()
    lib.omniseg_workspace_region(p._h, sl, 2, pr, 3, 5, 0, ctypes.byref(off), ctypes.byref(nb))
    assert nb.value == 9 * 16 * 4
    assert lib.omniseg_workspace_region(p._h, sl, 2, pr, 3, 9, 0, ctypes.byref(off), ctypes.byref(nb)) == 1
    assert lib.omniseg_workspace_region(p._h, sl, 2, pr, 3, 1, 4, ctypes.byref(off), ctypes.byref(nb)) == 1


def _segment(p, sl, ns, pr, npairs, outs, ws=FAKE, wsb=1 << 40, packed=FAKE):
    return om.lib().omniseg_segment_slide(p._h, packed, sl, ns, pr, npairs, outs, ws, wsb, None)


def _outs(n):
    o = (om.Output * n)()
    for i in range(n):
        o[i].mask = FAKE
        o[i].mask_pitch = 1 << 20
    return o


@pytest.mark.parametrize("case", ["bad_class", "bad_scale", "dup_pair", "small_slide", "pitch",
                                  "null_rgb", "null_mask", "mask_pitch", "ws_small", "misaligned",
                                  "too_many_slides", "null_logit"])
def test_segment_rejects_before_any_hip_call(case):
    p = om.Plan(base=8, levels=3, head_out=1, n_classes=2, scales=(0, 1), tile=64, stride=32,
                emit_logits=(case == "null_logit"))
    sl = _slides([(100, 80)])
    pr = _pairs([(0, 0), (1, 1)])
    outs = _outs(2)
    if case == "null_logit":
        for i in range(2):
            outs[i].logit = 0
            outs[i].logit_pitch = 1 << 20
        assert _segment(p, sl, 1, pr, 2, outs) == 1
        return
    if case == "bad_class":
        pr = _pairs([(2, 0)])
        assert _segment(p, sl, 1, pr, 1, outs) == 1
    elif case == "bad_scale":
        pr = _pairs([(0, 2)])
        assert _segment(p, sl, 1, pr, 1, outs) == 1
    elif case == "dup_pair":
        pr = _pairs([(0, 0), (0, 0)])
        assert _segment(p, sl, 1, pr, 2, outs) == 1
    elif case == "small_slide":
        assert _segment(p, _slides([(1, 80)]), 1, pr, 2, outs) == 1
    elif case == "pitch":
        s = _slides([(100, 80)])
        s[0].row_pitch = 100
        assert _segment(p, s, 1, pr, 2, outs) == 1
    elif case == "null_rgb":
        s = _slides([(100, 80)])
        s[0].rgb = 0
        assert _segment(p, s, 1, pr, 2, outs) == 1
    elif case == "null_mask":
        outs[1].mask = 0
        assert _segment(p, sl, 1, pr, 2, outs) == 1
    elif case == "mask_pitch":
        outs[0].mask_pitch = 79
        assert _segment(p, sl, 1, pr, 2, outs) == 1
    elif case == "ws_small":
        assert _segment(p, sl, 1, pr, 2, outs, wsb=1024) == 3
    elif case == "misaligned":
        assert _segment(p, sl, 1, pr, 2, outs, ws=FAKE + 8) == 1
    elif case == "too_many_slides":
        assert _segment(p, _slides([(100, 80)] * 33), 33, pr, 2, _outs(66)) == 1


def test_stitch_rejects_before_any_hip_call():
    lib = om.lib()
    n = ctypes.c_int64()
    assert lib.omniseg_stitch_workspace_bytes(64, 32, 100, 90, ctypes.byref(n)) == 0
    assert n.value == 256  # 4 x 3 grid of int32, aligned
    assert lib.omniseg_stitch_workspace_bytes(64, 65, 100, 90, ctypes.byref(n)) == 1
    # workspace too small
    assert lib.omniseg_stitch_tiles(64, 32, 100, 90, 0, FAKE, FAKE, 3, FAKE, 90, 0, 0, FAKE, 16, None) == 3
    # more tiles than grid positions
    assert lib.omniseg_stitch_tiles(64, 32, 100, 90, 0, FAKE, FAKE, 13, FAKE, 90, 0, 0, FAKE, 256, None) == 1
    # mask pitch
    assert lib.omniseg_stitch_tiles(64, 32, 100, 90, 0, FAKE, FAKE, 3, FAKE, 89, 0, 0, FAKE, 256, None) == 1
    # negative vote threshold
    assert lib.omniseg_stitch_tiles(64, 32, 100, 90, -1, FAKE, FAKE, 3, FAKE, 90, 0, 0, FAKE, 256, None) == 1
    # a grid above 2^30 positions
    assert lib.omniseg_stitch_workspace_bytes(16, 1, 1 << 20, 1 << 20, ctypes.byref(n)) == 2


@pytest.mark.parametrize("case", ["repeat_scale", "stride_range", "merge", "vote_low", "vote_high",
                                  "train_vote", "train_strides"])
def test_merge_and_stride_validation(case):
    """Per-scale strides and the vote merge are validated at plan creation."""
    base = dict(base=4, levels=2, head_out=1, n_classes=2, scales=(0, 2), tile=64, stride=32)
    ok = dict(scale_strides=(32, 16), merge=om.MERGE_VOTE, vote_thresholds=(1, 16))
    om.Plan(**base, **ok)  # valid: ceil(64/16)^2 = 16 tiles cover a 10x pixel at most
    bad = {
        "repeat_scale": dict(scales=(1, 1)),
        "stride_range": dict(scale_strides=(32, 65)),
        "merge": dict(merge=2),
        "vote_low": dict(vote_thresholds=(0, 4)),
        "vote_high": dict(vote_thresholds=(1, 17)),
        "train_vote": dict(scale_strides=None, vote_thresholds=(1, 4), training=True),
        "train_strides": dict(merge=om.MERGE_RAMP, vote_thresholds=None, training=True),
    }[case]
    kw = {**base, **ok, **bad}
    with pytest.raises(om.OmnisegError) as e:
        om.Plan(**kw)
    assert e.value.status == (2 if case.startswith("train") else 1)


@pytest.mark.parametrize("case", ["method", "even_median", "big_median", "area"])
def test_tissue_validation(case):
    kw = dict(base=4, levels=2, head_out=1, n_classes=1, scales=(0, 2), tile=64, stride=32, fg_filter=True,
              tissue_method=om.TISSUE_OTSU, median_kernel=9, min_tissue_area=10)
    om.Plan(**kw)
    kw.update({"method": dict(tissue_method=2), "even_median": dict(median_kernel=8),
               "big_median": dict(median_kernel=257), "area": dict(min_tissue_area=-1)}[case])
    with pytest.raises(om.OmnisegError) as e:
        om.Plan(**kw)
    assert e.value.status == 1


def test_tissue_regions_follow_the_method():
    lib = om.lib()
    sl = _slides([(300, 517), (129, 64)])
    pr = _pairs([(0, 0)])
    for method, want in [(om.TISSUE_GRAY, 0), (om.TISSUE_OTSU, 1)]:
        p = om.Plan(base=4, levels=2, head_out=1, n_classes=1, scales=(0, 2), tile=64, stride=32, fg_filter=True,
                    tissue_method=method, median_kernel=5)
        off, nb = ctypes.c_int64(), ctypes.c_int64()
        assert lib.omniseg_workspace_region(p._h, sl, 2, pr, 1, om.REGION_TISSUE_GRAY, 1, ctypes.byref(off),
                                            ctypes.byref(nb)) == 0
        assert nb.value == want * 33 * 16  # the 10x map of the 129 x 64 slide
        assert lib.omniseg_workspace_region(p._h, sl, 2, pr, 1, om.REGION_TISSUE_STATS, 0, ctypes.byref(off),
                                            ctypes.byref(nb)) == 0
        assert nb.value == want * 16


def test_merge_and_overlay_reject_before_any_hip_call():
    lib = om.lib()
    pl = (om.BasePlane * 1)()
    pl[0].mask, pl[0].pitch, pl[0].scale_log2, pl[0].mode, pl[0].out, pl[0].out_pitch = FAKE, 13, 3, 0, FAKE, 100
    for field, value in [("scale_log2", 4), ("mode", 2), ("pitch", 12), ("out_pitch", 99)]:
        bad = (om.BasePlane * 1)()
        ctypes.memmove(bad, pl, ctypes.sizeof(pl))
        setattr(bad[0], field, value)
        assert lib.omniseg_merge_to_base(100, 100, bad, 1, None) == 1, field
    assert lib.omniseg_merge_to_base(100, 100, pl, 17, None) == 1
    assert lib.omniseg_merge_to_base(0, 100, pl, 1, None) == 1
    bl = (om.BasePlane * 1)()
    ctypes.memmove(bl, pl, ctypes.sizeof(pl))
    bl[0].mode = 1  # bilinear needs the logit plane
    assert lib.omniseg_merge_to_base(100, 100, bl, 1, None) == 1
    sl = om.Slide(FAKE, 100, 80, 240)
    oc = (om.OverlayClass * 1)()
    oc[0].mask, oc[0].pitch, oc[0].scale_log2, oc[0].alpha = FAKE, 80, 0, 300
    assert lib.omniseg_overlay(ctypes.byref(sl), oc, 1, FAKE, 240, None, 0, None) == 1  # alpha > 256
    oc[0].alpha = 128
    assert lib.omniseg_overlay(ctypes.byref(sl), oc, 1, FAKE, 239, None, 0, None) == 1  # out pitch
    assert lib.omniseg_overlay(ctypes.byref(sl), oc, 1, FAKE, 240, FAKE, 59, None) == 1  # 10x pitch
    assert lib.omniseg_overlay(ctypes.byref(sl), oc, 17, FAKE, 240, None, 0, None) == 1


def test_conv_refuses_images_above_2gib_before_any_hip_call():
    """The conv kernels address one image's input with 32-bit offsets."""
    lib = om.lib()
    big = 1 << 40
    # 4096 x 4096 x 64 BF16 channels = 2^31 bytes: refused; 32 channels fit
    assert lib.omniseg_conv3x3(om.BF16, om.CONV_RELU, 1, 4096, 4096, 64, 64, 64, FAKE, FAKE, FAKE, None, None, FAKE,
                               None, -1, FAKE, big, None) == 2
    # POOL reads a 2H x 2W input: 2048^2 output x 4 x 64 x 2 bytes is refused too
    assert lib.omniseg_conv3x3(om.BF16, om.CONV_POOL_RELU, 1, 2048, 2048, 64, 64, 64, FAKE, FAKE, FAKE, None, None,
                               FAKE, None, -1, FAKE, big, None) == 2
    assert lib.omniseg_conv3x3_fp8(om.CONV_RELU, 1, 4096, 4096, 128, 128, 64, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                                   FAKE, None, -1, FAKE, big, None) == 2


def test_tile_grid_size_guard():
    """A tile grid of more than 32767 tiles per side is refused before any HIP call."""
    p = om.Plan(base=4, levels=2, head_out=1, n_classes=1, scales=(0,), tile=16, stride=1)
    sl = _slides([(40000, 64)])
    assert _segment(p, sl, 1, _pairs([(0, 0)]), 1, _outs(1)) == 2


def _tiles(ts):
    arr = (om.Tile * len(ts))()
    for i, (s, y, x) in enumerate(ts):
        arr[i].scale, arr[i].jy, arr[i].jx = s, y, x
    return arr


@pytest.mark.parametrize("case", ["no_flag", "dup_tile", "tile_out", "too_many", "scale_out", "ws_small",
                                  "null_grad", "one_level"])
def test_training_entry_points_reject_before_any_hip_call(case):
    lib = om.lib()
    p = om.Plan(base=4, levels=1 if case == "one_level" else 3, head_out=2, n_classes=6, scales=(0, 1), tile=32,
                stride=16, training=(case != "no_flag"))
    sl = _slides([(64, 64)])
    pr = _pairs([(0, 0), (3, 1)])
    tl = [(0, 0, 0), (1, 0, 0)]
    if case == "dup_tile":
        tl = [(0, 1, 1), (0, 1, 1)]
    elif case == "tile_out":
        tl = [(0, 3, 0)]
    elif case == "too_many":
        tl = [(0, 0, 0)] * 257
    elif case == "scale_out":
        tl = [(2, 0, 0)]
    t = _tiles(tl)
    n = ctypes.c_int64()
    st = lib.omniseg_train_workspace_bytes(p._h, sl, t, len(tl), pr, 2, ctypes.byref(n))
    if case in ("ws_small", "null_grad"):
        assert st == 0 and n.value > 0
        if case == "ws_small":
            assert lib.omniseg_train_forward(p._h, FAKE, sl, t, len(tl), pr, 2, FAKE, FAKE, FAKE, 4096, None) == 3
        else:
            assert lib.omniseg_backward(p._h, FAKE, sl, t, len(tl), pr, 2, FAKE, 0, FAKE, n.value, None) == 1
        return
    assert st in (1, 2), st
    assert lib.omniseg_train_forward(p._h, FAKE, sl, t, len(tl), pr, 2, FAKE, FAKE, FAKE, 1 << 40, None) == st


def test_plane_offsets_and_bce_validation():
    lib = om.lib()
    p = om.Plan(base=4, levels=3, head_out=2, n_classes=6, scales=(0, 1), tile=32, stride=16, training=True)
    sl = _slides([(65, 40)])
    pr = _pairs([(0, 0), (3, 1), (5, 0)])
    off = (ctypes.c_int64 * 4)()
    assert lib.omniseg_plane_offsets(p._h, sl, pr, 3, off) == 0
    assert list(off) == [0, 65 * 40, 65 * 40 + 33 * 20, 2 * 65 * 40 + 33 * 20]
    assert lib.omniseg_bce_loss(FAKE, FAKE, FAKE, 0, FAKE, 0, FAKE, 16384, None) == 1
    assert lib.omniseg_bce_loss(FAKE, FAKE, FAKE, 10, FAKE, 0, FAKE, 100, None) == 3


def test_conv_config_query_and_precision_gate():
    """Every configuration has a shape and a precision set; the row-reuse
    configurations are BF16 only, and the stand-alone conv refuses a
    configuration at a precision it does not run at, or one that does not
    fit the shape, before any HIP call."""
    assert om.N_CONV_CONFIGS == 13
    for c in range(om.N_CONV_CONFIGS):
        by, bx, bn, wm, wn, precs = om.conv_config_info(c)
        assert wm * wn in (4, 8) and by % 8 == 0 and bx in (8, 16) and bn % 32 == 0
        assert om.BF16 in precs
        assert (om.FP32 in precs) == (c < 6) and (om.FP8 in precs) == (6 <= c < 10)
    with pytest.raises(om.OmnisegError):
        om.conv_config_info(om.N_CONV_CONFIGS)
    lib = om.lib()
    ws = ctypes.c_int64()
    assert lib.omniseg_conv3x3_workspace_bytes(om.FP32, 64, 64, 64, ctypes.byref(ws)) == 0
    def call(prec, cfg, h=32, w=32, mode=om.CONV_RELU, pool=None):
        return lib.omniseg_conv3x3(prec, mode, 1, h, w, 64, 64, 64, FAKE, FAKE, FAKE, None, None, FAKE, pool, cfg,
                                   FAKE, ws.value, None)
    assert call(om.FP32, 6) == 1           # row-reuse configuration at FP32
    assert call(om.BF16, 8, h=16) == 1     # 32-row block on a 16-row image
    assert call(om.BF16, 3, w=24) == 1     # 16-pixel block on a 24-pixel-wide image
    # the pooled copy: BF16 / FP8 only, RES_RELU only, row-reuse configurations only
    assert call(om.FP32, -1, mode=om.CONV_RES_RELU, pool=FAKE) == 2
    assert call(om.BF16, -1, mode=om.CONV_RELU, pool=FAKE) == 1
    assert call(om.BF16, 1, mode=om.CONV_RES_RELU, pool=FAKE) == 1


def test_fp8_plan_validation_and_activation_table():
    """FP8 plans: inference only, deepest level a multiple of 16; the
    activation table has one entry per padded channel of every stored
    activation, kind-major then level; the packing and calibration entry
    points refuse the wrong precision before any HIP call."""
    lib = om.lib()
    h = ctypes.c_void_p()
    c = _cfg(precision=om.FP8, flags=om.FLAG_TRAINING)
    assert lib.omniseg_plan_create(ctypes.byref(c), ctypes.byref(h)) == 2 and not h.value
    c = _cfg(precision=om.FP8, tile=32, stride=16)  # 32 / 2^2 = 8 rows at the bottleneck
    assert lib.omniseg_plan_create(ctypes.byref(c), ctypes.byref(h)) == 2 and not h.value
    p8 = om.Plan(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 1, 2, 3), tile=256, stride=128,
                 precision=om.FP8)
    p32 = om.Plan(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 1, 2, 3), tile=256, stride=128)
    C = [64 * 2 ** l for l in range(5)]
    assert p8.activation_channels == p32.activation_channels == 2 * sum(C) + 2 * sum(C[:4])
    off = 0
    for kind, nl in ((om.ACT_ENC_A, 5), (om.ACT_ENC_E, 5), (om.ACT_DEC_A, 4), (om.ACT_DEC_D, 4)):
        for l in range(nl):
            assert p8.activation_offset(kind, l) == off
            off += C[l]
    with pytest.raises(om.OmnisegError):
        p8.activation_offset(om.ACT_DEC_D, 4)  # D_{L-1} is E_{L-1}: no own entry
    # FP8 packed weights: 64-channel chunks, one byte per weight, plus scale tables
    assert 0 < p8.packed_bytes < p32.packed_bytes / 3
    assert lib.omniseg_pack_weights(p8._h, FAKE, FAKE, None) == 2
    assert lib.omniseg_pack_weights_fp8(p32._h, FAKE, FAKE, FAKE, None) == 1
    sl = (om.Slide * 1)()
    sl[0].rgb, sl[0].height, sl[0].width, sl[0].row_pitch = FAKE, 512, 512, 1536
    pr = (om.Pair * 1)()
    assert lib.omniseg_calibrate_fp8(p8._h, FAKE, sl, 1, pr, 1, 64, FAKE, FAKE, 1 << 40, None) == 1
    assert lib.omniseg_calibrate_fp8(p32._h, FAKE, sl, 1, pr, 1, 0, FAKE, FAKE, 1 << 40, None) == 1


def test_conv_tuning_get_set():
    """Tuning entries start at -1 (default), can be pinned per layer and read
    back, and out-of-range stages, levels and configurations are refused."""
    p = om.Plan(base=8, levels=3, head_out=1, n_classes=1, scales=(0,), tile=64, stride=32)
    assert all(p.get_conv_tuning(st, l) == -1 for st in range(4) for l in range(3))
    p.set_conv_tuning(2, 1, 10)
    p.set_conv_tuning(1, 0, 0)
    assert p.get_conv_tuning(2, 1) == 10 and p.get_conv_tuning(1, 0) == 0 and p.get_conv_tuning(2, 0) == -1
    p.set_conv_tuning(2, 1, -1)
    assert p.get_conv_tuning(2, 1) == -1
    for st, l, c in [(4, 0, 0), (-1, 0, 0), (0, 3, 0), (0, -1, 0), (0, 0, om.N_CONV_CONFIGS), (0, 0, -2)]:
        with pytest.raises(om.OmnisegError) as e:
            p.set_conv_tuning(st, l, c)
        assert e.value.status == 1  # OMNISEG_ERR_ARG
    with pytest.raises(om.OmnisegError):
        p.get_conv_tuning(0, 3)

"""ctypes binding of libomniseg.so (argument marshalling only).

Every step of the segmentation runs in the library's HIP kernels; torch is
used here only to allocate device memory and to supply the current HIP
stream.  The functions mirror the C ABI in include/omniseg.h.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# OMNISEG_LIBRARY selects another build of the same library (the host
# sanitizer build of build.build_sanitized, for the ABI tests).
LIB_PATH = os.environ.get("OMNISEG_LIBRARY") or os.path.join(_HERE, "libomniseg.so")

FP32, BF16, FP8 = 0, 1, 2
ACT_ENC_A, ACT_ENC_E, ACT_DEC_A, ACT_DEC_D = range(4)
FLAG_EMIT_LOGITS = 1
FLAG_TRAINING = 2
FLAG_GRAPH = 4
MERGE_RAMP, MERGE_VOTE = 0, 1
UPSAMPLE_NEAREST, UPSAMPLE_BILINEAR = 0, 1
TISSUE_GRAY, TISSUE_OTSU = 0, 1
(REGION_PAD, REGION_PYRAMID, REGION_TISSUE, REGION_TILE_COUNT, REGION_TILE_LIST,
 REGION_TILE_INDEX, REGION_TILE_LOGITS, REGION_TISSUE_GRAY, REGION_TISSUE_STATS) = range(9)
ABI_VERSION = 7

CONV_RELU, CONV_RES_RELU, CONV_POOL_RELU, CONV_UPCAT_RELU, CONV_DGRAD, CONV_DGRAD_RES_MASK = range(6)
N_CONV_CONFIGS = 13

_lib = None


class OmnisegError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"omniseg status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("base_channels", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("head_out", ctypes.c_int32),
        ("n_classes", ctypes.c_int32),
        ("n_scales", ctypes.c_int32),
        ("scale_log2", ctypes.c_int32 * 4),
        ("tile", ctypes.c_int32),
        ("stride", ctypes.c_int32),
        ("fg_filter", ctypes.c_int32),
        ("fg_threshold", ctypes.c_int32),
        ("mask_and_fg", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("batch_tiles", ctypes.c_int32),
        ("logit_ring_tiles", ctypes.c_int32),
        ("scale_stride", ctypes.c_int32 * 4),
        ("merge", ctypes.c_int32),
        ("vote_threshold", ctypes.c_int32 * 4),
        ("tissue_method", ctypes.c_int32),
        ("median_kernel", ctypes.c_int32),
        ("min_tissue_area", ctypes.c_int32),
    ]


class Slide(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("row_pitch", ctypes.c_int64)]


class Pair(ctypes.Structure):
    _fields_ = [("cls", ctypes.c_int32), ("scale", ctypes.c_int32)]


class LaunchRecord(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_int32), ("level", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("config", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double), ("ms", ctypes.c_double)]


STAGE_NAMES = ("prep", "first_conv", "enc_a", "enc_b", "dec_a", "dec_b", "gap_ctrl", "head", "stitch")


class Tile(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_int32), ("jy", ctypes.c_int32), ("jx", ctypes.c_int32)]


class BasePlane(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_void_p), ("logit", ctypes.c_void_p), ("pitch", ctypes.c_int64),
                ("scale_log2", ctypes.c_int32), ("mode", ctypes.c_int32), ("out", ctypes.c_void_p),
                ("out_pitch", ctypes.c_int64)]


class OverlayClass(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_void_p), ("pitch", ctypes.c_int64), ("scale_log2", ctypes.c_int32),
                ("alpha", ctypes.c_int32), ("rgb", ctypes.c_uint8 * 4)]


class Output(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_void_p), ("logit", ctypes.c_void_p),
                ("mask_pitch", ctypes.c_int64), ("logit_pitch", ctypes.c_int64)]


def _declare(lib):
    P = ctypes.POINTER
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "omniseg_status_string": (ctypes.c_char_p, [i32]),
        "omniseg_last_error": (ctypes.c_char_p, []),
        "omniseg_plan_create": (i32, [P(Config), P(vp)]),
        "omniseg_plan_destroy": (i32, [vp]),
        "omniseg_weight_count": (i32, [vp, P(i64)]),
        "omniseg_packed_weight_bytes": (i32, [vp, P(i64)]),
        "omniseg_pack_weights": (i32, [vp, vp, vp, vp]),
        "omniseg_workspace_bytes": (i32, [vp, P(Slide), i32, P(Pair), i32, P(i64)]),
        "omniseg_segment_slide": (i32, [vp, vp, P(Slide), i32, P(Pair), i32, P(Output), vp, i64, vp]),
        "omniseg_workspace_region": (i32, [vp, P(Slide), i32, P(Pair), i32, i32, i32, P(i64), P(i64)]),
        "omniseg_stitch_workspace_bytes": (i32, [i32, i32, i32, i32, P(i64)]),
        "omniseg_stitch_tiles": (i32, [i32, i32, i32, i32, i32, vp, vp, i32, vp, i64, vp, i64, vp, i64, vp]),
        "omniseg_stitch_tiles_noalloc": (i32, [i32, i32, i32, i32, i32, vp, vp, i32, vp, i64, vp, i64, vp]),
        "omniseg_set_profiling": (i32, [vp, i32]),
        "omniseg_set_conv_tuning": (i32, [vp, i32, i32, i32]),
        "omniseg_get_conv_tuning": (i32, [vp, i32, i32, P(i32)]),
        "omniseg_conv_config": (i32, [i32, P(i32), P(i32), P(i32), P(i32), P(i32), P(i32)]),
        "omniseg_autotune": (i32, [vp, vp, P(Slide), i32, P(Pair), i32, vp, i64, vp]),
        "omniseg_plane_offsets": (i32, [vp, P(Slide), P(Pair), i32, P(i64)]),
        "omniseg_train_workspace_bytes": (i32, [vp, P(Slide), P(Tile), i32, P(Pair), i32, P(i64)]),
        "omniseg_train_forward": (i32, [vp, vp, P(Slide), P(Tile), i32, P(Pair), i32, vp, vp, vp, i64, vp]),
        "omniseg_backward": (i32, [vp, vp, P(Slide), P(Tile), i32, P(Pair), i32, vp, vp, vp, i64, vp]),
        "omniseg_bce_loss": (i32, [vp, vp, vp, i64, vp, vp, vp, i64, vp]),
        "omniseg_conv3x3_workspace_bytes": (i32, [i32, i32, i32, i32, P(i64)]),
        "omniseg_conv3x3": (i32, [i32, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, vp, i64,
                                  vp]),
        "omniseg_read_profile": (i32, [vp, P(LaunchRecord), i32, P(i32)]),
        "omniseg_conv3x3_wgrad_workspace_bytes": (i32, [i32, i32, i32, i32, i32, i32, P(i64)]),
        "omniseg_conv3x3_wgrad": (i32, [i32, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, i64, vp]),
        "omniseg_conv3x3_fp8_workspace_bytes": (i32, [i32, i32, i32, P(i64)]),
        "omniseg_conv3x3_fp8": (i32, [i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp,
                                      i64, vp]),
        "omniseg_activation_channels": (i32, [vp, P(i64)]),
        "omniseg_activation_offset": (i32, [vp, i32, i32, P(i64)]),
        "omniseg_calibrate_fp8": (i32, [vp, vp, P(Slide), i32, P(Pair), i32, i32, vp, vp, i64, vp]),
        "omniseg_pack_weights_fp8": (i32, [vp, vp, vp, vp, vp]),
        "omniseg_merge_to_base": (i32, [i32, i32, P(BasePlane), i32, vp]),
        "omniseg_overlay": (i32, [P(Slide), P(OverlayClass), i32, vp, i64, vp, i64, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def lib():
    """Load libomniseg.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2305_14566_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        _declare(l)
        _lib = l
    return _lib


def _check(status):
    if status != 0:
        l = lib()
        raise OmnisegError(status, f"{l.omniseg_status_string(status).decode()}: "
                                   f"{l.omniseg_last_error().decode()}")


def _stream(stream=None):
    if stream is None:
        if not torch.cuda.is_available():
            return None
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def level_size(n, k):
    return -(-n // (1 << k))


class Plan:
    """A validated configuration (host side only)."""

    def __init__(self, base=8, levels=3, head_out=1, n_classes=1, scales=(0,), tile=128,
                 stride=64, fg_filter=False, fg_threshold=220, mask_and_fg=False,
                 precision=FP32, emit_logits=False, batch_tiles=0, training=False, graph=False,
                 logit_ring_tiles=0, scale_strides=None, merge=MERGE_RAMP, vote_thresholds=None,
                 tissue_method=TISSUE_GRAY, median_kernel=1, min_tissue_area=0):
        c = Config()
        c.abi_version = ABI_VERSION
        c.base_channels = base
        c.levels = levels
        c.head_out = head_out
        c.n_classes = n_classes
        c.n_scales = len(scales)
        for i, k in enumerate(scales):
            c.scale_log2[i] = k
        c.tile = tile
        c.stride = stride
        c.fg_filter = int(fg_filter)
        c.fg_threshold = fg_threshold
        c.mask_and_fg = int(mask_and_fg)
        c.precision = precision
        c.flags = ((FLAG_EMIT_LOGITS if emit_logits else 0) | (FLAG_TRAINING if training else 0)
                   | (FLAG_GRAPH if graph else 0))
        c.batch_tiles = batch_tiles
        c.logit_ring_tiles = logit_ring_tiles
        for i, v in enumerate(scale_strides or ()):
            c.scale_stride[i] = v
        c.merge = merge
        c.tissue_method = tissue_method
        c.median_kernel = median_kernel
        c.min_tissue_area = min_tissue_area
        for i, v in enumerate(vote_thresholds or ()):
            c.vote_threshold[i] = v
        self.cfg = c
        self.scales = tuple(scales)
        self.emit_logits = emit_logits
        self._h = ctypes.c_void_p()
        _check(lib().omniseg_plan_create(ctypes.byref(c), ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.omniseg_plan_destroy(h)
            self._h = None

    @property
    def weight_count(self):
        n = ctypes.c_int64()
        _check(lib().omniseg_weight_count(self._h, ctypes.byref(n)))
        return n.value

    @property
    def packed_bytes(self):
        n = ctypes.c_int64()
        _check(lib().omniseg_packed_weight_bytes(self._h, ctypes.byref(n)))
        return n.value

    def set_profiling(self, enable):
        _check(lib().omniseg_set_profiling(self._h, int(bool(enable))))

    def read_profile(self):
        """Per-launch records of the last profiled segment call (list of dicts)."""
        n = ctypes.c_int32()
        _check(lib().omniseg_read_profile(self._h, None, 0, ctypes.byref(n)))
        recs = (LaunchRecord * max(1, n.value))()
        _check(lib().omniseg_read_profile(self._h, recs, n.value, ctypes.byref(n)))
        return [dict(stage=STAGE_NAMES[r.stage], level=r.level, tiles=r.tiles, flops=r.flops,
                     bytes=r.bytes, ms=r.ms, config=r.config) for r in recs[:n.value]]

    def autotune(self, slides, pairs, packed, workspace, stream=None):
        """Time every valid conv tile configuration per layer; keep the fastest."""
        sl, pr = self._arrays(slides, pairs)
        _check(lib().omniseg_autotune(self._h, _ptr(packed), sl, len(slides), pr, len(pairs), _ptr(workspace),
                                      workspace.numel(), _stream(stream)))

    def set_conv_tuning(self, stage, level, config):
        """Pin the tile configuration of one conv layer (stage 0 enc_a, 1 enc_b,
        2 dec_a, 3 dec_b; config -1 = the default)."""
        _check(lib().omniseg_set_conv_tuning(self._h, stage, level, config))

    def get_conv_tuning(self, stage, level):
        v = ctypes.c_int32()
        _check(lib().omniseg_get_conv_tuning(self._h, stage, level, ctypes.byref(v)))
        return v.value

    def pack(self, canonical, stream=None):
        """Canonical FP32 weights (device tensor) -> packed device buffer (uint8)."""
        if canonical.dtype != torch.float32 or not canonical.is_cuda or not canonical.is_contiguous():
            raise ValueError("canonical weights must be a contiguous float32 device tensor")
        if canonical.numel() != self.weight_count:
            raise ValueError(f"expected {self.weight_count} weights, got {canonical.numel()}")
        packed = torch.empty(self.packed_bytes, dtype=torch.uint8, device=canonical.device)
        _check(lib().omniseg_pack_weights(self._h, _ptr(canonical), _ptr(packed), _stream(stream)))
        return packed

    # ---- FP8 -------------------------------------------------------------------

    @property
    def activation_channels(self):
        n = ctypes.c_int64()
        _check(lib().omniseg_activation_channels(self._h, ctypes.byref(n)))
        return n.value

    def activation_offset(self, kind, level):
        n = ctypes.c_int64()
        _check(lib().omniseg_activation_offset(self._h, kind, level, ctypes.byref(n)))
        return n.value

    def calibrate_fp8(self, slides, pairs, packed, workspace, n_tiles=64, stream=None):
        """Per-channel activation maxima (device float32 activation table) of
        this FP32 plan's backbone over the first n_tiles kept tiles."""
        sl, pr = self._arrays(slides, pairs)
        amax = torch.empty(self.activation_channels, dtype=torch.float32, device=slides[0].device)
        _check(lib().omniseg_calibrate_fp8(self._h, _ptr(packed), sl, len(slides), pr, len(pairs), n_tiles,
                                           _ptr(amax), _ptr(workspace), workspace.numel(), _stream(stream)))
        return amax

    def pack_fp8(self, canonical, amax, stream=None):
        """Canonical FP32 weights + activation maxima (device) -> packed FP8 buffer."""
        if canonical.dtype != torch.float32 or not canonical.is_cuda or not canonical.is_contiguous():
            raise ValueError("canonical weights must be a contiguous float32 device tensor")
        if canonical.numel() != self.weight_count:
            raise ValueError(f"expected {self.weight_count} weights, got {canonical.numel()}")
        if amax.dtype != torch.float32 or amax.numel() != self.activation_channels:
            raise ValueError("amax must be the float32 activation table of this network")
        packed = torch.empty(self.packed_bytes, dtype=torch.uint8, device=canonical.device)
        _check(lib().omniseg_pack_weights_fp8(self._h, _ptr(canonical), _ptr(amax.contiguous()), _ptr(packed),
                                              _stream(stream)))
        return packed

    def _arrays(self, slides, pairs):
        sl = (Slide * len(slides))()
        for i, s in enumerate(slides):
            if s.dtype != torch.uint8 or s.dim() != 3 or s.shape[2] != 3:
                raise ValueError("slides must be uint8 [H, W, 3] tensors")
            if s.stride(2) != 1 or s.stride(1) != 3:
                raise ValueError("slide rows must be interleaved RGB")
            sl[i].rgb = s.data_ptr()
            sl[i].height = s.shape[0]
            sl[i].width = s.shape[1]
            sl[i].row_pitch = s.stride(0)
        pr = (Pair * len(pairs))()
        for i, (c, k) in enumerate(pairs):
            pr[i].cls = c
            pr[i].scale = k
        return sl, pr

    def workspace_bytes(self, slides, pairs):
        sl, pr = self._arrays(slides, pairs)
        n = ctypes.c_int64()
        _check(lib().omniseg_workspace_bytes(self._h, sl, len(slides), pr, len(pairs), ctypes.byref(n)))
        return n.value

    def region(self, slides, pairs, region, index=0):
        sl, pr = self._arrays(slides, pairs)
        off, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().omniseg_workspace_region(self._h, sl, len(slides), pr, len(pairs), region, index,
                                              ctypes.byref(off), ctypes.byref(nb)))
        return off.value, nb.value

    # ---- training -------------------------------------------------------------

    def _train_arrays(self, slide, tiles, pairs):
        sl, pr = self._arrays([slide], pairs)
        tl = (Tile * len(tiles))()
        for i, (si, jy, jx) in enumerate(tiles):
            tl[i].scale = si
            tl[i].jy = jy
            tl[i].jx = jx
        return sl, tl, pr

    def plane_offsets(self, slide, pairs):
        sl, pr = self._arrays([slide], pairs)
        off = (ctypes.c_int64 * (len(pairs) + 1))()
        _check(lib().omniseg_plane_offsets(self._h, sl, pr, len(pairs), off))
        return list(off)

    def train_workspace_bytes(self, slide, tiles, pairs):
        sl, tl, pr = self._train_arrays(slide, tiles, pairs)
        n = ctypes.c_int64()
        _check(lib().omniseg_train_workspace_bytes(self._h, sl, tl, len(tiles), pr, len(pairs), ctypes.byref(n)))
        return n.value

    def train_forward(self, slide, tiles, pairs, packed, workspace, stream=None):
        """Forward over a tile batch; returns (flat logits, flat coverage)."""
        sl, tl, pr = self._train_arrays(slide, tiles, pairs)
        total = self.plane_offsets(slide, pairs)[-1]
        logit = torch.empty(total, dtype=torch.float32, device=slide.device)
        covered = torch.empty(total, dtype=torch.uint8, device=slide.device)
        _check(lib().omniseg_train_forward(self._h, _ptr(packed), sl, tl, len(tiles), pr, len(pairs), _ptr(logit),
                                           _ptr(covered), _ptr(workspace), workspace.numel(), _stream(stream)))
        return logit, covered

    def backward(self, slide, tiles, pairs, packed, workspace, grad_logit, stream=None):
        """dLoss/dweights (canonical FP32 order) after train_forward."""
        sl, tl, pr = self._train_arrays(slide, tiles, pairs)
        if grad_logit.dtype != torch.float32 or not grad_logit.is_contiguous():
            raise ValueError("grad_logit must be contiguous float32")
        gw = torch.empty(self.weight_count, dtype=torch.float32, device=slide.device)
        _check(lib().omniseg_backward(self._h, _ptr(packed), sl, tl, len(tiles), pr, len(pairs), _ptr(grad_logit),
                                      _ptr(gw), _ptr(workspace), workspace.numel(), _stream(stream)))
        return gw

    def alloc_outputs(self, slides, pairs):
        masks, logits = [], []
        for s in slides:
            mrow, lrow = [], []
            for (c, si) in pairs:
                k = self.scales[si]
                hk, wk = level_size(s.shape[0], k), level_size(s.shape[1], k)
                mrow.append(torch.empty((hk, wk), dtype=torch.uint8, device=s.device))
                lrow.append(torch.empty((hk, wk), dtype=torch.float32, device=s.device)
                            if self.emit_logits else None)
            masks.append(mrow)
            logits.append(lrow)
        return masks, logits

    def segment(self, slides, pairs, packed, workspace=None, outputs=None, stream=None):
        """Run the whole path; returns (masks, logits, workspace).

        masks[i][p] is uint8 [H_k, W_k]; logits[i][p] float32 or None.
        """
        sl, pr = self._arrays(slides, pairs)
        need = self.workspace_bytes(slides, pairs)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=slides[0].device)
        masks, logits = outputs if outputs is not None else self.alloc_outputs(slides, pairs)
        outs = (Output * (len(slides) * len(pairs)))()
        for i in range(len(slides)):
            for p in range(len(pairs)):
                o = outs[i * len(pairs) + p]
                m = masks[i][p]
                o.mask = m.data_ptr()
                o.mask_pitch = m.stride(0)
                lg = logits[i][p]
                o.logit = lg.data_ptr() if lg is not None else 0
                o.logit_pitch = lg.stride(0) if lg is not None else 0
        _check(lib().omniseg_segment_slide(self._h, _ptr(packed), sl, len(slides), pr, len(pairs), outs,
                                           _ptr(workspace), workspace.numel(), _stream(stream)))
        return masks, logits, workspace


def stitch_tiles(tile, stride, height, width, tile_logits, tile_yx, emit_logits=True, stream=None,
                 vote_threshold=0):
    """Stand-alone stitch of one plane; returns (mask uint8, logit float32 or None).
    vote_threshold > 0: majority vote (the logit plane then holds vote counts)."""
    l = lib()
    n = ctypes.c_int64()
    _check(l.omniseg_stitch_workspace_bytes(tile, stride, height, width, ctypes.byref(n)))
    dev = tile_logits.device
    ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
    mask = torch.empty((height, width), dtype=torch.uint8, device=dev)
    logit = torch.empty((height, width), dtype=torch.float32, device=dev) if emit_logits else None
    n_tiles = tile_yx.shape[0]
    _check(l.omniseg_stitch_tiles(tile, stride, height, width, vote_threshold, _ptr(tile_logits), _ptr(tile_yx), n_tiles,
                                  _ptr(mask), mask.stride(0), _ptr(logit),
                                  logit.stride(0) if logit is not None else 0, _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return mask, logit


def stitch_tiles_noalloc(tile, stride, height, width, tile_logits, tile_yx, mask, logit=None, stream=None,
                         vote_threshold=0):
    """stitch_tiles into caller-provided outputs with the library's own index
    grid (no workspace, nothing allocated by the library)."""
    n_tiles = tile_yx.shape[0]
    _check(lib().omniseg_stitch_tiles_noalloc(tile, stride, height, width, vote_threshold, _ptr(tile_logits),
                                              _ptr(tile_yx), n_tiles, _ptr(mask), mask.stride(0), _ptr(logit),
                                              logit.stride(0) if logit is not None else 0, _stream(stream)))
    return mask, logit


def merge_to_base(height, width, planes, stream=None, outs=None):
    """Merge per-class planes to 40x masks.  planes: list of (k, mode, src)
    with src the scale-k uint8 mask (NEAREST) or float32 logit plane
    (BILINEAR), 2-D device tensors.  outs: optional (height, width) uint8
    device tensors (views with any row stride) to write into.  Returns the
    40x uint8 masks."""
    n = len(planes)
    arr = (BasePlane * n)()
    given, outs = outs, []
    for i, (k, mode, src) in enumerate(planes):
        out = torch.empty((height, width), dtype=torch.uint8, device=src.device) if given is None else given[i]
        if tuple(out.shape) != (height, width) or out.dtype != torch.uint8 or out.stride(1) != 1:
            raise ValueError("each output must be a (height, width) uint8 tensor with unit column stride")
        if mode == UPSAMPLE_BILINEAR:
            arr[i].logit = src.data_ptr()
        else:
            arr[i].mask = src.data_ptr()
        arr[i].pitch = src.stride(0)
        arr[i].scale_log2 = k
        arr[i].mode = mode
        arr[i].out = out.data_ptr()
        arr[i].out_pitch = out.stride(0)
        outs.append(out)
    _check(lib().omniseg_merge_to_base(height, width, arr, n, _stream(stream)))
    return outs


def overlay(slide, classes, with_10x=True, out=None, stream=None):
    """Colour overlay of class masks on a 40x slide (uint8 HWC device tensor).
    classes: list of (mask, k, (r, g, b), alpha).  Returns (out, out10 or None)."""
    H, W, _ = slide.shape
    sl = Slide(slide.data_ptr(), H, W, slide.stride(0))
    arr = (OverlayClass * max(len(classes), 1))()
    for i, (m, k, rgb, alpha) in enumerate(classes):
        arr[i].mask = m.data_ptr()
        arr[i].pitch = m.stride(0)
        arr[i].scale_log2 = k
        arr[i].alpha = alpha
        for ch in range(3):
            arr[i].rgb[ch] = rgb[ch]
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.uint8, device=slide.device)
    o10 = torch.empty(((H + 3) // 4, (W + 3) // 4, 3), dtype=torch.uint8, device=slide.device) if with_10x else None
    _check(lib().omniseg_overlay(ctypes.byref(sl), arr, len(classes), out.data_ptr(), out.stride(0),
                                 o10.data_ptr() if o10 is not None else None,
                                 o10.stride(0) if o10 is not None else 0, _stream(stream)))
    return out, o10


def bce_loss(logit, target, valid, with_grad=True, stream=None):
    """Mean BCE-with-logits over valid entries; returns (loss float64 tensor, grad or None)."""
    dev = logit.device
    loss = torch.empty((), dtype=torch.float64, device=dev)
    grad = torch.empty_like(logit) if with_grad else None
    ws = torch.empty(16384, dtype=torch.uint8, device=dev)
    _check(lib().omniseg_bce_loss(_ptr(logit), _ptr(target), _ptr(valid), logit.numel(), _ptr(loss), _ptr(grad),
                                  _ptr(ws), ws.numel(), _stream(stream)))
    return loss, grad


class OmniSegFn(torch.autograd.Function):
    """Differentiable stitched logits of a tile batch w.r.t. the canonical weights.

    forward(weights, plan, slide, tiles, pairs) -> (flat logits, flat coverage);
    backward runs the library's hand-written reverse pass.
    """

    @staticmethod
    def forward(ctx, weights, plan, slide, tiles, pairs):
        packed = plan.pack(weights.detach().contiguous())
        ws = torch.empty(plan.train_workspace_bytes(slide, tiles, pairs), dtype=torch.uint8, device=slide.device)
        logit, covered = plan.train_forward(slide, tiles, pairs, packed, ws)
        ctx.state = (plan, slide, tiles, pairs, packed, ws)
        ctx.mark_non_differentiable(covered)
        return logit, covered

    @staticmethod
    def backward(ctx, grad_logit, grad_covered):
        plan, slide, tiles, pairs, packed, ws = ctx.state
        gw = plan.backward(slide, tiles, pairs, packed, ws, grad_logit.contiguous().float())
        return gw, None, None, None, None


class BCELossFn(torch.autograd.Function):
    """Mean BCE-with-logits over covered pixels (library kernel)."""

    @staticmethod
    def forward(ctx, logit, target, valid):
        loss, grad = bce_loss(logit.detach().contiguous(), target.contiguous(), valid.contiguous())
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad * grad_out.to(grad.dtype), None, None


def conv3x3(precision, mode, x0, weights, bias=None, x1=None, aux=None, cin=None, cu=None, cout=None,
            height=None, width=None, config=-1, stream=None, pool=False):
    """Stand-alone backbone conv on NHWC tensors with 32-padded channels.

    Returns y (same dtype as x0) of shape [n, H, W, pad32(out channels)];
    with pool=True also its 2x2 max-pool [n, H/2, W/2, ...] from the same
    kernel, as (y, y_pool).
    """
    n = x0.shape[0]
    cout_, cin_ = weights.shape[0], weights.shape[1]
    cin = cin_ if cin is None else cin
    cout = cout_ if cout is None else cout
    cu = cin if cu is None else cu
    if height is None:
        height = x0.shape[1] // 2 if mode == CONV_POOL_RELU else (x0.shape[1] * 2 if mode == CONV_UPCAT_RELU
                                                                  else x0.shape[1])
        width = x0.shape[2] // 2 if mode == CONV_POOL_RELU else (x0.shape[2] * 2 if mode == CONV_UPCAT_RELU
                                                                 else x0.shape[2])
    p32 = lambda c: -(-c // 32) * 32
    if mode >= CONV_DGRAD:
        out_c = p32(cu) + p32(cin - cu) if cu < cin else p32(cin)
    else:
        out_c = p32(cout)
    y = torch.empty((n, height, width, out_c), dtype=x0.dtype, device=x0.device)
    yp = torch.empty((n, height // 2, width // 2, out_c), dtype=x0.dtype, device=x0.device) if pool else None
    nb = ctypes.c_int64()
    _check(lib().omniseg_conv3x3_workspace_bytes(precision, cin, cu, cout, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=x0.device)
    _check(lib().omniseg_conv3x3(precision, mode, n, height, width, cin, cu, cout, _ptr(weights), _ptr(bias),
                                 _ptr(x0), _ptr(x1), _ptr(aux), _ptr(y), _ptr(yp), config, _ptr(ws), ws.numel(),
                                 _stream(stream)))
    return (y, yp) if pool else y


def conv3x3_wgrad(precision, mode, x0, dy, cin, cout, x1=None, cu=None, stream=None):
    """Weight gradient (canonical FP32 [cout][cin][3][3]) of the stand-alone
    conv `mode` (CONV_RELU, CONV_POOL_RELU or CONV_UPCAT_RELU) with input x0
    (x1) and output gradient dy [n, H, W, pad32(cout)]."""
    n, height, width = dy.shape[0], dy.shape[1], dy.shape[2]
    cu = cin if cu is None else cu
    nb = ctypes.c_int64()
    _check(lib().omniseg_conv3x3_wgrad_workspace_bytes(n, height, width, cin, cu, cout, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dy.device)
    dw = torch.empty((cout, cin, 3, 3), dtype=torch.float32, device=dy.device)
    _check(lib().omniseg_conv3x3_wgrad(precision, mode, n, height, width, cin, cu, cout, _ptr(x0), _ptr(x1), _ptr(dy),
                                       _ptr(dw), _ptr(ws), ws.numel(), _stream(stream)))
    return dw


def conv3x3_fp8(mode, x0, weights, bias, in_scale, out_scale, x1=None, cu=None, height=None, width=None,
                config=-1, stream=None, pool=False):
    """Stand-alone FP8 backbone conv: x0 (x1) uint8 E4M3 codes, NHWC with
    32-padded channels, channel scales in_scale (real channel order) and
    out_scale.  Returns the uint8 output codes [n, H, W, pad32(cout)]."""
    n = x0.shape[0]
    cout, cin = weights.shape[0], weights.shape[1]
    cu = cin if cu is None else cu
    if height is None:
        height = x0.shape[1] // 2 if mode == CONV_POOL_RELU else (x0.shape[1] * 2 if mode == CONV_UPCAT_RELU
                                                                  else x0.shape[1])
        width = x0.shape[2] // 2 if mode == CONV_POOL_RELU else (x0.shape[2] * 2 if mode == CONV_UPCAT_RELU
                                                                 else x0.shape[2])
    y = torch.empty((n, height, width, -(-cout // 32) * 32), dtype=torch.uint8, device=x0.device)
    yp = torch.empty((n, height // 2, width // 2, y.shape[3]), dtype=torch.uint8, device=x0.device) if pool else None
    nb = ctypes.c_int64()
    _check(lib().omniseg_conv3x3_fp8_workspace_bytes(cin, cu, cout, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=x0.device)
    _check(lib().omniseg_conv3x3_fp8(mode, n, height, width, cin, cu, cout, _ptr(weights), _ptr(bias),
                                     _ptr(in_scale), _ptr(out_scale), _ptr(x0), _ptr(x1), _ptr(y), _ptr(yp), config,
                                     _ptr(ws), ws.numel(), _stream(stream)))
    return (y, yp) if pool else y


def conv_config(config):
    """(by, bx, bn, wm, wn) of a conv tile configuration id."""
    return conv_config_info(config)[:5]


def conv_config_info(config):
    """(by, bx, bn, wm, wn, precisions) of a conv tile configuration id;
    precisions is the set of precisions (FP32, BF16, FP8) it runs at."""
    v = [ctypes.c_int32() for _ in range(6)]
    _check(lib().omniseg_conv_config(config, *[ctypes.byref(x) for x in v]))
    vals = [x.value for x in v]
    return tuple(vals[:5]) + (frozenset(p for p in (FP32, BF16, FP8) if vals[5] >> p & 1),)

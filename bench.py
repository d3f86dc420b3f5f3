#!/usr/bin/env python3
"""Throughput of the slide-wise segmentation path on one MI355X.

Headline workload (the batching configuration): 16 seeded synthetic slides
of uneven size (heights 2000-8000 px, widths 4000-40000 px, 10-60% tissue),
4 scales (40/20/10/5x) x 6 classes (24 class-scale pairs), 256 x 256 tiles
at stride 128 with foreground-only tile lists, a base-64 5-level residual
U-Net with a controller-generated 8-8-8-2 dynamic head, ramp-weighted stitch
into whole-slide masks.  A step is one omniseg_segment_slide call over all 16
slides (pad, pyramid, tissue map, tile list, BF16 backbone, controller, head,
streamed stitch into a ring logit store), replayed as one HIP graph, with
the slides already in HBM and the masks written to HBM.
value = total slide pixels x pairs / step time, in Mpixel/s per class-scale.

Beside it: the same 16 slides one call per slide; the plain FP32 backbone
and FP8 on one 8192 x 8192 slide; the training step; masks of BF16 and FP8
against FP32 and against the FP64 oracle (1024^2 crop) with trained weights;
the paper's tiling and majority vote; merge and colour mapping; the FP64
oracle timed on the host cores (cpu_baseline).

Prints one JSON line.  --gpus N > 1 is refused: this path runs on one GPU.
"""

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WSI Mpixel/s per class-scale (BF16 batched vs FP32 plain) at ≥0.999 Dice; %MFMA peak"
UNIT = "Mpixel/s per class-scale"
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp8": 5000.0}
HBM_PEAK_GBS = 8000.0

CFG = dict(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 1, 2, 3), tile=256, stride=128,
           fg_filter=True)
PAIRS = [(c, si) for si in range(4) for c in range(6)]
# The tiling of the paper's experiments (Section 3.2): 512^2 tiles at 40x with
# stride 256 and vote threshold 1, at 10x and 5x with stride 64 and threshold 4.
PAPER_CFG = dict(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 2, 3), tile=512, stride=256,
                 fg_filter=True, scale_strides=(256, 64, 64), vote_thresholds=(1, 4, 4),
                 tissue_method="otsu", median_kernel=59, min_tissue_area=64)
# Best magnification per class (Section 1: glomeruli 5x, tubules 10x,
# capillaries 40x; arteries taken at 10x), as scale slots of CFG's 40/20/10/5x:
# TUFT, CAP, PT, DT, PTC, VES.
CLASS_SLOT = (3, 3, 2, 2, 0, 2)
CLASS_COLOURS = ((230, 25, 75), (60, 180, 75), (255, 225, 25), (0, 130, 200), (245, 130, 48), (145, 30, 180))
SLIDE = 8192          # side of the single-slide workload (slide seed 2)
CROP = 1024           # precision crop of that slide, a stand-alone slide
REGION = 2048         # training region (slide seed 3, with ground truth)
TRAIN_LR = 1e-3       # Adam, cosine decay to 0 over the steps
TRAIN_BATCH = 32

# HBM bytes of one launch of each conv layer of the bench network on a full
# batch of 256 tiles, with the configuration BENCH_CONV_TABLE pins, from two
# rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE) of
#   bench.py --counters
# summarised by bench.py --summarize-counters: each counter scaled by its
# reading for the 1 GiB device copy the command makes first.  They describe
# the conv source whose SHA-256 is stored here; any other source reports
# null.
MEASURED_TRAFFIC = {
    "conv_source_sha256": "af1b7ff352d6f758bb0f1fb5fe0d3878c9a3211e3b8937ffaed7b5d8550a4cd7",
    "batch": 256,
    # (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000) bytes of one full-batch launch per layer
    "kernels": {
        "omniseg::k_conv3x3_rows2p<32, 64, 4, 2, 0, 0>": {
            "enc_a2": (277461444, 537328896),
            "enc_a3": (433181913, 268464896),
        },
        "omniseg::k_conv3x3_rows2p<32, 64, 4, 2, 0, 1>": {
            "dec_b1": (1909318610, 1087182176),
            "dec_b2": (1065358019, 540254080),
            "dec_b3": (1066830218, 273384992),
            "enc_b1": (2013380524, 1441024160),
            "enc_b2": (1094047346, 760669152),
            "enc_b3": (1069392807, 374582816),
        },
        "omniseg::k_conv3x3_rows2p<32, 64, 4, 2, 2, 0>": {
            "dec_a0": (3332663357, 2147897760),
            "dec_a1": (2055258207, 1074858176),
            "dec_a2": (1711877637, 537401920),
            "dec_a3": (2215174866, 268813472),
        },
        "omniseg::k_conv3x3_rows<16, 64, 4, 2, 0, 0>": {
            "enc_a4": (1259464721, 134217728),
        },
        "omniseg::k_conv3x3_rows<16, 64, 4, 2, 0, 1>": {
            "enc_b4": (2654240968, 134217728),
        },
        "omniseg::k_conv3x3_ws<0>": {
            "enc_a1": (597060402, 1073742560),
        },
        "omniseg::k_conv3x3_ws<1>": {
            "dec_b0": (2414780364, 2147496832),
            "enc_b0": (2421045979, 2684709440),
        },
    },
}

# HBM bytes (FETCH_SIZE x 2 + WRITE_SIZE, the same passes) of one launch of
# the mapping leg's kernels on the 8192^2 slide: the merge to 40x and the
# overlay of the six classes, and the stand-alone stitch of one 40x plane from
# all its grid tiles with mask and logit out; each for the source file whose
# SHA-256 is stored with it (any other source reports null).
MEASURED_MAP_TRAFFIC = {
    "k_merge_base": ("k_map.hip", "723d3d48b11ebff318d67407ddd621026d9124b71440febff24b3913129a3aae", 848068366),
    "k_overlay": ("k_map.hip", "723d3d48b11ebff318d67407ddd621026d9124b71440febff24b3913129a3aae", 818004708),
    "k_stitch4": ("k_stitch.hip", "4a162bdf1593cbb7e1c9f3e33bc44fc20234b7656d30e202a52b94375bf330d3", 1376365176),
}


def measured_map_traffic(kernel):
    """Measured HBM bytes of one mapping-leg launch of `kernel`, or None when
    its source changed since the measurement."""
    import hashlib

    if kernel not in MEASURED_MAP_TRAFFIC:
        return None
    src, want, nbytes = MEASURED_MAP_TRAFFIC[kernel]
    with open(os.path.join(ROOT, "paper_2305_14566_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return nbytes if sha == want else None


def measured_traffic(kernel, records):
    """HBM bytes per launch of `kernel` averaged over its launches in
    `records`: each launch's layer as measured on a full batch (FETCH_SIZE +
    WRITE_SIZE, MEASURED_TRAFFIC), scaled by the tiles the launch processed
    over the batch size (a launch past the kept-tile count reads only the
    count).  None when the conv source changed since the measurement, or a
    layer the kernel ran for was not measured."""
    import hashlib

    src = os.path.join(ROOT, "paper_2305_14566_amd", "csrc", "k_conv.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    k = MEASURED_TRAFFIC["kernels"].get(kernel)
    if k is None or sha != MEASURED_TRAFFIC["conv_source_sha256"] or not records:
        return None
    per = [k.get(f"{r['stage']}{r['level']}") for r in records]
    if any(v is None for v in per):
        return None
    B = MEASURED_TRAFFIC["batch"]
    return sum((f + w) * r["tiles"] / B for (f, w), r in zip(per, records)) / len(per)


def conv_symbol(om, prec, stage, config, level=None):
    """Kernel symbol (as rocprofv3 prints it) that a conv launch of the bench
    network uses."""
    # BF16 and FP8 fuse the max-pool into the encoder's residual conv, so
    # conv_a then reads the pooled tensor with the plain loader
    loader, epi = {"enc_a": (1 if prec == "fp32" else 0, 0), "enc_b": (0, 1), "dec_a": (2, 0), "dec_b": (0, 1)}[stage]
    by, bx, bn, wm, wn = om.conv_config(config)
    if prec == "fp8":
        return f"omniseg::k_conv3x3_fp8<{by}, {bn}, {wm}, {wn}, {loader}, {epi}>"
    # the eight-wave configuration runs the layers with 64 input channels
    # (level-0 residual convs, level-1 conv_a) in its weight-stationary form
    if prec == "bf16" and config == 10 and ((stage in ("enc_b", "dec_b") and level == 0) or
                                            (stage == "enc_a" and level == 1)):
        # the last decoder conv also computes the head's precls (epilogue 4)
        return f"omniseg::k_conv3x3_ws<{4 if stage == 'dec_b' else epi}>"
    if prec == "bf16" and config == 11:  # large-block row-reuse configuration
        return f"omniseg::k_conv3x3_rows2<{by}, {bn}, {wm}, {wn}, {loader}, {epi}>"
    if prec == "bf16" and config == 12:  # its persistent form
        return f"omniseg::k_conv3x3_rows2p<{by}, {bn}, {wm}, {wn}, {loader}, {epi}>"
    if prec == "bf16" and config >= 6:  # row-reuse configurations
        return f"omniseg::k_conv3x3_rows<{by}, {bn}, {wm}, {wn}, {loader}, {epi}>"
    t = "unsigned short" if prec == "bf16" else "float"
    return f"omniseg::k_conv3x3<{t}, {by}, {bx}, {bn}, {wm}, {wn}, {loader}, {epi}>"


def roofline(om, records, prec):
    """Aggregate the profile by kernel symbol; report the dominant conv kernel."""
    groups = {}
    for r in records:
        if r["stage"] not in ("enc_a", "enc_b", "dec_a", "dec_b"):
            continue
        sym = conv_symbol(om, prec, r["stage"], r["config"], r["level"])
        g = groups.setdefault(sym, dict(n=0, flops=0.0, ms=0.0, bytes=0.0, recs=[]))
        g["recs"].append(r)
        g["n"] += 1
        g["flops"] += r["flops"]
        g["ms"] += r["ms"]
        g["bytes"] += r["bytes"]
    sym, g = max(groups.items(), key=lambda kv: kv[1]["ms"])
    achieved = g["flops"] / (g["ms"] * 1e-3) / 1e12
    conv_ms = sum(v["ms"] for v in groups.values())
    conv_flops = sum(v["flops"] for v in groups.values())
    return dict(bound="mfma", kernel=sym, launches=g["n"],
                flops_per_launch=g["flops"] / g["n"], avg_launch_ms=g["ms"] / g["n"],
                achieved=achieved, peak=PEAK_TFLOPS[prec], unit="TFLOP/s",
                frac=achieved / PEAK_TFLOPS[prec], traffic=measured_traffic(sym, g["recs"]),
                algorithmic_bytes_per_launch=g["bytes"] / g["n"],
                all_convs_tflops=conv_flops / (conv_ms * 1e-3) / 1e12,
                all_convs_frac=conv_flops / (conv_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec])


def layer_summary(records, steps):
    """Per (stage, level) conv time and rate, per step."""
    out = {}
    for r in records:
        if r["stage"] not in ("enc_a", "enc_b", "dec_a", "dec_b"):
            continue
        s = out.setdefault(f"{r['stage']}{r['level']}", dict(ms=0.0, flops=0.0, bytes=0.0, launches=0,
                                                             config=r["config"]))
        s["ms"] += r["ms"] / steps
        s["flops"] += r["flops"] / steps
        s["bytes"] += r["bytes"] / steps
        s["launches"] += 1
    for s in out.values():
        s["tflops"] = s["flops"] / max(s["ms"], 1e-9) / 1e9
    return out


def stage_summary(records):
    out = {}
    for r in records:
        s = out.setdefault(r["stage"], dict(ms=0.0, flops=0.0, bytes=0.0, launches=0))
        s["ms"] += r["ms"]
        s["flops"] += r["flops"]
        s["bytes"] += r["bytes"]
        s["launches"] += 1
    for s in out.values():
        s["tflops"] = s["flops"] / max(s["ms"], 1e-9) / 1e9
        s["gbs"] = s["bytes"] / max(s["ms"], 1e-9) / 1e6
    return out


def _plan(om, prec, batch_tiles, cfg=CFG, emit_logits=False, graph=False, ring=0):
    vote = "vote_thresholds" in cfg
    otsu = cfg.get("tissue_method") == "otsu"
    return om.Plan(base=cfg["base"], levels=cfg["levels"], head_out=cfg["head_out"],
                   n_classes=cfg["n_classes"], scales=cfg["scales"], tile=cfg["tile"],
                   stride=cfg["stride"], fg_filter=cfg["fg_filter"],
                   precision={"bf16": om.BF16, "fp32": om.FP32, "fp8": om.FP8}[prec], emit_logits=emit_logits,
                   batch_tiles=batch_tiles, scale_strides=cfg.get("scale_strides"), graph=graph,
                   logit_ring_tiles=ring,
                   merge=om.MERGE_VOTE if vote else om.MERGE_RAMP, vote_thresholds=cfg.get("vote_thresholds"),
                   tissue_method=om.TISSUE_OTSU if otsu else om.TISSUE_GRAY,
                   median_kernel=cfg.get("median_kernel", 1), min_tissue_area=cfg.get("min_tissue_area", 0))


def _timed(torch, fn, n, stream):
    """Mean ms of n back-to-back calls, by events on `stream`."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / max(1, n)


def _kept(om, plan, slides, pairs, ws):
    import torch

    off, _ = plan.region(slides, pairs, om.REGION_TILE_COUNT)
    return int(ws[off:off + 4].view(torch.int32).item())


def run_leg(om, torch, dslide, flat_dev, pairs, prec, steps, warmup, batch_tiles, calib_tiles=64, cfg=CFG,
            emit_logits=False, amax=None, tune=True):
    """One slide, one precision: `steps` timed calls back to back (no
    profiling), then one profiled call for the per-launch records."""
    plan = _plan(om, prec, batch_tiles, cfg, emit_logits=emit_logits)
    ws = torch.empty(plan.workspace_bytes([dslide], pairs), dtype=torch.uint8, device=dslide.device)
    extra = {}
    if prec == "fp8":
        if amax is None:
            # per-channel activation scales from the FP32 path on the first kept tiles
            p32 = _plan(om, "fp32", batch_tiles, cfg)
            ws32 = torch.empty(p32.workspace_bytes([dslide], pairs), dtype=torch.uint8, device=dslide.device)
            t_cal = time.perf_counter()
            amax = p32.calibrate_fp8([dslide], pairs, p32.pack(flat_dev), ws32, n_tiles=calib_tiles)
            torch.cuda.synchronize()
            extra["calibration_s"] = time.perf_counter() - t_cal
            extra["calibration_tiles"] = calib_tiles
            del ws32, p32
        packed = plan.pack_fp8(flat_dev, amax)
    else:
        packed = plan.pack(flat_dev)
    outs = plan.alloc_outputs([dslide], pairs)
    t_tune = time.perf_counter()
    if tune:
        plan.autotune([dslide], pairs, packed, ws)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    call = lambda: plan.segment([dslide], pairs, packed, workspace=ws, outputs=outs)
    for _ in range(warmup):
        call()
    stream = torch.cuda.current_stream()
    ms = _timed(torch, call, steps, stream)
    plan.set_profiling(True)
    call()
    records = plan.read_profile()
    plan.set_profiling(False)
    kept = _kept(om, plan, [dslide], pairs, ws)
    masks = [m.cpu().numpy().astype(bool) for m in outs[0][0]]
    logits = [lg.cpu().numpy() for lg in outs[1][0]] if emit_logits else None
    tuned = sorted({(r["stage"], r["level"], r["config"]) for r in records if r["config"] >= 0})
    if cfg.get("tissue_method") == "otsu":
        off, nb = plan.region([dslide], pairs, om.REGION_TISSUE_STATS)
        extra["tissue_stats"] = [int(v) for v in ws[off:off + nb].view(torch.int32).cpu()]
    if emit_logits:
        # coverage of every plane: pixels under a kept tile (Lambda is exactly 0 elsewhere)
        extra["covered"] = _coverage(om, plan, [dslide], pairs, ws, cfg)[0]
    return dict(ms=ms, records=records, kept=kept, masks=masks, logits=logits,
                tuned={f"{st}{l}": list(om.conv_config(c)) for st, l, c in tuned}, tune_s=t_tune, **extra)


def _coverage(om, plan, slides, pairs, ws, cfg):
    """Per (slide, pair): boolean map of the pixels some kept tile covers."""
    import torch

    T = cfg["tile"]
    out = []
    for i, s in enumerate(slides):
        H, W = s.shape[0], s.shape[1]
        row = []
        for (c, si) in pairs:
            k = cfg["scales"][si]
            st = (cfg.get("scale_strides") or [cfg["stride"]] * 4)[si]
            Hk, Wk = -(-H // (1 << k)), -(-W // (1 << k))
            off, nb = plan.region(slides, pairs, om.REGION_TILE_INDEX, i * len(cfg["scales"]) + si)
            idx = ws[off:off + nb].view(torch.int32).cpu().numpy()
            ny = 1 if Hk <= T else -(-(Hk - T) // st) + 1
            nx = 1 if Wk <= T else -(-(Wk - T) // st) + 1
            idx = idx.reshape(ny, nx)
            cov = np.zeros((Hk, Wk), bool)
            for jy, jx in zip(*np.nonzero(idx >= 0)):
                cov[jy * st:jy * st + T, jx * st:jx * st + T] = True
            row.append(cov)
        out.append(row)
    return out


def paper_leg(om, torch, M, dslide, size, steps, batch_tiles):
    """The paper's tiling on the same slide: 512^2 tiles, 40x/10x/5x with
    strides 256/64/64, majority-vote merge with thresholds 1/4/4, 6 classes;
    BF16 throughput, and its masks against one FP32 step of the same plan."""
    import synth

    C = PAPER_CFG["n_classes"]
    flat = synth.he_normal_weights(12, PAPER_CFG["base"], PAPER_CFG["levels"], C, len(PAPER_CFG["scales"]),
                                   PAPER_CFG["head_out"])
    flat_dev = torch.from_numpy(flat).to(dslide.device)
    pairs = [(c, si) for si in range(len(PAPER_CFG["scales"])) for c in range(C)]
    bf = run_leg(om, torch, dslide, flat_dev, pairs, "bf16", steps, 1, batch_tiles, cfg=PAPER_CFG)
    fp = run_leg(om, torch, dslide, flat_dev, pairs, "fp32", 1, 0, batch_tiles, cfg=PAPER_CFG)
    px = size * size * len(pairs)
    dices = [M.dice(a, b) for a, b in zip(bf["masks"], fp["masks"])]
    stages = stage_summary(bf["records"])
    return {"value": px / (bf["ms"] * 1e-3) / 1e6, "unit": UNIT, "ms_per_step": bf["ms"], "steps": steps,
            "dtype": "bf16", "kept_tiles": bf["kept"], "pairs": len(pairs),
            "workload": f"the {size}x{size} slide, 512 tiles, scales 40x/10x/5x at strides 256/64/64, "
                        "majority vote with thresholds 1/4/4, 6 classes, Otsu tissue map (5x, median 59, "
                        "components of < 64 coarse pixels removed)",
            "tissue_stats": dict(zip(("otsu_threshold", "components", "kept_components"), bf["tissue_stats"][:3])),
            "prep_ms": stages.get("prep", {}).get("ms"),
            "fp32_ms_per_step": fp["ms"], "speedup_bf16_vs_fp32": fp["ms"] / bf["ms"],
            "bf16_vs_fp32_vote_masks": {"dice_min": min(dices), "dice_mean": float(np.mean(dices))},
            "stitch_ms": stages.get("stitch", {}).get("ms"),
            "roofline": dict(roofline(om, bf["records"], "bf16"), traffic=None)}


def mapping_leg(om, torch, dslide, flat_dev, size, reps, batch_tiles):
    """Slide-wise aggregation and mapping on the single slide: each class's
    stitched logits at its best scale merged to a 40x mask (bilinear), then
    the six-colour overlay on the 40x slide and its 10x map; and the
    stand-alone stitch of one 40x plane from all its grid tiles.  Timed with
    HIP events on the launch stream over `reps` back-to-back repetitions."""
    plan = _plan(om, "bf16", batch_tiles, emit_logits=True)
    packed = plan.pack(flat_dev)
    masks, logits, _ = plan.segment([dslide], PAIRS, packed)
    torch.cuda.synchronize()
    H = W = size
    planes = []
    for c, si in enumerate(CLASS_SLOT):
        p = PAIRS.index((c, si))
        planes.append((CFG["scales"][si], om.UPSAMPLE_BILINEAR, logits[0][p]))
    out = torch.empty((H, W, 3), dtype=torch.uint8, device=dslide.device)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    m40 = om.merge_to_base(H, W, planes)
    om.overlay(dslide, [(m, 0, col, 128) for m, col in zip(m40, CLASS_COLOURS)], out=out)
    torch.cuda.synchronize()
    # back-to-back launches between the events, so that the host's launch
    # latency is paid once per leg rather than once per repetition
    classes = [(m, 0, col, 128) for m, col in zip(m40, CLASS_COLOURS)]
    ev[0].record(stream)
    for _ in range(reps):
        om.merge_to_base(H, W, planes, outs=m40)
    ev[1].record(stream)
    for _ in range(reps):
        _, o10 = om.overlay(dslide, classes, out=out)
    ev[2].record(stream)
    torch.cuda.synchronize()
    t_merge = ev[0].elapsed_time(ev[1]) / reps
    t_over = ev[1].elapsed_time(ev[2]) / reps
    # the stand-alone stitch of one 40x plane from all its grid tiles (random
    # logits), the plane-wise form of the segment call's streamed stitch
    T, s_ = CFG["tile"], CFG["stride"]
    ny = (H - T + s_ - 1) // s_ + 1
    yx = torch.tensor([(j // ny, j % ny) for j in range(ny * ny)], dtype=torch.int32, device=dslide.device)
    g = torch.Generator(device=dslide.device)
    g.manual_seed(17)
    tl = torch.randn((ny * ny, T, T), generator=g, device=dslide.device)
    om.stitch_tiles(T, s_, H, W, tl, yx, emit_logits=True)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(reps):
        om.stitch_tiles(T, s_, H, W, tl, yx, emit_logits=True)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_stitch = ev[0].elapsed_time(ev[1]) / reps
    stitch_bytes = 4 * ny * ny * T * T + 5 * H * W  # every tile logit once; mask and logit out
    del tl
    px = H * W
    merge_bytes = sum(4 * ((H + (1 << k) - 1) >> k) * ((W + (1 << k) - 1) >> k) + px for k, _, _ in planes)
    over_bytes = 3 * px + len(m40) * px + 3 * px + 3 * ((H + 3) // 4) * ((W + 3) // 4)
    return {"workload": f"the {size}x{size} slide: 6 classes merged to 40x from their best scales "
                        "(TUFT, CAP 5x; PT, DT, VES 10x; PTC 40x; bilinear on the stitched logits), then the "
                        "6-colour overlay (alpha 128/256) and its 10x map",
            "merge_ms": t_merge, "overlay_ms": t_over, "reps": reps,
            "merge_roofline": dict(bound="hbm", achieved=merge_bytes / (t_merge * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                                   unit="GB/s", frac=merge_bytes / (t_merge * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                   traffic=measured_map_traffic("k_merge_base"), algorithmic_bytes=merge_bytes),
            "overlay_roofline": dict(bound="hbm", achieved=over_bytes / (t_over * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                                     unit="GB/s", frac=over_bytes / (t_over * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     traffic=measured_map_traffic("k_overlay"), algorithmic_bytes=over_bytes),
            "stitch_standalone": {"workload": f"omniseg_stitch_tiles: one {H}x{W} 40x plane from all its {ny * ny} "
                                              f"grid tiles ({T}^2 at stride {s_}, random logits), mask and logit out",
                                  "ms": t_stitch,
                                  "roofline": dict(bound="hbm", achieved=stitch_bytes / (t_stitch * 1e-3) / 1e9,
                                                   peak=HBM_PEAK_GBS, unit="GB/s",
                                                   frac=stitch_bytes / (t_stitch * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                                   traffic=measured_map_traffic("k_stitch4"),
                                                   algorithmic_bytes=stitch_bytes)},
            "class_pixels_40x": [int(m.sum().item()) for m in m40]}


# ---------------------------------------------------------------------------
# inputs (seeded; generated in worker processes)
# ---------------------------------------------------------------------------

def _gen_input(job):
    import synth

    kind, arg = job
    if kind == "batch":
        rgb, _ = synth.strip_slide(arg["seed"], arg["H"], arg["W"], fg_frac=arg["fg_frac"], with_gt=False)
        return rgb
    if kind == "slide":
        rgb, _ = synth.strip_slide(2, arg, arg, fg_frac=0.30, with_gt=False)
        return rgb
    rgb, gt = synth.strip_slide(3, REGION, REGION, fg_frac=0.30)
    return rgb, gt


# ---------------------------------------------------------------------------
# training step (and the trained weights of the precision leg)
# ---------------------------------------------------------------------------

def train_leg(om, torch, rgb, gt, steps, batch=TRAIN_BATCH):
    """The bench network (4 scales x 6 classes) trained on the 2048^2 region:
    each step 32 random tiles of the region's 284 grid tiles (all scales), a
    BF16 forward through backbone, head and stitch, the loss on the stitched
    logits, the library's hand-written backward and an Adam update of the
    FP32 canonical weights (lr TRAIN_LR after 25 warm-up steps, cosine decay).  Start: the
    He-normal draw with every block's residual conv zeroed
    (synth.training_init_weights); the loss weights each class's positive
    pixels by its negative/positive ratio in the region, at most 10 (the
    classes cover 0.2-1 % of the pixels).  Returns the report and the
    trained FP32 weights."""
    import synth

    dev = torch.device("cuda:0")
    C, scales = CFG["n_classes"], CFG["scales"]
    flat = synth.training_init_weights(13, CFG["base"], CFG["levels"], C, len(scales), CFG["head_out"])
    plan = om.Plan(base=CFG["base"], levels=CFG["levels"], head_out=CFG["head_out"], n_classes=C, scales=scales,
                   tile=CFG["tile"], stride=CFG["stride"], precision=om.BF16, training=True)
    pin_conv_table(plan)  # the forward convs; the backward's take the library's default per layer
    slide = torch.from_numpy(rgb).to(dev)
    y = torch.from_numpy(synth.soft_targets(gt, scales, PAIRS)).to(dev)
    offs = plan.plane_offsets(slide, PAIRS)
    pw = torch.empty_like(y)
    for p in range(len(PAIRS)):
        pos = float(y[offs[p]:offs[p + 1]].mean())
        pw[offs[p]:offs[p + 1]] = float(np.clip((1 - pos) / max(pos, 1e-6), 1.0, 10.0))
    w = torch.from_numpy(flat).to(dev).requires_grad_(True)
    opt = torch.optim.Adam([w], lr=TRAIN_LR, fused=True)  # one kernel per update
    T, s = CFG["tile"], CFG["stride"]
    ng = lambda n: 1 if n <= T else -(-(n - T) // s) + 1
    grid = [(si, jy, jx) for si, k in enumerate(scales) for jy in range(ng(-(-REGION // (1 << k))))
            for jx in range(ng(-(-REGION // (1 << k))))]
    rng = np.random.default_rng(14)
    sp = torch.nn.functional.softplus
    losses = []

    def step(it):
        for g in opt.param_groups:  # 25 warm-up steps, then cosine decay
            g["lr"] = TRAIN_LR * min(1.0, (it + 1) / 25.0) * 0.5 * (1.0 + np.cos(np.pi * it / steps))
        tiles = [grid[i] for i in sorted(rng.choice(len(grid), size=batch, replace=False))]
        opt.zero_grad()
        logit, covered = om.OmniSegFn.apply(w, plan, slide, tiles, PAIRS)
        v = covered.to(torch.float32)  # mean over covered entries, without data-dependent indexing
        loss = ((pw * y * sp(-logit) + (1 - y) * sp(logit)) * v).sum() / v.sum()
        loss.backward()
        opt.step()
        losses.append(loss.detach())

    step(0)  # untimed: loads the code objects
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for it in range(1, steps):
        step(it)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(1, steps - 1)
    lv = [float(x) for x in losses]
    fwd_flops = 18.0 * CFG["base"] ** 2 * T * T * (3.0 / CFG["base"] + 1 + 5.5 * (CFG["levels"] - 1)) * batch
    rep = {"ms_per_step": ms, "tiles_per_step": batch, "grid_tiles": len(grid), "steps": steps,
           "dtype": "bf16 (FP32 master weights, Adam)", "tiles_per_s": batch / (ms * 1e-3),
           "algorithmic_tflop_per_step": 3 * fwd_flops / 1e12,
           "achieved_tflops": 3 * fwd_flops / (ms * 1e-3) / 1e12,
           "achieved_frac_bf16_peak": 3 * fwd_flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"],
           "loss_first10_last10": [float(np.mean(lv[:10])), float(np.mean(lv[-10:]))],
           "workload": f"{REGION}x{REGION} synthetic region with ground truth, {batch} random 256^2 tiles of "
                       "40x/20x/10x/5x per step, 6 classes x 4 scales, base-64 5-level U-Net, class-weighted BCE "
                       "on the stitched logits, hand-written backward, Adam (lr 1e-3, cosine)"}
    return rep, w.detach().contiguous()


# ---------------------------------------------------------------------------
# the headline: 16 slides in one call, one HIP graph
# ---------------------------------------------------------------------------

def batch16_leg(om, torch, slides, specs, flat_dev, steps, warmup, batch_tiles, autotune):
    """All kept tiles of 16 uneven slides, 4 scales and 6 classes through one
    omniseg_segment_slide call (graph-captured, ring logit store), against
    the same call without the graph and against one call per slide."""
    dev = slides[0].device
    plan = _plan(om, "bf16", batch_tiles, graph=True, ring=1)
    eager = _plan(om, "bf16", batch_tiles, ring=1)
    packed = plan.pack(flat_dev)
    ws = torch.empty(plan.workspace_bytes(slides, PAIRS), dtype=torch.uint8, device=dev)
    print(f"# 16-slide workspace {ws.numel() / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    outs = plan.alloc_outputs(slides, PAIRS)
    t_tune = time.perf_counter()
    if autotune:
        plan.autotune(slides, PAIRS, packed, ws)
    else:
        pin_conv_table(plan)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    for st in range(4):
        for lv in range(CFG["levels"]):
            eager.set_conv_tuning(st, lv, plan.get_conv_tuning(st, lv))
    side = torch.cuda.Stream()  # graphs are captured on a created stream
    batched = lambda: plan.segment(slides, PAIRS, packed, workspace=ws, outputs=outs, stream=side)
    for _ in range(warmup):
        batched()
    ms = _timed(torch, batched, steps, side)
    kept = _kept(om, plan, slides, PAIRS, ws)
    print(f"# batched (graph): {ms:.0f} ms for {kept} kept tiles", file=sys.stderr, flush=True)
    ref = [[m.clone() for m in row] for row in outs[0]]
    ms_eager = _timed(torch, lambda: eager.segment(slides, PAIRS, packed, workspace=ws, outputs=outs, stream=side),
                      1, side)
    same_eager = all(torch.equal(a, b) for ra, rb in zip(ref, outs[0]) for a, b in zip(ra, rb))

    def sequential():
        for i, sl in enumerate(slides):
            eager.segment([sl], PAIRS, packed, workspace=ws, outputs=([outs[0][i]], [outs[1][i]]), stream=side)

    ms_seq = _timed(torch, sequential, 1, side)
    same_seq = all(torch.equal(a, b) for ra, rb in zip(ref, outs[0]) for a, b in zip(ra, rb))
    print(f"# eager {ms_eager:.0f} ms, one call per slide {ms_seq:.0f} ms", file=sys.stderr, flush=True)
    eager.set_profiling(True)
    eager.segment(slides, PAIRS, packed, workspace=ws, outputs=outs, stream=side)
    records = eager.read_profile()
    eager.set_profiling(False)
    torch.cuda.synchronize()
    px = sum(sp["H"] * sp["W"] for sp in specs) * len(PAIRS)
    tuned = sorted({(r["stage"], r["level"], r["config"]) for r in records if r["config"] >= 0})
    st = stage_summary(records)
    r = {"workload": "16 synthetic slides (seeds 100-115), heights 2000-8000, widths 4000-40000, 10-60% tissue; "
                     "4 scales x 6 classes; 256 tiles at stride 128, foreground only; base-64 5-level U-Net + "
                     "dynamic head, ramp stitch; BF16; one call, one HIP graph, ring logit store",
         "slides": len(specs), "gigapixels_40x": sum(sp["H"] * sp["W"] for sp in specs) / 1e9,
         "pairs": len(PAIRS), "kept_tiles": kept, "workspace_gib": ws.numel() / 2**30,
         "graph_ms": ms, "eager_ms": ms_eager, "per_slide_calls_ms": ms_seq,
         "speedup_batched_vs_per_slide": ms_seq / ms, "speedup_graph_vs_eager": ms_eager / ms,
         "masks_equal": {"eager_vs_graph": same_eager, "per_slide_vs_graph": same_seq},
         "value": px / (ms * 1e-3) / 1e6, "per_slide_value": px / (ms_seq * 1e-3) / 1e6,
         "tflop_per_step": sum(x["flops"] for x in records) / 1e12,
         "conv_table": "autotuned on this workload" if autotune else "pinned (BENCH_CONV_TABLE)",
         "tune_s": t_tune, "stages": st, "roofline": roofline(om, records, "bf16"),
         "layers": layer_summary(records, 1),
         "conv_tiles": {f"{s_}{l}": list(om.conv_config(c)) for s_, l, c in tuned}}
    if "stitch" in st:
        r["roofline_stitch"] = dict(bound="hbm", achieved=st["stitch"]["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                                    frac=st["stitch"]["gbs"] / HBM_PEAK_GBS, traffic=None)
        sl = sorted(((x["ms"], x["bytes"]) for x in records if x["stage"] == "stitch"), reverse=True)
        r["stitch_launches"] = {"n": len(sl), "with_work": sum(1 for _, b in sl if b > 0),
                                "median_ms": sl[len(sl) // 2][0], "slowest_ms_gb": [[m, b / 1e9] for m, b in sl[:8]],
                                "empty_ms_total": sum(m for m, b in sl if b == 0)}
    del ws
    return r


# ---------------------------------------------------------------------------
# precision: trained weights, BF16 / FP8 against FP32 (whole slide) and the
# FP64 oracle (1024^2 crop)
# ---------------------------------------------------------------------------

def _cmp(M, masks, logits, ref_masks, ref_logits, covered):
    """Max logit error (normwise and absolute), per-plane Dice, the largest
    disagreement and the largest at-risk fraction: covered pixels whose
    reference logit lies within the plane's largest absolute error of the
    threshold (either mask value is correct there)."""
    dice, dis, risk, nerr, aerr = [], [], [], [], []
    for m, lg, rm, rl, cv in zip(masks, logits, ref_masks, ref_logits, covered):
        lg = np.asarray(lg, np.float64)
        rl = np.asarray(rl, np.float64)
        e = float(np.abs(lg - rl).max()) if lg.size else 0.0
        dice.append(M.dice(m, rm))
        dis.append(M.disagreement(m, rm))
        risk.append(float((np.abs(rl[cv]) <= e).mean()) if cv.any() else 0.0)
        nerr.append(M.normwise_error(lg, rl, cv))
        aerr.append(e)
    return {"dice_min": min(dice), "dice_mean": float(np.mean(dice)), "dice": [round(d, 6) for d in dice],
            "disagreement_max": max(dis), "at_risk_max": max(risk), "at_risk": [round(r, 6) for r in risk],
            "logit_error_normwise_max": max(nerr), "logit_abs_error_max": max(aerr)}


def precision_gpu(om, torch, M, dslide, dcrop, wt, batch_tiles):
    """GPU side of the precision leg with the trained weights: FP32, BF16
    and FP8 masks and logits of the whole slide and of the crop."""
    res, crop = {}, {}
    fp = run_leg(om, torch, dslide, wt, PAIRS, "fp32", 1, 0, batch_tiles, emit_logits=True, tune=False)
    bf = run_leg(om, torch, dslide, wt, PAIRS, "bf16", 1, 0, batch_tiles, emit_logits=True, tune=False)
    f8 = run_leg(om, torch, dslide, wt, PAIRS, "fp8", 1, 0, batch_tiles, emit_logits=True, tune=False)
    cov = fp["covered"]
    res["fp32_positive_fraction_mean"] = float(np.mean([m.mean() for m in fp["masks"]]))
    res["fp32_abs_logit_median_covered"] = float(np.median(np.concatenate(
        [np.abs(lg[c]) for lg, c in zip(fp["logits"], cov)])))
    res["bf16_vs_fp32"] = _cmp(M, bf["masks"], bf["logits"], fp["masks"], fp["logits"], cov)
    res["fp8_vs_fp32"] = _cmp(M, f8["masks"], f8["logits"], fp["masks"], fp["logits"], cov)
    for name, prec in (("fp32", "fp32"), ("bf16", "bf16"), ("fp8", "fp8")):
        r = run_leg(om, torch, dcrop, wt, PAIRS, prec, 1, 0, batch_tiles, emit_logits=True, tune=False)
        crop[name] = (r["masks"], r["logits"], r["covered"])
    return res, crop


def precision_vs_oracle(M, crop, ref):
    out = {}
    cov = crop["fp32"][2]
    for name in ("fp32", "bf16", "fp8"):
        masks, logits, _ = crop[name]
        out[f"{name}_vs_fp64"] = _cmp(M, masks, logits, ref["mask"], ref["logit"], cov)
    return out


# ---------------------------------------------------------------------------
# cpu_baseline: the FP64 oracle on the host cores, in a child process started
# before this process touches the GPU; it also supplies the FP64 reference
# planes of the precision crop
# ---------------------------------------------------------------------------

def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_worker(workdir):
    """Child process: the FP64 oracle on the 1024^2 crop (a stand-alone
    slide) with the trained weights the parent writes to workdir."""
    import synth
    from oracle import omniseg_oracle as O

    try:
        import threadpoolctl
    except ImportError:  # pragma: no cover
        threadpoolctl = None
    big, _ = synth.strip_slide(2, SLIDE, SLIDE, fg_frac=0.30, with_gt=False)
    y0, x0 = synth.strip_crop_origin(2, SLIDE, SLIDE, CROP)
    crop = np.ascontiguousarray(big[y0:y0 + CROP, x0:x0 + CROP])
    del big
    wpath = os.path.join(workdir, "weights.npy")
    t_wait = time.time()
    while not os.path.exists(wpath):
        if time.time() - t_wait > 1800 or os.getppid() == 1:
            sys.exit(3)
        time.sleep(0.2)
    flat = np.load(wpath)
    cfg = O.make_config(**CFG)
    threads = None
    if threadpoolctl is not None:
        threads = max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or None
    # single thread: one 40x tile (backbone, controller, 6-class head)
    wts = O.unpack_weights(flat, cfg)
    t1 = time.perf_counter()
    if threadpoolctl is not None:
        with threadpoolctl.threadpool_limits(1):
            O.tile_logits(O.tile_input(crop, 0, CFG["tile"], CFG["stride"], 1, 1), wts, cfg, 0, list(range(6)))
    else:  # pragma: no cover
        O.tile_logits(O.tile_input(crop, 0, CFG["tile"], CFG["stride"], 1, 1), wts, cfg, 0, list(range(6)))
    t_tile1 = time.perf_counter() - t1
    t0 = time.perf_counter()
    ref = O.segment([crop], flat, cfg, PAIRS)
    t_all = time.perf_counter() - t0
    arrays = {}
    for p in range(len(PAIRS)):
        arrays[f"logit{p}"] = ref["logit"][0][p]
        arrays[f"mask{p}"] = ref["mask"][0][p]
    np.savez(os.path.join(workdir, "ref.npz"), **arrays)
    info = {"seconds": t_all, "tiles": len(ref["tiles"]), "threads": threads, "single_thread_tile_s": t_tile1,
            "crop_origin": [y0, x0]}
    with open(os.path.join(workdir, "ref.json.tmp"), "w") as f:
        json.dump(info, f)
    os.replace(os.path.join(workdir, "ref.json.tmp"), os.path.join(workdir, "ref.json"))


def start_oracle_worker(workdir):
    env = dict(os.environ)
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", workdir], env=env)


def finish_cpu_baseline(proc, workdir, timeout_s):
    try:
        rc = proc.wait(timeout=timeout_s)
    except subprocess.TimeoutExpired:
        proc.kill()
        return None, None
    if rc != 0 or not os.path.exists(os.path.join(workdir, "ref.json")):
        return None, None
    with open(os.path.join(workdir, "ref.json")) as f:
        info = json.load(f)
    z = np.load(os.path.join(workdir, "ref.npz"))
    ref = {"logit": [z[f"logit{p}"] for p in range(len(PAIRS))], "mask": [z[f"mask{p}"] for p in range(len(PAIRS))]}
    px = CROP * CROP * len(PAIRS)
    base = {"value": px / info["seconds"] / 1e6, "unit": UNIT, "cores": info["threads"], "kind": "oracle",
            "sample": f"the whole {CROP}x{CROP} crop of the {SLIDE}^2 slide ({info['tiles']} kept tiles of 4 "
                      f"scales, 24 class-scale pairs) through the FP64 oracle with the trained weights: "
                      f"{info['seconds']:.1f} s, timed alongside the GPU legs",
            "cpu_model": _cpu_model(), "blas_threads": info["threads"], "host_cpus": os.cpu_count(),
            "single_thread": {"one_40x_tile_s": info["single_thread_tile_s"],
                              "value": CROP * CROP * len(PAIRS) / (info["single_thread_tile_s"] * info["tiles"]) / 1e6,
                              "note": "one tile timed at 1 BLAS thread, scaled by the crop's tile count"}}
    return base, ref


# Conv tile configuration of every backbone layer of the 16-slide workload,
# pinned so that every run launches the same kernels as the counter runs
# behind MEASURED_TRAFFIC (omniseg_autotune swaps near-equal configurations
# on timing noise).  Chosen per layer from this workload's own per-layer
# profile (BF16 TFLOP/s in the 16-slide call): the persistent large-block
# form (32 x 16 x 64, configuration 12) against the eight-wave 16 x 16 x 64
# form (10) and the one-block-per-workgroup large-block form (11): dec_a0
# 1142 (10) -> 1328, dec_a1 1347 (11) -> 1482, dec_a3 1485 (11) -> 1560,
# enc_a2 1004 -> 1091, enc_b2 1118 -> 1154, dec_b3 1319 -> 1374.  Configuration
# 10 keeps the layers with 64 input channels (enc_b0, dec_b0, enc_a1: its
# weight-stationary form) and level 4, whose 16-row tiles the 32-row block
# does not fit.
# Keys: (stage, level), stage 0 enc_a, 1 enc_b, 2 dec_a, 3 dec_b.
BENCH_CONV_DEFAULT = 10
BENCH_CONV_TABLE = {(2, 0): 12, (2, 1): 12, (2, 2): 12, (2, 3): 12, (1, 1): 12, (1, 2): 12, (1, 3): 12,
                    (0, 2): 12, (0, 3): 12, (3, 1): 12, (3, 2): 12, (3, 3): 12}


def pin_conv_table(plan):
    for stage in range(4):
        for level in range(CFG["levels"]):
            plan.set_conv_tuning(stage, level, BENCH_CONV_TABLE.get((stage, level), BENCH_CONV_DEFAULT))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed steps of the 16-slide call")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch-tiles", type=int, default=0)
    ap.add_argument("--slide-steps", type=int, default=5, help="timed BF16 steps on the single slide")
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--fp8-steps", type=int, default=3, help="FP8 leg on the single slide (0 = skip)")
    ap.add_argument("--train-steps", type=int, default=400,
                    help="training steps (the training-step timing and the trained weights of the precision leg)")
    ap.add_argument("--paper-steps", type=int, default=2,
                    help="leg with the paper's tiling (512 tiles, 40x/10x/5x, strides 256/64/64, "
                         "majority vote 1/4/4), BF16 and one FP32 step for the masks (0 = skip)")
    ap.add_argument("--map-reps", type=int, default=20,
                    help="aggregation and mapping leg (merge to 40x + overlay) repetitions (0 = skip)")
    ap.add_argument("--no-batch16", action="store_true", help="skip the 16-slide workload (headline: the slide)")
    ap.add_argument("--no-precision", action="store_true", help="skip the trained-weights precision leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle (cpu_baseline, FP64 crop)")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the 16-slide call's conv tiles instead of the pinned table")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="first copy this many GiB device to device (a plain copy of known size for "
                         "scaling profiler byte counters)")
    ap.add_argument("--counters", action="store_true",
                    help="profiler counter run through the stand-alone entry points: a 1 GiB device copy (the "
                         "byte counters' scale), one launch of every conv layer of the bench network on a full "
                         "256-tile batch with its pinned configuration, the stitch of one 8192^2 plane, the "
                         "merge and overlay of six classes; prints the launch list")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PATH",
                    help="FETCH_CSV WRITE_CSV COUNTERS_JSON [MFMA_CSV]: bytes per launch from FETCH_SIZE and "
                         "WRITE_SIZE passes of rocprofv3 --pmc over bench.py --counters (whose stdout is "
                         "COUNTERS_JSON), and MFMA busy per conv layer from a pass with SQ_VALU_MFMA_BUSY_CYCLES "
                         "and GRBM_GUI_ACTIVE; prints JSON")
    ap.add_argument("--oracle-worker", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.summarize_counters:
        print(json.dumps(summarize_counters(*args.summarize_counters)))
        return
    if args.oracle_worker:
        oracle_worker(args.oracle_worker)
        return
    if args.counters:
        counters_run(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not "
                                   "supported: the path runs on one GPU (--gpus must be 1)"}))
        sys.exit(2)
    t_start = time.perf_counter()
    log = lambda msg: print(f"# [{time.perf_counter() - t_start:6.1f} s] {msg}", file=sys.stderr, flush=True)

    # the CPU oracle runs in a child process started before this process
    # touches the GPU; it waits for the weights file
    workdir = tempfile.mkdtemp(prefix="omniseg_bench_")
    proc = None if args.no_cpu else start_oracle_worker(workdir)
    try:
        result = run(args, workdir, proc, log)
    finally:
        if proc is not None and proc.poll() is None:
            proc.kill()
    print(json.dumps(result))


def bench_conv_layers():
    """The 17 backbone convs of the bench network in forward order: (name,
    stage id, level, mode, cin, cu, cout, side, pooled copy)."""
    from paper_2305_14566_amd import omniseg as om

    C = [CFG["base"] << l for l in range(CFG["levels"])]
    S = [CFG["tile"] >> l for l in range(CFG["levels"])]
    out = []
    for l in range(CFG["levels"]):
        if l > 0:  # reads the pooled copy of the level above
            out.append((f"enc_a{l}", 0, l, om.CONV_RELU, C[l - 1], C[l - 1], C[l], S[l], False))
        out.append((f"enc_b{l}", 1, l, om.CONV_RES_RELU, C[l], C[l], C[l], S[l], l < CFG["levels"] - 1))
    for l in range(CFG["levels"] - 2, -1, -1):
        out.append((f"dec_a{l}", 2, l, om.CONV_UPCAT_RELU, 3 * C[l], 2 * C[l], C[l], S[l], False))
        out.append((f"dec_b{l}", 3, l, om.CONV_RES_RELU, C[l], C[l], C[l], S[l], False))
    return out


def counters_run(args, batch=256):
    """The launches behind the counter summaries in profiles/, through the
    stand-alone entry points: a 1 GiB device copy (the byte counters'
    scale); then, after a fill kernel that marks the phase, one launch of
    every backbone conv of the bench network on a full batch of 256 tiles
    (random non-negative BF16 activations, He-normal weights) with the
    configuration BENCH_CONV_TABLE pins (each preceded by its weight-packing
    kernel); the stitch of one 8192^2 40x plane from all its 63^2 tiles,
    mask and logit out (the mapping leg's stand-alone stitch); the merge to
    40x and the overlay of six classes on an 8192^2 slide.  Prints the
    launch list as JSON."""
    import torch

    from paper_2305_14566_amd import omniseg as om
    om.lib()
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(5)
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    out = {"copy_bytes": 1 << 30, "batch": batch, "layers": []}
    for name, stage, level, mode, cin, cu, cout, side, pool in bench_conv_layers():
        cfg = BENCH_CONV_TABLE.get((stage, level), BENCH_CONV_DEFAULT)
        if mode == om.CONV_UPCAT_RELU:
            x0 = torch.rand((batch, side // 2, side // 2, cu), generator=g).to(torch.bfloat16).to(dev)
            x1 = torch.rand((batch, side, side, cin - cu), generator=g).to(torch.bfloat16).to(dev)
        else:
            x0 = torch.rand((batch, side, side, cin), generator=g).to(torch.bfloat16).to(dev)
            x1 = None
        w = (torch.randn((cout, cin, 3, 3), generator=g) * (2.0 / (9 * cin)) ** 0.5).to(dev)
        b = torch.zeros(cout, device=dev)
        om.conv3x3(om.BF16, mode, x0, w, b, x1=x1, cu=cu if x1 is not None else None, config=cfg,
                   height=side, width=side, pool=pool)
        torch.cuda.synchronize()
        px = batch * side * side
        src_bytes = (batch * (side // 2) ** 2 * cu + px * (cin - cu)) * 2 if x1 is not None else px * cin * 2
        alg = src_bytes + px * cout * 2 + 9 * cin * cout * 2 + (px // 4 * cout * 2 if pool else 0)
        out["layers"].append([name, stage, level, cfg, 2.0 * 9 * cin * cout * px, float(alg)])
        del x0, x1
    torch.cuda.empty_cache()
    T, s_, H = CFG["tile"], CFG["stride"], SLIDE
    ny = (H - T + s_ - 1) // s_ + 1
    yx = torch.tensor([(j // ny, j % ny) for j in range(ny * ny)], dtype=torch.int32).to(dev)
    tl = torch.randn((yx.shape[0], T, T), generator=g).to(dev)
    om.stitch_tiles(T, s_, H, H, tl, yx, emit_logits=True)
    torch.cuda.synchronize()
    out["stitch"] = {"tiles": int(yx.shape[0]), "T": T, "s": s_, "side": H,
                     "alg_bytes": float(4 * yx.shape[0] * T * T + 5 * H * H)}
    del tl
    planes = []
    for c, si in enumerate(CLASS_SLOT):
        k = CFG["scales"][si]
        hk = (H + (1 << k) - 1) >> k
        planes.append((k, om.UPSAMPLE_BILINEAR, torch.randn((hk, hk), generator=g).to(dev)))
    rgb = torch.randint(0, 256, (H, H, 3), generator=g, dtype=torch.uint8).to(dev)
    m40 = om.merge_to_base(H, H, planes)
    om.overlay(rgb, [(m, 0, col, 128) for m, col in zip(m40, CLASS_COLOURS)])
    torch.cuda.synchronize()
    out["mapping"] = {"merge_alg_bytes": float(sum(4 * ((H + (1 << k) - 1) >> k) ** 2 + H * H for k, _, _ in planes)),
                      "overlay_alg_bytes": float(3 * H * H + 6 * H * H + 3 * H * H + 3 * ((H + 3) // 4) ** 2)}
    print(json.dumps(out))


def _counter_rows(path, counter):
    """Per-dispatch (kernel name, value) of one counter from a rocprofv3 CSV,
    in dispatch order."""
    import csv

    rows = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows[int(r["Dispatch_Id"])] = (r["Kernel_Name"].split("(")[0].replace("void ", ""),
                                               float(r["Counter_Value"]))
    return [rows[k] for k in sorted(rows)]


def _mfma_rows(path):
    """Per-dispatch (kernel, MFMA busy cycles summed over SIMDs, GUI active
    cycles summed over XCDs, elapsed ns) from a rocprofv3 CSV."""
    import csv

    rows = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = rows.setdefault(int(r["Dispatch_Id"]), {"k": r["Kernel_Name"].split("(")[0].replace("void ", ""),
                                                         "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
    return [rows[k] for k in sorted(rows)]


def summarize_counters(fetch_csv, write_csv, launches_json, mfma_csv=None):
    """Bytes per launch from a FETCH_SIZE and a WRITE_SIZE pass over
    `bench.py --counters` (whose stdout is launches_json): each counter
    scaled by its reading for the leading 1 GiB device copy; the conv
    launches matched in order with the layer list, the stitch and the merge
    and overlay kernels by name.  With mfma_csv (a
    pass with SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE over the same
    command) also the MFMA busy fraction of every conv layer."""
    import hashlib

    with open(launches_json) as f:
        L = json.loads([ln for ln in f if ln.startswith("{")][-1])
    fetch = _counter_rows(fetch_csv, "FETCH_SIZE")
    write = _counter_rows(write_csv, "WRITE_SIZE")
    assert [k for k, _ in fetch] == [k for k, _ in write], "the two passes saw different dispatches"
    names = [k for k, _ in fetch]
    copy = max(range(len(names)), key=lambda i: fetch[i][1] if "omniseg" not in names[i] else -1)
    f_scale = L["copy_bytes"] / (fetch[copy][1] * 1024)
    w_scale = L["copy_bytes"] / (write[copy][1] * 1024)
    nb = lambda i: (fetch[i][1] * 1024 * f_scale, write[i][1] * 1024 * w_scale)
    out = {"scale": {"fetch": f_scale, "write": w_scale, "copy_kernel": names[copy]}, "batch": L["batch"]}
    convs = [i for i in range(len(names)) if "k_conv3x3" in names[i]]
    assert len(convs) == len(L["layers"]), (len(convs), len(L["layers"]))
    out["conv_layers"] = {}
    for (name, stage, level, cfg, flops, alg), i in zip(L["layers"], convs):
        f, w = nb(i)
        out["conv_layers"][name] = dict(kernel=names[i], config=cfg, fetch=f, write=w, alg=alg)
    for ph, keys in (("stitch", ("k_stitch", "k_grid")), ("mapping", ("k_merge", "k_overlay"))):
        kern = {}
        for i in range(len(names)):
            if not any(k in names[i] for k in keys):
                continue
            f, w = nb(i)
            g = kern.setdefault(names[i], dict(n=0, fetch=0.0, write=0.0))
            g["n"] += 1
            g["fetch"] += f
            g["write"] += w
        out[ph] = {"kernels": kern, **L[ph]}
    if mfma_csv:
        m = _mfma_rows(mfma_csv)
        mconvs = [i for i, d in enumerate(m) if "k_conv3x3" in d["k"]]
        assert len(mconvs) == len(L["layers"]), ("mfma", len(mconvs), len(L["layers"]))
        for (name, stage, level, cfg, flops, alg), i in zip(L["layers"], mconvs):
            d = m[i]
            gui = d["GRBM_GUI_ACTIVE"] / 8  # summed over the 8 XCDs
            out["conv_layers"][name].update(
                mfma_busy_nominal=d["SQ_VALU_MFMA_BUSY_CYCLES"] / (d["ns"] * 2.4 * 1024),
                mfma_busy_active=d["SQ_VALU_MFMA_BUSY_CYCLES"] / (gui * 1024),
                clock_ghz=gui / d["ns"], tflops_profiled=flops / d["ns"] / 1e3)
    src = os.path.join(ROOT, "paper_2305_14566_amd", "csrc", "k_conv.hip")
    with open(src, "rb") as f:
        out["conv_source_sha256"] = hashlib.sha256(f.read()).hexdigest()
    return out


def run(args, workdir, proc, log):
    import concurrent.futures

    import synth

    specs = synth.batch_slide_specs(99, 16)
    jobs = ([] if args.no_batch16 else [("batch", sp) for sp in specs]) + [("slide", SLIDE), ("region", None)]
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        made = list(ex.map(_gen_input, jobs))
    gen_s = time.perf_counter() - t0
    batch_rgb = made[:-2]
    rgb, (region_rgb, region_gt) = made[-2], made[-1]
    log(f"inputs generated in {gen_s:.1f} s")

    import torch

    from paper_2305_14566_amd import metrics as M
    from paper_2305_14566_amd import omniseg as om

    om.lib()  # fails loudly without the HIP library
    dev = torch.device("cuda:0")
    if args.copy_gib > 0:
        n = int(args.copy_gib * 2 ** 30) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {n * 4} bytes device to device")
        del src, dst
    flat = synth.he_normal_weights(12, CFG["base"], CFG["levels"], CFG["n_classes"], len(CFG["scales"]),
                                   CFG["head_out"])
    flat_dev = torch.from_numpy(flat).to(dev)
    dslide = torch.from_numpy(rgb).to(dev)
    y0, x0 = synth.strip_crop_origin(2, SLIDE, SLIDE, CROP)
    dcrop = torch.from_numpy(np.ascontiguousarray(rgb[y0:y0 + CROP, x0:x0 + CROP])).to(dev)
    out = {}

    # 1. training step; its weights feed the precision leg and the CPU oracle
    wt = None
    if args.train_steps > 0:
        out["train_step"], wt = train_leg(om, torch, region_rgb, region_gt, args.train_steps)
        log(f"train: {out['train_step']['ms_per_step']:.1f} ms/step, loss {out['train_step']['loss_first10_last10']}")
    w_cpu = (wt.cpu().numpy() if wt is not None else flat).astype(np.float32)
    if proc is not None:
        np.save(os.path.join(workdir, "weights.tmp.npy"), w_cpu)
        os.replace(os.path.join(workdir, "weights.tmp.npy"), os.path.join(workdir, "weights.npy"))

    # 2. the headline: 16 slides in one graph-captured call
    if not args.no_batch16:
        dslides = [torch.from_numpy(r).to(dev) for r in batch_rgb]
        del batch_rgb
        b16 = batch16_leg(om, torch, dslides, specs, flat_dev, args.steps, args.warmup, args.batch_tiles,
                          args.autotune)
        del dslides
        torch.cuda.empty_cache()
        log(f"16 slides: {b16['graph_ms']:.0f} ms per call, {b16['value']:.0f} {UNIT}")

    # 3. the single 8192^2 slide: BF16, plain FP32, FP8 (He-normal weights)
    bf = run_leg(om, torch, dslide, flat_dev, PAIRS, "bf16", args.slide_steps, 1, args.batch_tiles)
    fp = run_leg(om, torch, dslide, flat_dev, PAIRS, "fp32", args.fp32_steps, 1, args.batch_tiles)
    px1 = SLIDE * SLIDE * len(PAIRS)
    fp32_value = px1 / (fp["ms"] * 1e-3) / 1e6
    log(f"slide: bf16 {bf['ms']:.1f} ms, fp32 {fp['ms']:.1f} ms")
    slide = {"workload": f"one {SLIDE}x{SLIDE} synthetic 40x slide (strip, ~30% tissue), 4 scales x 6 classes, "
                         "256 tiles at stride 128, foreground tiles only, base-64 5-level U-Net + dynamic head, "
                         "ramp stitch; He-normal weights (seed 12)",
             "kept_tiles": bf["kept"],
             "bf16": {"value": px1 / (bf["ms"] * 1e-3) / 1e6, "ms_per_step": bf["ms"], "steps": args.slide_steps,
                      "stages": stage_summary(bf["records"]), "roofline": roofline(om, bf["records"], "bf16"),
                      "conv_tiles": bf["tuned"]},
             "fp32_plain": {"value": fp32_value, "ms_per_step": fp["ms"], "steps": args.fp32_steps,
                            "roofline": roofline(om, fp["records"], "fp32"), "conv_tiles": fp["tuned"]},
             "speedup_bf16_vs_fp32": fp["ms"] / bf["ms"],
             "bf16_vs_fp32_masks_he_normal": {
                 "dice_min": min(M.dice(a, b) for a, b in zip(bf["masks"], fp["masks"])),
                 "disagreement_max": max(M.disagreement(a, b) for a, b in zip(bf["masks"], fp["masks"]))}}
    if args.fp8_steps > 0:
        f8 = run_leg(om, torch, dslide, flat_dev, PAIRS, "fp8", args.fp8_steps, 1, args.batch_tiles)
        slide["fp8"] = {"value": px1 / (f8["ms"] * 1e-3) / 1e6, "ms_per_step": f8["ms"], "steps": args.fp8_steps,
                        "dtype": "fp8 e4m3 (per-channel power-of-two scales), FP32 accumulation",
                        "calibration": f"{f8['calibration_tiles']} first kept tiles on the FP32 path",
                        "roofline": roofline(om, f8["records"], "fp8"), "speedup_vs_bf16": bf["ms"] / f8["ms"],
                        "stages": stage_summary(f8["records"])}
        log(f"slide: fp8 {f8['ms']:.1f} ms")
    out["slide"] = slide

    # 4. precision with trained weights (GPU side)
    crop = None
    if not args.no_precision and wt is not None:
        out["precision"], crop = precision_gpu(om, torch, M, dslide, dcrop, wt, args.batch_tiles)
        log("precision: GPU side done")

    # 5. the paper's tiling, and mapping
    if args.paper_steps > 0:
        out["paper_tiling"] = paper_leg(om, torch, M, dslide, SLIDE, args.paper_steps, args.batch_tiles)
        log(f"paper tiling: {out['paper_tiling']['ms_per_step']:.1f} ms/step")
    if args.map_reps > 0:
        out["mapping"] = mapping_leg(om, torch, dslide, flat_dev, SLIDE, args.map_reps, args.batch_tiles)
        log(f"mapping: merge {out['mapping']['merge_ms']:.2f} ms, overlay {out['mapping']['overlay_ms']:.2f} ms, "
            f"stand-alone stitch {out['mapping']['stitch_standalone']['ms']:.3f} ms")

    # 6. the CPU oracle: cpu_baseline and the FP64 crop
    cpu = None
    if proc is not None:
        log("waiting for the CPU oracle")
        cpu, ref = finish_cpu_baseline(proc, workdir, 1500)
        log("CPU oracle done" if cpu else "CPU oracle failed")
        if cpu and crop is not None:
            out["precision"].update({"crop": f"{CROP}x{CROP} window at {list(synth.strip_crop_origin(2, SLIDE, SLIDE, CROP))} "
                                             "of the slide, a stand-alone slide (60 tiles over 4 scales)"})
            out["precision"].update(precision_vs_oracle(M, crop, ref))

    # the JSON line
    if not args.no_batch16:
        head = b16
        value, ms, cfgd = b16["value"], b16["graph_ms"], {
            "workload": b16["workload"], "slides": 16, "pairs": len(PAIRS), "kept_tiles": b16["kept_tiles"],
            "gigapixels_40x": b16["gigapixels_40x"], "tflop_per_step": b16["tflop_per_step"]}
        steps, warm = args.steps, args.warmup
    else:
        head = None
        value, ms, cfgd = slide["bf16"]["value"], bf["ms"], {"workload": slide["workload"], "slides": 1,
                                                            "pairs": len(PAIRS), "kept_tiles": bf["kept"]}
        steps, warm = args.slide_steps, 1
    result = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": steps, "warmup": warm,
              "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "bf16", "data": "synthetic", "config": cfgd,
              "roofline": head["roofline"] if head else slide["bf16"]["roofline"],
              "fp32_plain": {"value": fp32_value, "workload": f"the single {SLIDE}^2 slide, FP32 backbone",
                             "bf16_batched_over_fp32_plain": value / fp32_value}}
    prec = out.get("precision", {})
    if "bf16_vs_fp64" in prec:
        q = prec["bf16_vs_fp64"]
        result["qualifier"] = {"dice_target": 0.999, "bf16_dice_min_vs_fp64": q["dice_min"],
                               "bf16_at_risk_max": q["at_risk_max"],
                               "bf16_logit_error_normwise": q["logit_error_normwise_max"],
                               "met": q["dice_min"] >= 0.999,
                               "on": f"the {CROP}^2 crop, trained weights ({args.train_steps} steps)"}
    if head:
        result["batch16"] = {k: v for k, v in head.items() if k not in ("roofline",)}
    result.update(out)
    if cpu:
        result["cpu_baseline"] = cpu
    return result


if __name__ == "__main__":
    main()

"""Merge to the 40x base and colour mapping on the GPU, against the oracle.

Nearest merges and the overlay are integer work and must match bit for bit;
the bilinear merge samples in FP32 (the oracle in FP64), so its masks must
match wherever the oracle's interpolated value is not within rounding of 0.
The chained test runs segment -> merge -> overlay and compares pixels whose
class masks are certain on both sides.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import omniseg_oracle as O
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("H,W", [(64, 64), (203, 131), (1, 9), (517, 300)])
def test_merge_to_base(H, W):
    print(f"merge H={H} W={W}", flush=True)
    rng = np.random.default_rng(H + W)
    planes, refs = [], []
    for k in range(4):
        Hk, Wk = O.level_size(H, k), O.level_size(W, k)
        m = (rng.uniform(size=(Hk, Wk)) < 0.4).astype(np.uint8) * rng.integers(1, 255, size=(Hk, Wk)).astype(np.uint8)
        lam = rng.standard_normal((Hk, Wk)).astype(np.float32)
        lam[rng.uniform(size=lam.shape) < 0.05] = 0.0
        planes.append((k, om.UPSAMPLE_NEAREST, torch.from_numpy(m).to(DEV)))
        refs.append(("n", O.upsample_nearest(m, k, H, W), None))
        planes.append((k, om.UPSAMPLE_BILINEAR, torch.from_numpy(lam).to(DEV)))
        v = O.upsample_bilinear(lam.astype(np.float64), k, H, W)
        refs.append(("b", v > 0, np.abs(v) <= 1e-5))
    outs = om.merge_to_base(H, W, planes)
    torch.cuda.synchronize()
    for (kind, want, risky), got in zip(refs, outs):
        g = got.cpu().numpy().astype(bool)
        if kind == "n":
            assert np.array_equal(g, want)
        else:
            assert np.array_equal(g[~risky], want[~risky])


@pytest.mark.parametrize("H,W", [(64, 512), (97, 1000), (200, 4160), (1500, 96)])
def test_merge_run_form_equals_pixel_form(H, W):
    """Sixteen-pixel run form (contiguous outputs, aligned sources) against
    the per-pixel form (outputs with an odd row stride), bit for bit, for
    bilinear and nearest planes at k = 0..3, with aligned and unaligned
    source rows; the comparison includes the pixels whose value is ~0.
    At 1500 rows each workgroup takes a band of six rows, so the run form
    carries source rows from one output row to the next."""
    print(f"merge run vs pixel H={H} W={W}", flush=True)
    rng = np.random.default_rng(3 * H + W)
    planes = []
    for k in range(4):
        Hk, Wk = O.level_size(H, k), O.level_size(W, k)
        for pad in (0, 3):  # pad 3: source rows not 16-byte aligned
            lam = rng.standard_normal((Hk, Wk + pad)).astype(np.float32)
            lam[rng.uniform(size=lam.shape) < 0.05] = 0.0
            planes.append((k, om.UPSAMPLE_BILINEAR, torch.from_numpy(lam).to(DEV)[:, :Wk]))
            m = (rng.uniform(size=(Hk, Wk + pad)) < 0.4).astype(np.uint8)
            planes.append((k, om.UPSAMPLE_NEAREST, torch.from_numpy(m).to(DEV)[:, :Wk]))
    fast = om.merge_to_base(H, W, planes)
    wide = torch.zeros((len(planes), H, W + 1), dtype=torch.uint8, device=DEV)
    slow = om.merge_to_base(H, W, planes, outs=[wide[i, :, :W] for i in range(len(planes))])
    torch.cuda.synchronize()
    for i, (f, s) in enumerate(zip(fast, slow)):
        assert torch.equal(f, s), i
    assert not wide[:, :, W].any()


@pytest.mark.parametrize("H,W,in_place", [(64, 64, False), (203, 131, False), (5, 3, False), (130, 97, True),
                                           (130, 100, True), (37, 256, False)])
def test_overlay_bit_exact(H, W, in_place):
    print(f"overlay H={H} W={W} in_place={in_place}", flush=True)
    rng = np.random.default_rng(7 * H + W)
    rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
    classes, dev = [], []
    for c in range(6):
        k = c % 4
        m = (rng.uniform(size=(O.level_size(H, k), O.level_size(W, k))) < 0.3).astype(np.uint8)
        col = tuple(int(v) for v in rng.integers(0, 256, 3))
        a = int(rng.integers(0, 257))
        classes.append((m, k, col, a))
        dev.append((torch.from_numpy(m).to(DEV), k, col, a))
    want = O.overlay(rgb, classes)
    slide = torch.from_numpy(rgb).to(DEV)
    out, o10 = om.overlay(slide, dev, out=slide if in_place else None)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    assert np.array_equal(o10.cpu().numpy(), O.map_10x(want))


def test_segment_merge_overlay_chain():
    """segment (ramp, 3 scales) -> per-class merge (bilinear and nearest) -> overlay."""
    rgb, _ = synth.strip_slide(61, 260, 330, fg_frac=0.4)
    cfg = O.make_config(base=8, levels=3, head_out=2, n_classes=3, scales=(0, 1, 2), tile=64, stride=32,
                        fg_filter=True)
    flat = synth.he_normal_weights(62, 8, 3, 3, 3, 2, bias_std=0.05)
    pairs = [(0, 2), (1, 1), (2, 0)]  # each class at its own scale
    plan = om.Plan(base=8, levels=3, head_out=2, n_classes=3, scales=(0, 1, 2), tile=64, stride=32,
                   fg_filter=True, emit_logits=True)
    slide = torch.from_numpy(rgb).to(DEV)
    packed = plan.pack(torch.from_numpy(flat).to(DEV))
    masks, logits, _ = plan.segment([slide], pairs, packed)
    ref = O.segment([rgb], flat, cfg, pairs)
    H, W = rgb.shape[:2]
    modes = [om.UPSAMPLE_BILINEAR, om.UPSAMPLE_NEAREST, om.UPSAMPLE_BILINEAR]
    planes = [(cfg["scales"][si], md, logits[0][p] if md == om.UPSAMPLE_BILINEAR else masks[0][p])
              for p, ((c, si), md) in enumerate(zip(pairs, modes))]
    m40 = om.merge_to_base(H, W, planes)
    colours = [((255, 0, 0), 160), ((0, 255, 0), 160), ((0, 0, 255), 160)]
    out, o10 = om.overlay(slide, [(m, 0, col, a) for m, (col, a) in zip(m40, colours)])
    torch.cuda.synchronize()
    sure = np.ones((H, W), bool)
    ref_classes = []
    for p, ((c, si), md) in enumerate(zip(pairs, modes)):
        k = cfg["scales"][si]
        lam = ref["logit"][0][p]
        err = np.abs(logits[0][p].cpu().numpy().astype(np.float64) - lam).max()
        if md == om.UPSAMPLE_BILINEAR:
            v = O.upsample_bilinear(lam, k, H, W)
            want = v > 0
            sure &= np.abs(v) > 2 * err + 1e-6
        else:
            want = O.upsample_nearest(ref["mask"][0][p], k, H, W)
            sure &= O.upsample_nearest(np.abs(lam) > 2 * err + 1e-6, k, H, W)
        got = m40[p].cpu().numpy().astype(bool)
        assert np.array_equal(got[sure], want[sure]), p
        ref_classes.append((want, 0) + colours[p])
    assert sure.mean() > 0.8  # the comparison covers most of the slide
    want_rgb = O.overlay(rgb, ref_classes)
    assert np.array_equal(out.cpu().numpy()[sure], want_rgb[sure])


def test_overlay_word_path_with_ragged_block():
    """Rows whose pitch is a multiple of 4 take the word-wide path; a width of
    4k + 2 leaves a partial last block that goes pixel by pixel."""
    H, W = 45, 98
    rng = np.random.default_rng(77)
    big = rng.integers(0, 256, size=(H, W + 2, 3)).astype(np.uint8)  # row pitch 300 bytes
    rgb = np.ascontiguousarray(big[:, :W])
    classes = []
    for c in range(3):
        k = c
        m = (rng.uniform(size=(O.level_size(H, k), O.level_size(W, k) + 4)) < 0.4).astype(np.uint8)
        classes.append((m, k, (int(rng.integers(256)), 40 * c, 255 - 30 * c), int(rng.integers(0, 257))))
    dslide = torch.from_numpy(big).to(DEV)[:, :W]
    out_big = torch.zeros((H, W + 2, 3), dtype=torch.uint8, device=DEV)
    dev = [(torch.from_numpy(m).to(DEV)[:, :O.level_size(W, k)], k, col, a) for (m, k, col, a) in classes]
    out, o10 = om.overlay(dslide, dev, out=out_big[:, :W])
    torch.cuda.synchronize()
    ref_classes = [(m[:, :O.level_size(W, k)], k, col, a) for (m, k, col, a) in classes]
    want = O.overlay(rgb, ref_classes)
    assert np.array_equal(out_big[:, :W].cpu().numpy(), want)
    assert np.array_equal(o10.cpu().numpy(), O.map_10x(want))
    assert not out_big[:, W:].any()  # nothing written past the width

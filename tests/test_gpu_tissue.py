"""Otsu tissue detection on the GPU against the oracle, bit for bit.

Every step is integer work except the Otsu score, which both sides evaluate
in FP64 with the same operations in the same order; the blurred gray map,
the threshold, the component counts, the tissue map and the tile list must
all match exactly.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import omniseg_oracle as O
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _speckled(seed, H, W):
    """A strip slide with dark specks on the background (tiny noise components)."""
    rgb, _ = synth.strip_slide(seed, H, W, fg_frac=0.3)
    rng = np.random.default_rng(seed)
    n = H * W // 4000
    ys, xs = rng.integers(0, H - 3, n), rng.integers(0, W - 3, n)
    for y, x in zip(ys, xs):
        rgb[y:y + 3, x:x + 3] = (150, 90, 130)
    return rgb


def _run(slides, scales, median, min_area, tile=32, stride=16):
    cfg = O.make_config(base=4, levels=1, head_out=1, n_classes=1, scales=scales, tile=tile, stride=stride,
                        fg_filter=True, tissue_method="otsu", median_kernel=median, min_tissue_area=min_area)
    plan = om.Plan(base=4, levels=1, head_out=1, n_classes=1, scales=scales, tile=tile, stride=stride,
                   fg_filter=True, tissue_method=om.TISSUE_OTSU, median_kernel=median, min_tissue_area=min_area)
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    flat = synth.he_normal_weights(7, 4, 1, 1, len(scales), 1)
    pairs = [(0, 0)]
    packed = plan.pack(torch.from_numpy(flat).to(DEV))
    masks, _, ws = plan.segment(ds, pairs, packed)
    torch.cuda.synchronize()

    def region(r, i=0):
        off, nb = plan.region(ds, pairs, r, i)
        return ws[off:off + nb].cpu().numpy()
    return cfg, region, masks


# (scales, median, min_area, specks removed): at 40x a 3 x 3 median turns each
# 3 x 3 speck into a 5-pixel cross, which min_area 6 removes
@pytest.mark.parametrize("scales,median,min_area,drop", [((0, 1, 2, 3), 9, 20, False), ((0, 2), 5, 0, False),
                                                         ((0, 1), 1, 3, False), ((0,), 3, 6, True),
                                                         ((0, 3), 59, 50, False)])
def test_otsu_tissue_map_bit_exact(scales, median, min_area, drop):
    print(f"otsu tissue scales={scales} median={median} min_area={min_area}", flush=True)
    slides = [_speckled(51, 700, 900), _speckled(52, 333, 517)]
    cfg, region, _ = _run(slides, scales, median, min_area)
    kc = max(scales)
    fgs = []
    for i, rgb in enumerate(slides):
        fg, blurred, (t, comps, kept) = O.tissue_map_otsu(rgb, kc, median, min_area)
        gray = region(om.REGION_TISSUE_GRAY, i).reshape(blurred.shape)
        assert np.array_equal(gray, blurred.astype(np.uint8)), i
        st = region(om.REGION_TISSUE_STATS, i).view(np.int32)
        assert list(st) == [t, comps, kept, 0], (i, list(st), (t, comps, kept))
        got = region(om.REGION_TISSUE, i).reshape(fg.shape).astype(bool)
        assert np.array_equal(got, fg), i
        fgs.append(fg)
        assert kept <= comps
        if drop:
            assert comps - kept >= 20  # the specks are removed
    ref_list = O.tile_list([s.shape[:2] for s in slides], cfg, fgs)
    cnt = int(region(om.REGION_TILE_COUNT).view(np.int32)[0])
    got = region(om.REGION_TILE_LIST).view(np.int32).reshape(-1, 4)[:cnt]
    assert [tuple(t) for t in got] == ref_list


def test_otsu_uniform_slide_has_no_tissue():
    rgb = np.full((96, 130, 3), 231, np.uint8)
    _, region, masks = _run([rgb], (0, 1), 3, 0)
    assert list(region(om.REGION_TISSUE_STATS).view(np.int32)) == [-1, 0, 0, 0]
    assert not region(om.REGION_TISSUE).any()
    assert int(region(om.REGION_TILE_COUNT).view(np.int32)[0]) == 0
    assert not masks[0][0].any()

"""Majority-vote merge and per-scale tile strides on the GPU, against the oracle.

The vote counts are integers: the stand-alone stitch, fed the same FP32 tile
logits as the oracle, must match it bit for bit (the decision logit > 0 is
taken on the same FP32 values).  Through the whole path the tile logits
differ from the FP64 oracle's by rounding, so a pixel's count may differ by
at most the number of covering tiles whose reference logit lies within the
measured logit error of zero, and the masks must agree wherever no such tile
covers the pixel.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import omniseg_oracle as O
from paper_2305_14566_amd import metrics as M
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
FP32_TOL = 1e-4


def _tiles(H, W, T, s, keep, rng):
    ny, nx = O.grid_count(H, T, s), O.grid_count(W, T, s)
    return [(jy, jx) for jy in range(ny) for jx in range(nx) if rng.uniform() < keep]


@pytest.mark.parametrize("H,W,T,s,keep,thr", [(300, 217, 64, 32, 0.7, 1), (300, 217, 64, 32, 0.7, 3),
                                              (97, 250, 32, 8, 0.9, 4), (128, 128, 128, 64, 1.0, 2),
                                              (200, 130, 64, 64, 0.8, 1), (5, 3, 16, 8, 1.0, 1),
                                              (1100, 600, 512, 64, 1.0, 4), (150, 133, 32, 7, 0.8, 3)])
def test_stitch_vote_bit_exact(H, W, T, s, keep, thr):
    print(f"vote stitch H={H} W={W} T={T} s={s} thr={thr}", flush=True)
    rng = np.random.default_rng(H * 7 + W + thr)
    tiles = _tiles(H, W, T, s, keep, rng)
    # small integers: about a fifth of the logits are exactly zero (no vote)
    logits = rng.integers(-2, 3, size=(len(tiles), T, T)).astype(np.float32)
    logits[::2] += rng.standard_normal((len(logits[::2]), T, T)).astype(np.float32) * 1e-3
    yx = torch.tensor(np.array(tiles, np.int32).reshape(-1, 2), device=DEV)
    mask, cnt = om.stitch_tiles(T, s, H, W, torch.from_numpy(logits).to(DEV), yx, vote_threshold=thr)
    torch.cuda.synchronize()
    V, C = O.vote(tiles, [l.astype(np.float64) for l in logits], H, W, T, s)
    assert np.array_equal(cnt.cpu().numpy(), V.astype(np.float32))
    assert np.array_equal(mask.cpu().numpy().astype(bool), V >= thr)


def test_stitch_vote_tall_plane():
    """Rows beyond the largest launch extent in y are covered too."""
    H, W, T, s = 70000, 20, 16, 8
    rng = np.random.default_rng(5)
    tiles = _tiles(H, W, T, s, 0.95, rng)
    logits = rng.standard_normal((len(tiles), T, T)).astype(np.float32)
    yx = torch.tensor(np.array(tiles, np.int32), device=DEV)
    lg = torch.from_numpy(logits).to(DEV)
    mask, cnt = om.stitch_tiles(T, s, H, W, lg, yx, vote_threshold=2)
    mr, lam = om.stitch_tiles(T, s, H, W, lg, yx)
    torch.cuda.synchronize()
    V, _ = O.vote(tiles, [l.astype(np.float64) for l in logits], H, W, T, s)
    assert np.array_equal(cnt.cpu().numpy(), V.astype(np.float32))
    assert np.array_equal(mask.cpu().numpy().astype(bool), V >= 2)
    ref, N, D = O.stitch(tiles, [l.astype(np.float64) for l in logits], H, W, T, s)
    g = lam.cpu().numpy().astype(np.float64)
    cov = D > 0
    assert np.abs(g[cov] - ref[cov]).max() <= 1e-5 * max(np.abs(ref[cov]).max(), 1.0)
    assert np.all(g[~cov] == 0) and (~cov).any()


# ------------------------------------------------------------------ whole path

def _case(merge):
    a, _ = synth.strip_slide(41, 300, 517, fg_frac=0.25)
    b, _ = synth.strip_slide(42, 129, 64, fg_frac=0.5)
    kw = dict(base=8, levels=3, head_out=2, n_classes=3, scales=(0, 2, 3), tile=64, stride=32,
              fg_filter=True, scale_strides=(32, 8, 8))
    if merge == "vote":
        kw.update(merge="vote", vote_thresholds=(1, 4, 4))
    cfg = O.make_config(**kw)
    flat = synth.he_normal_weights(43, 8, 3, 3, 3, 2, bias_std=0.05)
    pairs = [(0, 0), (2, 1), (1, 2), (1, 0)]
    return [a, b], cfg, flat, pairs


def _run(cfg, slides, flat, pairs):
    plan = om.Plan(base=cfg["base"], levels=cfg["levels"], head_out=cfg["head_out"],
                   n_classes=cfg["n_classes"], scales=cfg["scales"], tile=cfg["tile"], stride=cfg["stride"],
                   fg_filter=cfg["fg_filter"], emit_logits=True, scale_strides=cfg["scale_strides"],
                   merge=om.MERGE_VOTE if cfg["merge"] == "vote" else om.MERGE_RAMP,
                   vote_thresholds=cfg["vote_thresholds"])
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    packed = plan.pack(torch.from_numpy(flat).to(DEV))
    masks, logits, ws = plan.segment(ds, pairs, packed)
    torch.cuda.synchronize()
    return plan, ds, masks, logits, ws


def _region(plan, ds, pairs, ws, region, index=0):
    off, nb = plan.region(ds, pairs, region, index)
    return ws[off:off + nb].cpu().numpy()


def _tile_logit_error(plan, ds, pairs, ws, ref, T):
    slots = {}
    for (c, si) in pairs:
        slots.setdefault(si, []).append(c)
    ms = max(len(v) for v in slots.values())
    tl = _region(plan, ds, pairs, ws, om.REGION_TILE_LOGITS).view(np.float32)
    tl = tl[:len(ref["tiles"]) * ms * T * T].reshape(-1, ms, T, T)
    worst, amax = 0.0, 0.0
    for li, t in enumerate(ref["tiles"]):
        for j, c in enumerate(slots.get(t[1], [])):
            r = ref["tile_logits"][t][c]
            worst = max(worst, M.normwise_error(tl[li, j], r))
            amax = max(amax, float(np.abs(tl[li, j] - r).max()))
    return worst, amax


@pytest.mark.parametrize("merge", ["vote", "ramp"])
def test_per_scale_strides_end_to_end(merge):
    print(f"per-scale strides, merge={merge}", flush=True)
    slides, cfg, flat, pairs = _case(merge)
    plan, ds, masks, logits, ws = _run(cfg, slides, flat, pairs)
    ref = O.segment(slides, flat, cfg, pairs, keep_tiles=True)
    T = cfg["tile"]
    # integer steps: the tile list and every (slide, slot) index grid, bit for bit
    cnt = int(_region(plan, ds, pairs, ws, om.REGION_TILE_COUNT).view(np.int32)[0])
    assert cnt == len(ref["tiles"])
    got = _region(plan, ds, pairs, ws, om.REGION_TILE_LIST).view(np.int32).reshape(-1, 4)[:cnt]
    assert [tuple(t) for t in got] == ref["tiles"]
    for i, rgb in enumerate(slides):
        for si, k in enumerate(cfg["scales"]):
            s = cfg["scale_strides"][si]
            ny = O.grid_count(O.level_size(rgb.shape[0], k), T, s)
            nx = O.grid_count(O.level_size(rgb.shape[1], k), T, s)
            idx = _region(plan, ds, pairs, ws, om.REGION_TILE_INDEX, i * 3 + si).view(np.int32)
            want = -np.ones(ny * nx, np.int32)
            for li, t in enumerate(ref["tiles"]):
                if t[0] == i and t[1] == si:
                    want[t[2] * nx + t[3]] = li
            assert np.array_equal(idx, want), (i, si)
    err, amax = _tile_logit_error(plan, ds, pairs, ws, ref, T)
    assert err <= FP32_TOL, err
    for i in range(len(slides)):
        for p, (c, si) in enumerate(pairs):
            m = masks[i][p].cpu().numpy().astype(bool)
            lg = logits[i][p].cpu().numpy().astype(np.float64)
            if merge == "ramp":
                assert M.normwise_error(lg, ref["logit"][i][p]) <= FP32_TOL
                risky = np.abs(ref["logit"][i][p]) <= np.abs(lg - ref["logit"][i][p]).max()
                assert np.array_equal(m[~risky], ref["mask"][i][p][~risky])
                continue
            # vote counts: exact but for covering tiles whose logit is within the error of 0
            k = cfg["scales"][si]
            s = cfg["scale_strides"][si]
            Hk, Wk = O.level_size(slides[i].shape[0], k), O.level_size(slides[i].shape[1], k)
            ts = [(jy, jx) for (n, sj, jy, jx) in ref["tiles"] if n == i and sj == si]
            near = [(np.abs(ref["tile_logits"][(i, si, jy, jx)][c]) <= 2 * amax).astype(float) for (jy, jx) in ts]
            A, _ = O.vote(ts, near, Hk, Wk, T, s)
            V = ref["logit"][i][p]
            assert np.all(np.abs(lg - V) <= A), (i, p)
            sure = A == 0
            assert np.array_equal(m[sure], ref["mask"][i][p][sure]), (i, p)
            assert sure.mean() > 0.9


def test_tall_slide_integer_steps():
    """A slide taller than the largest launch extent in y at 40x and 20x:
    pyramid, tissue map and tile list stay bit exact."""
    H, W = 131200, 24
    rgb, _ = synth.strip_slide(44, H, W, fg_frac=0.3)
    cfg = O.make_config(base=4, levels=1, head_out=1, n_classes=1, scales=(0, 1), tile=16, stride=16,
                        fg_filter=True)
    plan = om.Plan(base=4, levels=1, head_out=1, n_classes=1, scales=(0, 1), tile=16, stride=16, fg_filter=True)
    ds = [torch.from_numpy(np.ascontiguousarray(rgb)).to(DEV)]
    flat = synth.he_normal_weights(45, 4, 1, 1, 2, 1)
    pairs = [(0, 0), (0, 1)]
    packed = plan.pack(torch.from_numpy(flat).to(DEV))
    masks, _, ws = plan.segment(ds, pairs, packed)
    torch.cuda.synchronize()
    Hk, Wk = O.level_size(H, 1), O.level_size(W, 1)
    ey, ex = O.grid_extent(Hk, 16, 16), O.grid_extent(Wk, 16, 16)
    pyr = _region(plan, ds, pairs, ws, om.REGION_PYRAMID, 1).view(np.uint16).reshape(ey, ex, 4)
    assert np.array_equal(pyr[..., :3], O.scale_sums(rgb, 1, ey, ex))
    fg = O.tissue_map(rgb, 1)
    assert np.array_equal(_region(plan, ds, pairs, ws, om.REGION_TISSUE).reshape(fg.shape).astype(bool), fg)
    ref_list = O.tile_list([(H, W)], cfg, [fg])
    cnt = int(_region(plan, ds, pairs, ws, om.REGION_TILE_COUNT).view(np.int32)[0])
    got = _region(plan, ds, pairs, ws, om.REGION_TILE_LIST).view(np.int32).reshape(-1, 4)[:cnt]
    assert [tuple(t) for t in got] == ref_list
    assert masks[0][0].shape == (H, W) and masks[0][1].shape == (Hk, Wk)


def _paper_like_case():
    """The paper's settings at a small size: 40x/10x/5x at strides 32/8/8
    (T/s = 2 and 8, as 512 at 256 and 64), vote thresholds 1/4/4, the Otsu
    tissue map (median 5, components of < 10 coarse pixels removed), masks
    gated by the tissue map."""
    a, _ = synth.strip_slide(71, 300, 517, fg_frac=0.25)
    cfg = O.make_config(base=8, levels=3, head_out=2, n_classes=3, scales=(0, 2, 3), tile=64, stride=32,
                        fg_filter=True, mask_and_fg=True, scale_strides=(32, 8, 8), merge="vote",
                        vote_thresholds=(1, 4, 4), tissue_method="otsu", median_kernel=5, min_tissue_area=10)
    flat = synth.he_normal_weights(72, 8, 3, 3, 3, 2, bias_std=0.05)
    pairs = [(0, 0), (2, 1), (1, 2)]
    return [a], cfg, flat, pairs


def _paper_plan(cfg, precision=om.FP32, graph=False):
    return om.Plan(base=cfg["base"], levels=cfg["levels"], head_out=cfg["head_out"], n_classes=cfg["n_classes"],
                   scales=cfg["scales"], tile=cfg["tile"], stride=cfg["stride"], fg_filter=True, mask_and_fg=True,
                   emit_logits=True, scale_strides=cfg["scale_strides"], merge=om.MERGE_VOTE,
                   vote_thresholds=cfg["vote_thresholds"], tissue_method=om.TISSUE_OTSU,
                   median_kernel=cfg["median_kernel"], min_tissue_area=cfg["min_tissue_area"], precision=precision,
                   batch_tiles=16, graph=graph)


def test_paper_settings_end_to_end():
    """Per-scale strides, Otsu tissue map, majority vote and tissue-gated masks together."""
    slides, cfg, flat, pairs = _paper_like_case()
    plan = _paper_plan(cfg)
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    masks, logits, ws = plan.segment(ds, pairs, plan.pack(torch.from_numpy(flat).to(DEV)))
    torch.cuda.synchronize()
    ref = O.segment(slides, flat, cfg, pairs, keep_tiles=True)
    fg, _, (t, comps, kept) = O.tissue_map_otsu(slides[0], 3, 5, 10)
    st = _region(plan, ds, pairs, ws, om.REGION_TISSUE_STATS).view(np.int32)
    assert list(st) == [t, comps, kept, 0]
    cnt = int(_region(plan, ds, pairs, ws, om.REGION_TILE_COUNT).view(np.int32)[0])
    got = _region(plan, ds, pairs, ws, om.REGION_TILE_LIST).view(np.int32).reshape(-1, 4)[:cnt]
    assert [tuple(x) for x in got] == ref["tiles"]
    err, amax = _tile_logit_error(plan, ds, pairs, ws, ref, cfg["tile"])
    assert err <= FP32_TOL, err
    for p, (c, si) in enumerate(pairs):
        k, s = cfg["scales"][si], cfg["scale_strides"][si]
        Hk, Wk = O.level_size(slides[0].shape[0], k), O.level_size(slides[0].shape[1], k)
        ts = [(jy, jx) for (n, sj, jy, jx) in ref["tiles"] if sj == si]
        near = [(np.abs(ref["tile_logits"][(0, si, jy, jx)][c]) <= 2 * amax).astype(float) for (jy, jx) in ts]
        A, _ = O.vote(ts, near, Hk, Wk, cfg["tile"], s)
        lg = logits[0][p].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(lg - ref["logit"][0][p]) <= A), p
        m = masks[0][p].cpu().numpy().astype(bool)
        sure = A == 0
        assert np.array_equal(m[sure], ref["mask"][0][p][sure]), p
        gate = O.fg_at_scale(fg, 3, k, Hk, Wk)
        assert not (m & ~gate).any()  # masks stay inside the tissue map


def test_paper_settings_graph_replay():
    """The captured work after the tile list (backbone, head, vote stitch)
    replays bit for bit, with eager work between replays."""
    slides, cfg, flat, pairs = _paper_like_case()
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    eager = _paper_plan(cfg, om.BF16)
    m_e, l_e, _ = eager.segment(ds, pairs, eager.pack(torch.from_numpy(flat).to(DEV)))
    plan = _paper_plan(cfg, om.BF16, graph=True)
    packed = plan.pack(torch.from_numpy(flat).to(DEV))
    ws = torch.empty(plan.workspace_bytes(ds, pairs), dtype=torch.uint8, device=DEV)
    outs = plan.alloc_outputs(ds, pairs)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs[0][0] + outs[1][0]:
            if t is not None:
                t.fill_(3)
        float(torch.ones(1000, device=DEV).sum())
        torch.cuda.synchronize()
        masks, logits, _ = plan.segment(ds, pairs, packed, workspace=ws, outputs=outs, stream=side)
        side.synchronize()
        for p in range(len(pairs)):
            assert torch.equal(masks[0][p], m_e[0][p]), (rep, p)
            assert torch.equal(logits[0][p], l_e[0][p]), (rep, p)

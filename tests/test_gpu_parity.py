"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Integer steps (pad colour, pyramid, tissue map, tile list) are compared bit
for bit.  Floating-point outputs are compared with a normwise relative
error: <= 1e-4 for the FP32 backbone; for BF16 <= max(2e-2, twice the error
of exact BF16 arithmetic), see test_tiny_instance_bf16.  Masks are compared
exactly except where the reference logit lies within the measured logit
error of the threshold, where either value is correct.
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
BF16_TOL = 2e-2


def _plan(ocfg, precision, batch_tiles=0, emit=True):
    return om.Plan(base=ocfg["base"], levels=ocfg["levels"], head_out=ocfg["head_out"],
                   n_classes=ocfg["n_classes"], scales=ocfg["scales"], tile=ocfg["tile"],
                   stride=ocfg["stride"], fg_filter=ocfg["fg_filter"],
                   fg_threshold=ocfg["fg_threshold"], mask_and_fg=ocfg["mask_and_fg"],
                   precision=precision, emit_logits=emit, batch_tiles=batch_tiles)


def _run(ocfg, slides, flat, pairs, precision, batch_tiles=0):
    plan = _plan(ocfg, precision, batch_tiles)
    dslides = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    packed = plan.pack(torch.from_numpy(flat).to(DEV))
    masks, logits, ws = plan.segment(dslides, pairs, packed)
    torch.cuda.synchronize()
    return plan, dslides, masks, logits, ws


def _region(plan, dslides, pairs, ws, region, index=0):
    off, nb = plan.region(dslides, pairs, region, index)
    return ws[off:off + nb].cpu().numpy()


def _compare_planes(gpu_mask, gpu_logit, ref_mask, ref_logit, tol, ref_N=None):
    lg = gpu_logit.cpu().numpy().astype(np.float64)
    m = gpu_mask.cpu().numpy().astype(bool)
    err = M.normwise_error(lg, ref_logit)
    assert err <= tol, err
    abs_err = np.abs(lg - ref_logit).max()
    risky = np.abs(ref_logit) <= abs_err
    assert np.array_equal(m[~risky], ref_mask[~risky])
    return err, M.dice(m, ref_mask), float(risky.mean())


# ------------------------------------------------------------------ stitch alone

@pytest.mark.parametrize("H,W,T,s,keep", [(300, 217, 64, 32, 0.7), (128, 128, 128, 64, 1.0),
                                          (97, 250, 32, 16, 0.5), (64, 64, 64, 64, 1.0),
                                          (200, 130, 64, 64, 0.8), (5, 3, 16, 8, 1.0),
                                          (150, 133, 32, 7, 0.8), (66, 70, 16, 6, 0.9),
                                          (36002, 22, 16, 12, 0.9)])
def test_stitch_tiles_matches_oracle(H, W, T, s, keep):
    """The last shape is tall enough that the four-pixel form takes bands of
    eight rows per workgroup, cut where the covering tiles change (every 12
    rows, offset by 16): pieces shorter than a band, a ragged last band and a
    ragged last column group."""
    rng = np.random.default_rng(H * 1000 + W)
    ny, nx = O.grid_count(H, T, s), O.grid_count(W, T, s)
    tiles = [(jy, jx) for jy in range(ny) for jx in range(nx) if rng.uniform() < keep]
    logits = rng.standard_normal((len(tiles), T, T)).astype(np.float32)
    yx = torch.tensor(np.array(tiles, np.int32).reshape(-1, 2), device=DEV)
    mask, lam = om.stitch_tiles(T, s, H, W, torch.from_numpy(logits).to(DEV), yx)
    torch.cuda.synchronize()
    ref, N, D = O.stitch(tiles, [l.astype(np.float64) for l in logits], H, W, T, s)
    g = lam.cpu().numpy().astype(np.float64)
    assert np.array_equal(g == 0, D == 0) or np.all(np.abs(g[D == 0]) == 0)
    cov = D > 0
    # compensated FP32 sum, one division: a few ulp of the largest term
    scale = np.abs(ref[cov]).max() if cov.any() else 1.0
    assert np.abs(g[cov] - ref[cov]).max() <= 1e-5 * max(scale, 1.0)
    risky = np.abs(N) <= 1e-5 * np.abs(N).max()
    assert np.array_equal(mask.cpu().numpy().astype(bool)[~risky], ((N > 0) & cov)[~risky])


def test_stitch_constant_and_cancellation():
    T, s, H, W = 64, 32, 160, 150
    ny, nx = O.grid_count(H, T, s), O.grid_count(W, T, s)
    tiles = [(jy, jx) for jy in range(ny) for jx in range(nx)]
    yx = torch.tensor(np.array(tiles, np.int32), device=DEV)
    const = torch.full((len(tiles), T, T), -3.25, device=DEV)
    mask, lam = om.stitch_tiles(T, s, H, W, const, yx)
    assert torch.all(lam == -3.25) and torch.all(mask == 0)
    # cancelling +-1e4 terms plus a small one: compensated FP32 tracks FP64
    rng = np.random.default_rng(3)
    big = np.where(rng.uniform(size=(len(tiles), T, T)) < 0.5, 1e4, -1e4).astype(np.float32)
    big += rng.uniform(-1e-3, 1e-3, size=big.shape).astype(np.float32)
    _, lam = om.stitch_tiles(T, s, H, W, torch.from_numpy(big).to(DEV), yx)
    ref, _, _ = O.stitch(tiles, [b.astype(np.float64) for b in big], H, W, T, s)
    err = np.abs(lam.cpu().numpy() - ref).max()
    assert err <= 2e-3, err


# ------------------------------------------------------------------ integer steps

def _prep_case():
    a, _ = synth.strip_slide(31, 300, 517, fg_frac=0.25)
    b, _ = synth.strip_slide(32, 129, 64, fg_frac=0.5)
    c, _ = synth.strip_slide(33, 640, 200, fg_frac=0.15)
    cfg = O.make_config(base=8, levels=3, head_out=2, n_classes=3, scales=(0, 1, 2, 3), tile=64,
                        stride=32, fg_filter=True, mask_and_fg=True)
    flat = synth.he_normal_weights(41, 8, 3, 3, 4, 2, bias_std=0.05)
    pairs = [(0, 0), (2, 1), (1, 2), (0, 3), (1, 0)]
    return [a, b, c], cfg, flat, pairs


def test_integer_steps_bit_exact():
    slides, cfg, flat, pairs = _prep_case()
    plan, ds, masks, logits, ws = _run(cfg, slides, flat, pairs, om.FP32)
    kc = max(cfg["scales"])
    T, s = cfg["tile"], cfg["stride"]
    for i, rgb in enumerate(slides):
        pad = _region(plan, ds, pairs, ws, om.REGION_PAD, i).view(np.int32)
        assert list(pad[:3]) == list(O.pad_colour(rgb)), i
        for si, k in enumerate(cfg["scales"]):
            if k == 0:
                continue
            Hk, Wk = O.level_size(rgb.shape[0], k), O.level_size(rgb.shape[1], k)
            ey, ex = O.grid_extent(Hk, T, s), O.grid_extent(Wk, T, s)
            got = _region(plan, ds, pairs, ws, om.REGION_PYRAMID, i * 4 + si).view(np.uint16)
            got = got.reshape(ey, ex, 4)
            assert np.array_equal(got[..., :3], O.scale_sums(rgb, k, ey, ex)), (i, k)
        fg = _region(plan, ds, pairs, ws, om.REGION_TISSUE, i)
        ref_fg = O.tissue_map(rgb, kc)
        assert np.array_equal(fg.reshape(ref_fg.shape).astype(bool), ref_fg), i
    fgs = [O.tissue_map(r, kc) for r in slides]
    ref_list = O.tile_list([r.shape[:2] for r in slides], cfg, fgs)
    cnt = int(_region(plan, ds, pairs, ws, om.REGION_TILE_COUNT).view(np.int32)[0])
    assert cnt == len(ref_list)
    assert 0 < cnt < sum(O.grid_count(O.level_size(r.shape[0], k), T, s) *
                         O.grid_count(O.level_size(r.shape[1], k), T, s)
                         for r in slides for k in cfg["scales"])
    got_list = _region(plan, ds, pairs, ws, om.REGION_TILE_LIST).view(np.int32).reshape(-1, 4)[:cnt]
    assert [tuple(t) for t in got_list] == ref_list
    for i, rgb in enumerate(slides):
        for si, k in enumerate(cfg["scales"]):
            idx = _region(plan, ds, pairs, ws, om.REGION_TILE_INDEX, i * 4 + si).view(np.int32)
            ny = O.grid_count(O.level_size(rgb.shape[0], k), T, s)
            nx = O.grid_count(O.level_size(rgb.shape[1], k), T, s)
            want = -np.ones(ny * nx, np.int32)
            for li, t in enumerate(ref_list):
                if t[0] == i and t[1] == si:
                    want[t[2] * nx + t[3]] = li
            assert np.array_equal(idx, want), (i, si)


def test_multiscale_multislide_end_to_end_fp32():
    slides, cfg, flat, pairs = _prep_case()
    plan, ds, masks, logits, ws = _run(cfg, slides, flat, pairs, om.FP32)
    ref = O.segment(slides, flat, cfg, pairs, keep_tiles=True)
    cnt = int(_region(plan, ds, pairs, ws, om.REGION_TILE_COUNT).view(np.int32)[0])
    T = cfg["tile"]
    tl = _region(plan, ds, pairs, ws, om.REGION_TILE_LOGITS).view(np.float32)
    # slots per scale: pairs are grouped by scale in request order
    slots = {}
    for (c, si) in pairs:
        slots.setdefault(si, []).append(c)
    max_slots = max(len(v) for v in slots.values())
    tl = tl[:len(ref["tiles"]) * max_slots * T * T].reshape(-1, max_slots, T, T)
    worst = 0.0
    for li, t in enumerate(ref["tiles"]):
        for j, c in enumerate(slots.get(t[1], [])):
            e = M.normwise_error(tl[li, j], ref["tile_logits"][t][c])
            worst = max(worst, e)
    assert cnt == len(ref["tiles"]) and worst <= FP32_TOL, worst
    for i in range(len(slides)):
        for p in range(len(pairs)):
            _compare_planes(masks[i][p], logits[i][p], ref["mask"][i][p], ref["logit"][i][p], FP32_TOL)


# ------------------------------------------------------------------ the tiny one-class instance

def _tiny():
    rgb, gt = synth.ellipse_slide(1)
    cfg = O.make_config(base=8, levels=3, head_out=1, n_classes=1, scales=(0,), tile=128, stride=64)
    flat = synth.he_normal_weights(11, 8, 3, 1, 1, 1)
    return [rgb], cfg, flat, [(0, 0)]


def test_tiny_instance_fp32():
    slides, cfg, flat, pairs = _tiny()
    plan, ds, masks, logits, ws = _run(cfg, slides, flat, pairs, om.FP32)
    ref = O.segment(slides, flat, cfg, pairs)
    cnt = int(_region(plan, ds, pairs, ws, om.REGION_TILE_COUNT).view(np.int32)[0])
    assert cnt == 9
    err, dice, risk = _compare_planes(masks[0][0], logits[0][0], ref["mask"][0][0], ref["logit"][0][0], FP32_TOL)
    print(f"fp32 logit_err={err:.3e} dice={dice:.5f} at_risk={risk:.5f}")


def test_tiny_instance_bf16():
    """BF16 backbone end to end.  Two exact-BF16 computations of this network
    that differ only in summation order already disagree by ~1e-2 (the
    network amplifies rounding strongly), so the end-to-end bound is relative
    to exact BF16 arithmetic: the oracle's bfloat16 emulation (same rounding
    points, FP64 elsewhere) sets it, and the error against FP64 must stay
    within twice the emulation's own error.  The kernels themselves are
    pinned layer by layer in test_gpu_conv.py."""
    slides, cfg, flat, pairs = _tiny()
    plan, ds, masks, logits, ws = _run(cfg, slides, flat, pairs, om.BF16)
    emu = O.segment(slides, flat, cfg, pairs, emulate="bf16")
    ref = O.segment(slides, flat, cfg, pairs)
    lg = logits[0][0].cpu().numpy().astype(np.float64)
    err_emu = M.normwise_error(lg, emu["logit"][0][0])
    emu_vs_ref = M.normwise_error(emu["logit"][0][0], ref["logit"][0][0])
    err, dice, risk = _compare_planes(masks[0][0], logits[0][0], ref["mask"][0][0], ref["logit"][0][0],
                                      max(BF16_TOL, 2.0 * emu_vs_ref))
    print(f"bf16 vs fp64 {err:.3e} (exact bf16 arithmetic: {emu_vs_ref:.3e}; gpu vs emulation {err_emu:.3e}) "
          f"dice={dice:.5f} at_risk={risk:.5f}")


@pytest.mark.parametrize("damp", [0.3, 0.5])
def test_bf16_damped_network_meets_target(damp):
    """The BF16 path where exact BF16 arithmetic can meet the 2e-2 target:
    the tiny instance with its weights scaled down (a contractive network,
    which shrinks rather than amplifies rounding).  Against FP64 the BF16
    logits must be within 2e-2 (normwise); against the oracle's BF16
    emulation (the same rounding points) within a quarter of BF16's own
    error; masks equal the FP64 masks off the at-risk pixels."""
    slides, cfg, flat, pairs = _tiny()
    flat = (flat * damp).astype(np.float32)
    plan, ds, masks, logits, ws = _run(cfg, slides, flat, pairs, om.BF16)
    emu = O.segment(slides, flat, cfg, pairs, emulate="bf16")
    ref = O.segment(slides, flat, cfg, pairs)
    lg = logits[0][0].cpu().numpy().astype(np.float64)
    err_emu = M.normwise_error(lg, emu["logit"][0][0])
    emu_vs_ref = M.normwise_error(emu["logit"][0][0], ref["logit"][0][0])
    err, dice, risk = _compare_planes(masks[0][0], logits[0][0], ref["mask"][0][0], ref["logit"][0][0], BF16_TOL)
    print(f"damped x{damp}: bf16 vs fp64 {err:.3e} (exact bf16 arithmetic {emu_vs_ref:.3e}; gpu vs emulation "
          f"{err_emu:.3e}) dice={dice:.5f} at_risk={risk:.5f}")
    assert err_emu <= 0.25 * emu_vs_ref, (err_emu, emu_vs_ref)


@pytest.mark.parametrize("base,tile", [(80, 48), (80, 64), (16, 48)])
def test_first_conv_launch_forms(base, tile):
    """The first conv in each of its launch forms, end to end at 40x and 20x
    (whose box-sum inputs exceed eight bits, so the BF16-MFMA form adds the
    inputs' upper parts): 16-row blocks (tile side not a multiple of 64) and
    64-row blocks, with more than four 16-channel fragments (C_0 = 80) and
    with one (C_0 = 16).  The weights are damped (x 0.3) so the network does
    not amplify rounding: the FP32 path must be within 1e-4 of FP64, and the
    BF16 path within a quarter of exact BF16 arithmetic's own error of the
    oracle's BF16 emulation (measured: under a tenth; a dropped or misplaced
    operand part would be off by far more)."""
    rgb, _ = synth.strip_slide(81, 80, 112, fg_frac=0.5)
    cfg = O.make_config(base=base, levels=2, head_out=2, n_classes=2, scales=(0, 1), tile=tile, stride=tile // 2)
    flat = (synth.he_normal_weights(82, base, 2, 2, 2, 2, bias_std=0.05) * 0.3).astype(np.float32)
    pairs = [(0, 0), (1, 0), (0, 1), (1, 1)]
    ref = O.segment([rgb], flat, cfg, pairs)
    emu = O.segment([rgb], flat, cfg, pairs, emulate="bf16")
    _, _, m32, l32, _ = _run(cfg, [rgb], flat, pairs, om.FP32)
    _, _, m16, l16, _ = _run(cfg, [rgb], flat, pairs, om.BF16)
    for p in range(len(pairs)):
        _compare_planes(m32[0][p], l32[0][p], ref["mask"][0][p], ref["logit"][0][p], FP32_TOL)
        lg = l16[0][p].cpu().numpy().astype(np.float64)
        err_emu = M.normwise_error(lg, emu["logit"][0][p])
        emu_vs_ref = M.normwise_error(emu["logit"][0][p], ref["logit"][0][p])
        print(f"base {base} tile {tile} pair {pairs[p]}: bf16 vs emulation {err_emu:.3e}, "
              f"emulation vs fp64 {emu_vs_ref:.3e}")
        assert err_emu <= 0.25 * emu_vs_ref, (pairs[p], err_emu, emu_vs_ref)
        _compare_planes(m16[0][p], l16[0][p], ref["mask"][0][p], ref["logit"][0][p],
                        max(BF16_TOL, 2.0 * emu_vs_ref))


def test_batching_and_determinism():
    """Several slides in one call equal per-slide calls, bit for bit, and a
    second run is bitwise identical (no atomics on the forward path)."""
    slides, cfg, flat, pairs = _prep_case()
    for prec in (om.FP32, om.BF16):
        _, _, m_all, l_all, _ = _run(cfg, slides, flat, pairs, prec, batch_tiles=7)
        _, _, m_again, l_again, _ = _run(cfg, slides, flat, pairs, prec, batch_tiles=7)
        for i, rgb in enumerate(slides):
            _, _, m1, l1, _ = _run(cfg, [rgb], flat, pairs, prec, batch_tiles=64)
            for p in range(len(pairs)):
                assert torch.equal(m_all[i][p], m1[0][p])
                assert torch.equal(l_all[i][p], l1[0][p])
                assert torch.equal(l_all[i][p], l_again[i][p])
                assert torch.equal(m_all[i][p], m_again[i][p])


# ------------------------------------------------------------------ the full-width network

def _wide_case(H=512, W=384):
    rgb, _ = synth.strip_slide(2, H, W, fg_frac=0.5)
    cfg = O.make_config(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 1, 2, 3), tile=256,
                        stride=128, fg_filter=True)
    flat = synth.he_normal_weights(12, 64, 5, 6, 4, 2)
    pairs = [(c, k) for k in range(4) for c in range(6)]
    return rgb, cfg, flat, pairs


@pytest.mark.parametrize("precision,tol", [(om.FP32, FP32_TOL), (om.BF16, BF16_TOL)])
def test_wide_network_sampled_tiles(precision, tol):
    """Base 64, 5 levels, 6 classes x 4 scales, 256 tiles at stride 128:
    tile logits of sampled tiles against the oracle."""
    rgb, cfg, flat, pairs = _wide_case()
    plan, ds, masks, logits, ws = _run(cfg, [rgb], flat, pairs, precision)
    fg = O.tissue_map(rgb, 3)
    ref_tiles = O.tile_list([rgb.shape[:2]], cfg, [fg])
    cnt = int(_region(plan, ds, pairs, ws, om.REGION_TILE_COUNT).view(np.int32)[0])
    assert cnt == len(ref_tiles)
    T = 256
    tl = _region(plan, ds, pairs, ws, om.REGION_TILE_LOGITS).view(np.float32).reshape(-1, 6, T, T)
    wts = O.unpack_weights(flat, cfg)
    rng = np.random.default_rng(5)
    picks = sorted(set([0, len(ref_tiles) - 1] + list(rng.choice(len(ref_tiles), 1))))
    wb = O.bf16_weights(wts)
    for li in picks:
        n, si, jy, jx = ref_tiles[li]
        x = O.tile_input(rgb, cfg["scales"][si], T, 128, jy, jx)
        ref = O.tile_logits(x, wts, cfg, si, list(range(6)))
        err = M.normwise_error(tl[li], ref)
        if precision == om.FP32:
            print(f"tile {ref_tiles[li]} err={err:.3e}")
            assert err <= tol, (li, err)
        else:
            emu = O.tile_logits(x, wb, cfg, si, list(range(6)), store=O.round_bf16)
            err_emu = M.normwise_error(tl[li], emu)
            emu_vs_ref = M.normwise_error(emu, ref)
            print(f"tile {ref_tiles[li]} bf16 vs fp64 {err:.3e} (exact bf16 arithmetic {emu_vs_ref:.3e}; "
                  f"gpu vs emulation {err_emu:.3e})")
            assert err <= max(tol, 2.0 * emu_vs_ref), (li, err)


def test_precls_fused_into_last_conv_equals_unfused():
    """BF16 with a 64-channel D_0: when the last decoder conv runs
    weight-stationary (configuration 10, enough pixel blocks) it also computes
    the head's precls and stores F instead of D_0; the head's own precls does
    the same arithmetic, so pinning that conv to another configuration (no
    fusion) must give the same tile logits and masks bit for bit."""
    rgb, cfg, flat, pairs = _wide_case()
    dslide = torch.from_numpy(np.ascontiguousarray(rgb)).to(DEV)
    outs, recs = [], []
    for dec_b0 in (10, 6):
        plan = _plan(cfg, om.BF16)
        plan.set_conv_tuning(3, 0, dec_b0)
        packed = plan.pack(torch.from_numpy(flat).to(DEV))
        plan.set_profiling(True)
        masks, logits, ws = plan.segment([dslide], pairs, packed)
        torch.cuda.synchronize()
        recs.append([r for r in plan.read_profile() if r["stage"] == "dec_b" and r["level"] == 0])
        tl = _region(plan, [dslide], pairs, ws, om.REGION_TILE_LOGITS)
        outs.append((tl, [m.cpu().numpy() for m in masks[0]]))
    assert np.array_equal(outs[0][0], outs[1][0])
    for a_, b_ in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a_, b_)
    # the fused launch stores 32 bytes of F per pixel instead of 128 of D_0
    assert sum(r["bytes"] for r in recs[0]) < sum(r["bytes"] for r in recs[1])


def test_graph_replay_matches_eager():
    """With OMNISEG_FLAG_GRAPH the work after the tile list is captured once
    and replayed; every replay must equal the eager result bit for bit."""
    slides, cfg, flat, pairs = _prep_case()
    for prec in (om.FP32, om.BF16):
        _, _, m_eager, l_eager, _ = _run(cfg, slides, flat, pairs, prec, batch_tiles=16)
        plan = om.Plan(base=cfg["base"], levels=cfg["levels"], head_out=cfg["head_out"],
                       n_classes=cfg["n_classes"], scales=cfg["scales"], tile=cfg["tile"], stride=cfg["stride"],
                       fg_filter=cfg["fg_filter"], mask_and_fg=cfg["mask_and_fg"], precision=prec,
                       emit_logits=True, batch_tiles=16, graph=True)
        ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
        packed = plan.pack(torch.from_numpy(flat).to(DEV))
        ws = torch.empty(plan.workspace_bytes(ds, pairs), dtype=torch.uint8, device=DEV)
        outs = plan.alloc_outputs(ds, pairs)
        side = torch.cuda.Stream()  # the null stream cannot be captured
        torch.cuda.synchronize()
        for rep in range(4):
            for row in outs[0] + outs[1]:
                for t in row:
                    if t is not None:
                        t.fill_(7)  # eager work between replays; replay must overwrite it
            float(torch.ones(1000, device=DEV).sum())
            torch.cuda.synchronize()
            masks, logits, _ = plan.segment(ds, pairs, packed, workspace=ws, outputs=outs, stream=side)
            side.synchronize()
            for i in range(len(slides)):
                for p in range(len(pairs)):
                    assert torch.equal(masks[i][p], m_eager[i][p]), (prec, rep, i, p)
                    assert torch.equal(logits[i][p], l_eager[i][p]), (prec, rep, i, p)


def test_profile_records_accumulate_until_read():
    """Profiled calls append to one record list; a read returns all of them
    (again on a repeated read) and the next profiled call starts a new list."""
    slides, cfg, flat, pairs = _prep_case()
    plan = _plan(cfg, om.FP32)
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    packed = plan.pack(torch.from_numpy(flat).to(DEV))
    ws = torch.empty(plan.workspace_bytes(ds, pairs), dtype=torch.uint8, device=DEV)
    outs = plan.alloc_outputs(ds, pairs)
    plan.set_profiling(True)
    plan.segment(ds, pairs, packed, workspace=ws, outputs=outs)
    one = plan.read_profile()
    assert one and plan.read_profile() == one
    key = lambda recs: [(r["stage"], r["level"], r["tiles"], r["config"]) for r in recs]
    plan.segment(ds, pairs, packed, workspace=ws, outputs=outs)
    plan.segment(ds, pairs, packed, workspace=ws, outputs=outs)
    two = plan.read_profile()
    assert key(two) == key(one) * 2 and all(r["ms"] > 0 for r in two)
    plan.set_profiling(False)
    plan.segment(ds, pairs, packed, workspace=ws, outputs=outs)  # unprofiled: the list stays
    assert plan.read_profile() == two
    torch.cuda.synchronize()

"""FP8 (E4M3) backbone on the GPU (through the C ABI).

Calibration: the FP32 path's per-channel activation maxima against the
oracle's (activation_amax), and the power-of-two scales derived from them
equal.  End to end: the FP8 result against the oracle's FP8 emulation (the
same scales and rounding points, FP64 elsewhere) and against exact FP64.

Two computations of one FP8 definition differ only where FP32 summation
order moves a value across an E4M3 rounding boundary.  In the He-normal
network such a flip grows until it is as large as FP8's own error (the
network is chaotic at this precision: exact FP8 arithmetic is already
~50 % from FP64), so there the bound is the BF16 one: within twice the
error of exact FP8 arithmetic.  The same weights scaled by 0.3 give a
network that damps perturbations; there the GPU must match the emulation
to a small fraction of FP8's error, which pins every scale, fold and
rounding point of the path (a value flips to a neighbouring code with
probability about (FP32 error) / (code spacing), so the flips' RMS effect
is a few percent of the rounding noise of FP8 itself; a scale taken from
the wrong tensor is off by powers of two and gives a ratio of order one).
The bound is a quarter of the emulation's error.  The kernels are pinned
code by code in test_gpu_conv.py.
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
KINDS = ((om.ACT_ENC_A, "enc{}.A", 0), (om.ACT_ENC_E, "enc{}.E", 0), (om.ACT_DEC_A, "dec{}.A", 1),
         (om.ACT_DEC_D, "dec{}.D", 1))


def _plan(cfg, precision, emit=True):
    return om.Plan(base=cfg["base"], levels=cfg["levels"], head_out=cfg["head_out"], n_classes=cfg["n_classes"],
                   scales=cfg["scales"], tile=cfg["tile"], stride=cfg["stride"], fg_filter=cfg["fg_filter"],
                   fg_threshold=cfg["fg_threshold"], mask_and_fg=cfg["mask_and_fg"], precision=precision,
                   emit_logits=emit)


def _table_to_dict(plan, table, cfg):
    L = cfg["levels"]
    C = O.channels(cfg)
    out = {}
    for kind, name, short in KINDS:
        for l in range(L - short):
            off = plan.activation_offset(kind, l)
            out[name.format(l)] = table[off:off + C[l]]
            pad = table[off + C[l]:off + -(-C[l] // 32) * 32]
            assert np.all(pad == 0), name.format(l)  # padded channels stay 0
    return out


def _gpu_fp8(cfg, slides, flat, pairs, n_tiles):
    """Calibrate on the FP32 path, pack FP8, segment; returns (amax dict, masks, logits)."""
    ds = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in slides]
    w = torch.from_numpy(flat).to(DEV)
    p32 = _plan(cfg, om.FP32, emit=False)
    ws = torch.empty(p32.workspace_bytes(ds, pairs), dtype=torch.uint8, device=DEV)
    amax = p32.calibrate_fp8(ds, pairs, p32.pack(w), ws, n_tiles=n_tiles)
    p8 = _plan(cfg, om.FP8)
    packed = p8.pack_fp8(w, amax)
    masks, logits, ws8 = p8.segment(ds, pairs, packed)
    torch.cuda.synchronize()
    return p8, ds, _table_to_dict(p8, amax.cpu().numpy().astype(np.float64), cfg), masks, logits, ws8


def _oracle_scales(cfg, slides, flat, n_tiles):
    wts = O.unpack_weights(flat, cfg)
    fgs = [O.tissue_map(r, max(cfg["scales"]), cfg["fg_threshold"]) if cfg["fg_filter"] else None for r in slides]
    tl = O.tile_list([r.shape[:2] for r in slides], cfg, fgs)[:n_tiles]
    xs = [O.tile_input(slides[n], cfg["scales"][si], cfg["tile"], cfg["stride"], jy, jx) for (n, si, jy, jx) in tl]
    amax = O.activation_amax(xs, wts, cfg)
    return wts, amax, {k: O.pow2_scale(v) for k, v in amax.items()}


def _check_calibration(gpu_amax, ref_amax):
    for k, ref in ref_amax.items():
        got = gpu_amax[k]
        # FP32 backbone vs FP64: per-channel maxima agree to FP32 accuracy
        assert np.all(np.abs(got - ref) <= 1e-5 * max(ref.max(), 1e-30)), k
        # and the scales derived from them are the same powers of two
        assert np.array_equal(O.pow2_scale(got), O.pow2_scale(ref)), k


def _tiny():
    rgb, _ = synth.ellipse_slide(1)
    cfg = O.make_config(base=8, levels=3, head_out=1, n_classes=1, scales=(0,), tile=128, stride=64)
    flat = synth.he_normal_weights(11, 8, 3, 1, 1, 1)
    return [rgb], cfg, flat, [(0, 0)]


def _compare(gpu_logit, emu_logit, ref_logit):
    err_emu = M.normwise_error(gpu_logit, emu_logit)
    emu_vs_ref = M.normwise_error(emu_logit, ref_logit)
    err = M.normwise_error(gpu_logit, ref_logit)
    return err, emu_vs_ref, err_emu


def test_fp8_tiny_instance():
    """The one-class 256x256 instance (He-normal weights): calibration on all
    9 tiles, then the FP8 path against FP64 within twice the error of exact
    FP8 arithmetic; a second run is bitwise identical."""
    slides, cfg, flat, pairs = _tiny()
    plan, ds, gpu_amax, masks, logits, _ = _gpu_fp8(cfg, slides, flat, pairs, n_tiles=64)
    _, ref_amax, S = _oracle_scales(cfg, slides, flat, 64)
    _check_calibration(gpu_amax, ref_amax)
    emu = O.segment(slides, flat, cfg, pairs, emulate="fp8", fp8_scales=S)
    ref = O.segment(slides, flat, cfg, pairs)
    lg = logits[0][0].cpu().numpy().astype(np.float64)
    err, emu_vs_ref, err_emu = _compare(lg, emu["logit"][0][0], ref["logit"][0][0])
    m = masks[0][0].cpu().numpy().astype(bool)
    print(f"fp8 vs fp64 {err:.3e} (exact fp8 arithmetic {emu_vs_ref:.3e}; gpu vs emulation {err_emu:.3e}); "
          f"dice vs fp64 {M.dice(m, ref['mask'][0][0]):.5f}, vs emulation {M.dice(m, emu['mask'][0][0]):.5f}")
    assert err <= 2.0 * emu_vs_ref
    _, _, _, masks2, logits2, _ = _gpu_fp8(cfg, slides, flat, pairs, n_tiles=64)
    assert torch.equal(logits[0][0], logits2[0][0]) and torch.equal(masks[0][0], masks2[0][0])


@pytest.mark.parametrize("n_tiles", [64, 3])
def test_fp8_damped_network_matches_emulation(n_tiles):
    """Weights scaled by 0.3: the GPU's FP8 logits and masks against the FP8
    emulation, to a small fraction of FP8's own error (scales calibrated on
    all tiles, and on the first 3 only so that later tiles saturate)."""
    slides, cfg, flat, pairs = _tiny()
    flat = (flat * 0.3).astype(np.float32)
    plan, ds, gpu_amax, masks, logits, _ = _gpu_fp8(cfg, slides, flat, pairs, n_tiles=n_tiles)
    _, ref_amax, S = _oracle_scales(cfg, slides, flat, n_tiles)
    _check_calibration(gpu_amax, ref_amax)
    emu = O.segment(slides, flat, cfg, pairs, emulate="fp8", fp8_scales=S)
    ref = O.segment(slides, flat, cfg, pairs)
    lg = logits[0][0].cpu().numpy().astype(np.float64)
    err, emu_vs_ref, err_emu = _compare(lg, emu["logit"][0][0], ref["logit"][0][0])
    m = masks[0][0].cpu().numpy().astype(bool)
    print(f"damped: fp8 vs fp64 {err:.3e} (exact fp8 arithmetic {emu_vs_ref:.3e}; gpu vs emulation "
          f"{err_emu:.3e}); mask disagreement vs emulation {M.disagreement(m, emu['mask'][0][0]):.2e}")
    assert err_emu <= 0.25 * emu_vs_ref, (err_emu, emu_vs_ref)
    risky = np.abs(emu["logit"][0][0]) <= np.abs(lg - emu["logit"][0][0]).max()
    assert np.array_equal(m[~risky], emu["mask"][0][0][~risky])


def test_fp8_wide_network_sampled_tiles():
    """Base 64, 5 levels, 6 classes x 4 scales, 256 tiles at stride 128
    (weights scaled by 0.3), scales calibrated on the first tile: tile
    logits of sampled tiles against the FP8 emulation."""
    rgb, _ = synth.strip_slide(2, 512, 384, fg_frac=0.5)
    cfg = O.make_config(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 1, 2, 3), tile=256, stride=128,
                        fg_filter=True)
    flat = (synth.he_normal_weights(12, 64, 5, 6, 4, 2) * 0.3).astype(np.float32)
    pairs = [(c, k) for k in range(4) for c in range(6)]
    plan, ds, gpu_amax, masks, logits, ws = _gpu_fp8(cfg, [rgb], flat, pairs, n_tiles=1)
    wts, ref_amax, S = _oracle_scales(cfg, [rgb], flat, 1)
    _check_calibration(gpu_amax, ref_amax)
    fg = O.tissue_map(rgb, 3)
    ref_tiles = O.tile_list([rgb.shape[:2]], cfg, [fg])
    T = 256
    off, nb = plan.region(ds, pairs, om.REGION_TILE_LOGITS)
    tl = ws[off:off + nb].cpu().numpy().view(np.float32).reshape(-1, 6, T, T)
    w8 = O.fp8_weights(wts, cfg, S)
    for li in (0, len(ref_tiles) - 1):
        n, si, jy, jx = ref_tiles[li]
        x = O.tile_input(rgb, cfg["scales"][si], T, 128, jy, jx)
        emu = O.tile_logits(x, w8, cfg, si, list(range(6)), act_scales=S)
        ref = O.tile_logits(x, wts, cfg, si, list(range(6)))
        err, emu_vs_ref, err_emu = _compare(tl[li], emu, ref)
        print(f"tile {ref_tiles[li]} fp8 vs fp64 {err:.3e} (exact fp8 arithmetic {emu_vs_ref:.3e}; "
              f"gpu vs emulation {err_emu:.3e})")
        assert err_emu <= 0.25 * emu_vs_ref, (li, err_emu, emu_vs_ref)

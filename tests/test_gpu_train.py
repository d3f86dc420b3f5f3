"""Training path on the GPU (through the C ABI): stitched batch logits, BCE
loss and the hand-written backward against the FP64 oracle's loss and
reverse pass (which the CPU tests pin to torch autograd and FP64 central
differences)."""

import numpy as np
import pytest
import torch

import synth
from oracle import omniseg_oracle as O
from paper_2305_14566_amd import metrics as M
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _fd_case():
    rgb, gt = synth.tiny_slide(4, 64, 64)
    cfg = O.make_config(base=4, levels=3, head_out=2, n_classes=6, scales=(0, 1), tile=32, stride=16)
    flat = synth.he_normal_weights(15, 4, 3, 6, 2, 2, bias_std=0.05)
    pairs = [(c, si) for si in range(2) for c in range(6)]
    batch = [(si, jy, jx) for (_, si, jy, jx) in O.tile_list([(64, 64)], cfg)]
    return rgb, gt, cfg, flat, pairs, batch


def _targets(gt, cfg, pairs):
    return synth.soft_targets(gt, cfg["scales"], pairs)


def _gpu_step(rgb, gt, cfg, flat, pairs, batch, precision):
    plan = om.Plan(base=cfg["base"], levels=cfg["levels"], head_out=cfg["head_out"], n_classes=cfg["n_classes"],
                   scales=cfg["scales"], tile=cfg["tile"], stride=cfg["stride"], precision=precision, training=True)
    slide = torch.from_numpy(rgb).to(DEV)
    w = torch.from_numpy(flat.astype(np.float32)).to(DEV).requires_grad_(True)
    logit, covered = om.OmniSegFn.apply(w, plan, slide, batch, pairs)
    y = torch.from_numpy(_targets(gt, cfg, pairs)).to(DEV)
    loss = om.BCELossFn.apply(logit, y, covered)
    loss.backward()
    torch.cuda.synchronize()
    return plan, slide, logit.detach(), covered, float(loss.detach()), w.grad.detach().cpu().numpy().astype(np.float64)


def test_train_fp32_matches_oracle():
    rgb, gt, cfg, flat, pairs, batch = _fd_case()
    plan, slide, logit, covered, loss, grad = _gpu_step(rgb, gt, cfg, flat, pairs, batch, om.FP32)
    ref_loss, ref_grad, ref_lam = O.train_loss(rgb, gt, flat.astype(np.float64), cfg, pairs, batch)
    offs = plan.plane_offsets(slide, pairs)
    lg = logit.cpu().numpy().astype(np.float64)
    cov = covered.cpu().numpy().astype(bool)
    for p, pr in enumerate(pairs):
        ref = ref_lam[pr].ravel()
        got = lg[offs[p]:offs[p + 1]]
        assert np.array_equal(cov[offs[p]:offs[p + 1]], np.ones_like(ref, bool))  # full batch covers all
        assert M.normwise_error(got, ref) <= 1e-4, pr
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss), (loss, ref_loss)
    err = M.normwise_error(grad, ref_grad)
    cos = float(grad @ ref_grad / np.linalg.norm(grad) / np.linalg.norm(ref_grad))
    print(f"fp32 loss {loss:.8f} oracle {ref_loss:.8f}; gradient normwise error {err:.3e}, cosine {cos:.9f}")
    assert err <= 1e-4, err


def test_train_partial_batch_and_coverage():
    """A batch that leaves pixels uncovered: coverage planes, zero logits
    there, and the loss over covered pixels only."""
    rgb, gt, cfg, flat, pairs, batch = _fd_case()
    batch = [batch[0], batch[4], batch[-1]]
    plan, slide, logit, covered, loss, grad = _gpu_step(rgb, gt, cfg, flat, pairs, batch, om.FP32)
    ref_loss, ref_grad, ref_lam = O.train_loss(rgb, gt, flat.astype(np.float64), cfg, pairs, batch)
    offs = plan.plane_offsets(slide, pairs)
    lg = logit.cpu().numpy()
    cv = covered.cpu().numpy().astype(bool)
    assert 0 < cv.mean() < 1
    assert np.all(lg[~cv] == 0)
    for p, pr in enumerate(pairs):
        assert M.normwise_error(lg[offs[p]:offs[p + 1]], ref_lam[pr].ravel()) <= 1e-4
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    assert M.normwise_error(grad, ref_grad) <= 1e-4


def test_gpu_gradient_directional_differences():
    """GPU loss differences along random directions agree with the GPU
    gradient (FP32 loss, so a loose bound; kinks make single directions
    unreliable, so most, not all, must agree)."""
    rgb, gt, cfg, flat, pairs, batch = _fd_case()
    plan, slide, _, _, loss, grad = _gpu_step(rgb, gt, cfg, flat, pairs, batch, om.FP32)
    y = torch.from_numpy(_targets(gt, cfg, pairs)).to(DEV)

    def gpu_loss(wv):
        w = torch.from_numpy(wv.astype(np.float32)).to(DEV)
        lg, cv = om.OmniSegFn.apply(w, plan, slide, batch, pairs)
        l, _ = om.bce_loss(lg, y, cv, with_grad=False)
        return float(l)

    rng = np.random.default_rng(7)
    ok = 0
    for _ in range(4):
        v = rng.standard_normal(flat.size)
        v /= np.linalg.norm(v)
        eps = 1e-2
        fd = (gpu_loss(flat + eps * v) - gpu_loss(flat - eps * v)) / (2 * eps)
        an = float(grad @ v)
        ok += abs(fd - an) <= 2e-2 * max(abs(an), 1e-3 * np.abs(grad).max())
    assert ok >= 3, ok


def test_backward_deterministic():
    rgb, gt, cfg, flat, pairs, batch = _fd_case()
    for prec in (om.FP32, om.BF16):
        _, _, l1, _, _, g1 = _gpu_step(rgb, gt, cfg, flat, pairs, batch, prec)
        _, _, l2, _, _, g2 = _gpu_step(rgb, gt, cfg, flat, pairs, batch, prec)
        assert torch.equal(l1, l2) and np.array_equal(g1, g2)


@pytest.mark.parametrize("precision", [om.FP32, om.BF16])
def test_train_wide_network(precision):
    """Base 64, 5 levels, 6 classes x 2 scales, 256 tiles at stride 128: a
    two-tile batch against the oracle's loss and gradient."""
    rgb, gt = synth.strip_slide(3, 512, 512, fg_frac=0.5)
    cfg = O.make_config(base=64, levels=5, head_out=2, n_classes=6, scales=(0, 1), tile=256, stride=128)
    flat = synth.he_normal_weights(13, 64, 5, 6, 2, 2)
    pairs = [(c, si) for si in range(2) for c in range(6)]
    batch = [(0, 1, 1), (1, 0, 0)]
    plan, slide, logit, covered, loss, grad = _gpu_step(rgb, gt, cfg, flat, pairs, batch, precision)
    ref_loss, ref_grad, ref_lam = O.train_loss(rgb, gt, flat.astype(np.float64), cfg, pairs, batch)
    err = M.normwise_error(grad, ref_grad)
    cos = float(grad @ ref_grad / np.linalg.norm(grad) / np.linalg.norm(ref_grad))
    print(f"precision {precision}: loss {loss:.6f} oracle {ref_loss:.6f}; grad normwise {err:.3e} cos {cos:.6f}")
    if precision == om.FP32:
        assert abs(loss - ref_loss) <= 1e-4 * abs(ref_loss)
        assert err <= 1e-3, err
    else:
        assert abs(loss - ref_loss) <= 5e-2 * abs(ref_loss)
        assert cos >= 0.98, cos

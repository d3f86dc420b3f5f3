"""Single-layer parity of the backbone's MFMA conv kernel (through the C ABI)
against the oracle's FP64 conv on identical inputs.

Every loader (plain, fused 2x2 max-pool, fused upsample + concat), every
epilogue (bias+ReLU, residual, data gradient, residual gradient with ReLU
mask), both spatial blocks (8x16, 8x8), both channel blocks (64, 32) and
both precisions.  For BF16 the inputs and weights are BF16 values and the
only differences left are FP32 accumulation and the final BF16 rounding, so
the bound is one BF16 ulp per element.
"""

import numpy as np
import pytest
import torch

from oracle import omniseg_oracle as O
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def p32(c):
    return -(-c // 32) * 32


def to_nhwc(arrs, dtype):
    """List of [C, H, W] float64 arrays -> [n, H, W, pad32(C)] device tensor."""
    C, H, W = arrs[0].shape
    out = np.zeros((len(arrs), H, W, p32(C)), np.float32)
    for i, a in enumerate(arrs):
        out[i, :, :, :C] = np.transpose(a, (1, 2, 0))
    t = torch.from_numpy(out).to(DEV)
    return t.to(torch.bfloat16) if dtype == om.BF16 else t


def from_nhwc(t, C):
    return [np.transpose(x, (2, 0, 1))[:C].astype(np.float64) for x in t.float().cpu().numpy()]


def q(x, prec):
    return O.round_bf16(x) if prec == om.BF16 else np.asarray(x, np.float32).astype(np.float64)


def check(got, ref, prec):
    got = np.stack(got)
    ref = np.stack(ref)
    scale = np.abs(ref).max() + 1e-30
    if prec == om.BF16:
        bound = 2.0 ** -8 * np.abs(ref) + 1e-6 * scale
    else:
        bound = 1e-5 * scale
    bad = np.abs(got - ref) > bound
    assert not bad.any(), (bad.sum(), np.abs(got - ref).max(), scale)


CASES = [(3, 16, 32, 40, 64), (2, 8, 24, 64, 96), (2, 16, 16, 8, 16), (1, 24, 40, 96, 64)]


@pytest.mark.parametrize("prec", [om.FP32, om.BF16])
@pytest.mark.parametrize("n,H,W,cin,cout", CASES)
@pytest.mark.parametrize("mode", ["relu", "res", "pool", "upcat", "dgrad", "dgrad_res"])
def test_conv_layer(prec, n, H, W, cin, cout, mode):
    rng = np.random.default_rng(hash((n, H, W, cin, cout, mode)) % 2 ** 32)
    if mode in ("res", "dgrad_res"):
        cin = cout
    Wt = q(rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin)), prec)
    b = rng.standard_normal(cout) * 0.1
    wdev = torch.from_numpy(Wt.astype(np.float32)).to(DEV)
    bdev = torch.from_numpy(b.astype(np.float32)).to(DEV)
    if mode == "relu" or mode == "res":
        X = [q(rng.standard_normal((cin, H, W)), prec) for _ in range(n)]
        m = om.CONV_RELU if mode == "relu" else om.CONV_RES_RELU
        y = om.conv3x3(prec, m, to_nhwc(X, prec), wdev, bdev)
        ref = [np.maximum(O.conv3x3(x, Wt, b) + (x if mode == "res" else 0), 0) for x in X]
        check(from_nhwc(y, cout), ref, prec)
    elif mode == "pool":
        X = [q(np.abs(rng.standard_normal((cin, 2 * H, 2 * W))), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_POOL_RELU, to_nhwc(X, prec), wdev, bdev)
        ref = [np.maximum(O.conv3x3(O.maxpool2(x), Wt, b), 0) for x in X]
        check(from_nhwc(y, cout), ref, prec)
    elif mode == "upcat":
        cu = max(1, (2 * cin) // 3)
        D = [q(rng.standard_normal((cu, H // 2, W // 2)), prec) for _ in range(n)]
        E = [q(rng.standard_normal((cin - cu, H, W)), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_UPCAT_RELU, to_nhwc(D, prec), wdev, bdev, x1=to_nhwc(E, prec), cu=cu)
        ref = [np.maximum(O.conv3x3(np.concatenate([O.up2(d), e]), Wt, b), 0) for d, e in zip(D, E)]
        check(from_nhwc(y, cout), ref, prec)
    elif mode == "dgrad":
        G = [q(rng.standard_normal((cout, H, W)), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_DGRAD, to_nhwc(G, prec), wdev)
        ref = [O.conv3x3_backward(np.zeros((cin, H, W)), Wt, g)[0] for g in G]
        check(from_nhwc(y, cin), ref, prec)
    else:
        G = [q(rng.standard_normal((cout, H, W)), prec) for _ in range(n)]
        A = [q(rng.standard_normal((cin, H, W)), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_DGRAD_RES_MASK, to_nhwc(G, prec), wdev, aux=to_nhwc(A, prec))
        ref = [(O.conv3x3_backward(np.zeros((cin, H, W)), Wt, g)[0] + g) * (a > 0) for g, a in zip(G, A)]
        check(from_nhwc(y, cin), ref, prec)


@pytest.mark.parametrize("prec", [om.FP32, om.BF16])
def test_conv_dgrad_concat_layout(prec):
    """Data gradient of the decoder's concat conv: the output follows the
    concat padding (upsampled part padded, then the skip part padded)."""
    rng = np.random.default_rng(3)
    n, H, W, cu, ce, cout = 2, 16, 16, 40, 24, 32
    cin = cu + ce
    Wt = q(rng.standard_normal((cout, cin, 3, 3)) * 0.1, prec)
    G = [q(rng.standard_normal((cout, H, W)), prec) for _ in range(n)]
    y = om.conv3x3(prec, om.CONV_DGRAD, to_nhwc(G, prec), torch.from_numpy(Wt.astype(np.float32)).to(DEV), cu=cu)
    assert y.shape[-1] == p32(cu) + p32(ce)
    yn = y.float().cpu().numpy()
    got = [np.concatenate([np.transpose(v[..., :cu], (2, 0, 1)), np.transpose(v[..., p32(cu):p32(cu) + ce], (2, 0, 1))])
           for v in yn]
    ref = [O.conv3x3_backward(np.zeros((cin, H, W)), Wt, g)[0] for g in G]
    check(got, ref, prec)
    assert np.all(yn[..., cu:p32(cu)] == 0) and np.all(yn[..., p32(cu) + ce:] == 0)


@pytest.mark.parametrize("prec", [om.FP32, om.BF16])
@pytest.mark.parametrize("config", list(range(om.N_CONV_CONFIGS)))
@pytest.mark.parametrize("mode", ["res", "pool", "upcat", "dgrad_res"])
def test_every_tile_configuration(prec, config, mode):
    """Each conv tile configuration the autotuner may pick, on a shape it fits."""
    by, bx, bn, wm, wn = om.conv_config(config)
    n, H, W = 2, 2 * by, 2 * bx
    cout = bn if bn > 32 else 32
    cin = cout if mode in ("res", "dgrad_res") else 48
    rng = np.random.default_rng(config * 17 + len(mode))
    Wt = q(rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin)), prec)
    b = rng.standard_normal(cout) * 0.1
    wdev = torch.from_numpy(Wt.astype(np.float32)).to(DEV)
    bdev = torch.from_numpy(b.astype(np.float32)).to(DEV)
    if mode == "res":
        X = [q(rng.standard_normal((cin, H, W)), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_RES_RELU, to_nhwc(X, prec), wdev, bdev, config=config)
        check(from_nhwc(y, cout), [np.maximum(O.conv3x3(x, Wt, b) + x, 0) for x in X], prec)
    elif mode == "pool":
        X = [q(np.abs(rng.standard_normal((cin, 2 * H, 2 * W))), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_POOL_RELU, to_nhwc(X, prec), wdev, bdev, config=config)
        check(from_nhwc(y, cout), [np.maximum(O.conv3x3(O.maxpool2(x), Wt, b), 0) for x in X], prec)
    elif mode == "upcat":
        cu = 32
        D = [q(rng.standard_normal((cu, H // 2, W // 2)), prec) for _ in range(n)]
        E = [q(rng.standard_normal((cin - cu, H, W)), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_UPCAT_RELU, to_nhwc(D, prec), wdev, bdev, x1=to_nhwc(E, prec), cu=cu,
                       config=config)
        check(from_nhwc(y, cout), [np.maximum(O.conv3x3(np.concatenate([O.up2(d), e]), Wt, b), 0)
                                   for d, e in zip(D, E)], prec)
    else:
        G = [q(rng.standard_normal((cout, H, W)), prec) for _ in range(n)]
        A = [q(rng.standard_normal((cin, H, W)), prec) for _ in range(n)]
        y = om.conv3x3(prec, om.CONV_DGRAD_RES_MASK, to_nhwc(G, prec), wdev, aux=to_nhwc(A, prec), config=config)
        check(from_nhwc(y, cin), [(O.conv3x3_backward(np.zeros((cin, H, W)), Wt, g)[0] + g) * (a > 0)
                                  for g, a in zip(G, A)], prec)

"""Weight gradients of single backbone convs (the backward's wgrad kernels,
FP32 MFMA and BF16 MFMA) against the FP64 oracle's conv3x3_backward on the
same inputs.  Products of BF16 values are exact in FP32 and the pixel sums
run in FP32, so both precisions must match FP64 to FP32 accumulation error:
the BF16 inputs are BF16 values, not roundings of the reference's."""

import numpy as np
import pytest
import torch

from oracle import omniseg_oracle as O
from paper_2305_14566_amd import metrics as M
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
P32 = lambda c: -(-c // 32) * 32


def _nhwc(x, dtype):
    """(n, C, H, W) float64 -> device NHWC with 32-padded channels."""
    n, C, H, W = x.shape
    out = np.zeros((n, H, W, P32(C)), np.float32)
    out[..., :C] = x.transpose(0, 2, 3, 1)
    return torch.from_numpy(out).to(DEV).to(dtype)


def _values(rng, shape, dtype, nonneg=False):
    v = rng.standard_normal(shape)
    if nonneg:
        v = np.maximum(v, 0.0)
    t = torch.from_numpy(v.astype(np.float32))
    if dtype == torch.bfloat16:
        t = t.to(torch.bfloat16).to(torch.float32)  # the values both sides use
    return t.numpy().astype(np.float64)


@pytest.mark.parametrize("precision", [om.FP32, om.BF16])
@pytest.mark.parametrize("mode,n,H,cin,cu,cout", [
    (om.CONV_RELU, 2, 32, 64, 64, 64),     # 16-pixel rows, 64-channel output blocks
    (om.CONV_RELU, 3, 16, 40, 40, 24),     # padded channels, 32-channel output blocks
    (om.CONV_RELU, 2, 8, 32, 32, 96),      # 8-pixel rows
    (om.CONV_POOL_RELU, 2, 16, 64, 64, 128),
    (om.CONV_POOL_RELU, 1, 8, 20, 20, 40),
    (om.CONV_UPCAT_RELU, 2, 32, 96, 64, 32),
    (om.CONV_UPCAT_RELU, 2, 16, 56, 40, 72),
])
def test_wgrad_matches_oracle(precision, mode, n, H, cin, cu, cout):
    print(f"wgrad precision={precision} mode={mode} n={n} H={H} cin={cin} cu={cu} cout={cout}", flush=True)
    dtype = torch.bfloat16 if precision == om.BF16 else torch.float32
    rng = np.random.default_rng(1000 * mode + H + cin + cout)
    W = H
    if mode == om.CONV_POOL_RELU:
        x0 = _values(rng, (n, cin, 2 * H, 2 * W), dtype, nonneg=True)
        xin = [O.maxpool2(x0[i]) for i in range(n)]
        x1 = None
    elif mode == om.CONV_UPCAT_RELU:
        x0 = _values(rng, (n, cu, H // 2, W // 2), dtype, nonneg=True)
        x1 = _values(rng, (n, cin - cu, H, W), dtype, nonneg=True)
        xin = [np.concatenate([O.up2(x0[i]), x1[i]]) for i in range(n)]
    else:
        x0 = _values(rng, (n, cin, H, W), dtype, nonneg=True)
        xin = [x0[i] for i in range(n)]
        x1 = None
    dy = _values(rng, (n, cout, H, W), dtype)
    ref = np.zeros((cout, cin, 3, 3))
    for i in range(n):
        _, dW, _ = O.conv3x3_backward(xin[i], np.zeros((cout, cin, 3, 3)), dy[i])
        ref += dW
    got = om.conv3x3_wgrad(precision, mode, _nhwc(x0, dtype), _nhwc(dy, dtype), cin, cout,
                           x1=_nhwc(x1, dtype) if x1 is not None else None, cu=cu)
    torch.cuda.synchronize()
    err = M.normwise_error(got.cpu().numpy().astype(np.float64), ref)
    print(f"  normwise error {err:.3e}")
    assert err <= 1e-5, err


def test_wgrad_deterministic():
    rng = np.random.default_rng(3)
    x0 = _nhwc(_values(rng, (4, 64, 32, 32), torch.bfloat16, True), torch.bfloat16)
    dy = _nhwc(_values(rng, (4, 64, 32, 32), torch.bfloat16), torch.bfloat16)
    a = om.conv3x3_wgrad(om.BF16, om.CONV_RELU, x0, dy, 64, 64)
    b = om.conv3x3_wgrad(om.BF16, om.CONV_RELU, x0, dy, 64, 64)
    torch.cuda.synchronize()
    assert torch.equal(a, b)

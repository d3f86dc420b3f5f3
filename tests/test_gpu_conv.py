"""Single-layer parity of the backbone's MFMA conv kernel (through the C ABI)
against the oracle's FP64 conv on identical inputs.

Every loader (plain, fused 2x2 max-pool, fused upsample + concat), every
epilogue (bias+ReLU, residual, data gradient, residual gradient with ReLU
mask), both spatial blocks (8x16, 8x8), both channel blocks (64, 32) and
both precisions.  For BF16 the inputs and weights are BF16 values and the
only differences left are FP32 accumulation and the final BF16 rounding, so
the bound is one BF16 ulp per element.
"""

import zlib

import numpy as np
import pytest
import torch

from oracle import omniseg_oracle as O
from paper_2305_14566_amd import omniseg as om

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def seed_of(*key):
    """A seed that is the same in every process (str hashes are not)."""
    return zlib.crc32(repr(key).encode())


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
    rng = np.random.default_rng(seed_of(n, H, W, cin, cout, mode))
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
    """Each conv tile configuration the autotuner may pick, on a shape it
    fits (two blocks per axis and per channel block), at every precision it
    declares; at any other precision the entry point must refuse it."""
    by, bx, bn, wm, wn, precs = om.conv_config_info(config)
    n, H, W = 2, 2 * by, 2 * bx
    if prec not in precs:
        x = torch.zeros((n, H, W, 32), dtype=torch.float32, device=DEV)
        w = torch.zeros((32, 32, 3, 3), dtype=torch.float32, device=DEV)
        with pytest.raises(om.OmnisegError):
            om.conv3x3(prec, om.CONV_RELU, x, w, torch.zeros(32, device=DEV), config=config)
        return
    cout = 2 * bn
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


@pytest.mark.parametrize("mode", ["relu", "res", "pool_out", "upcat", "pool_in", "dgrad", "dgrad_res"])
@pytest.mark.parametrize("size", ["small", "many_blocks"])
def test_large_block_form_equals_row_reuse_bit_for_bit(mode, size):
    """The double-buffered large-block form (32 rows x 16 pixels x 64
    channels, register epilogue) and its persistent launch sum the same taps
    of the same chunks in the same order as the eight-wave row-reuse form,
    so their outputs, and the fused pooled copy, equal that form's bit for
    bit: over 6 chunks, two channel blocks and several pixel blocks per tile.
    "many_blocks" gives the persistent form's 256 workgroups 2-3 blocks each
    (a number of blocks that the eight XCD ranges do not divide evenly), so
    the next block's first chunk is loaded during the last chunk and the
    epilogue of the current one."""
    big, ref_cfg, pers = 11, 10, 12
    assert om.conv_config_info(big)[:5] == (32, 16, 64, 4, 2) and om.conv_config_info(ref_cfg)[:5] == (16, 16, 64, 4, 2)
    assert om.conv_config_info(pers)[:5] == (32, 16, 64, 4, 2)
    rng = np.random.default_rng(seed_of("large-block", mode + size))
    n, H, W, C = (3, 64, 96, 128) if size == "small" else (13, 96, 128, 128)
    dev = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(DEV)
    Wt = q(rng.standard_normal((C, 192 if mode == "upcat" else C, 3, 3)) * np.sqrt(2.0 / (9 * C)), om.BF16)
    b = dev(rng.standard_normal(C) * 0.1)
    kw = {}
    if mode == "upcat":
        x0 = to_nhwc([q(rng.standard_normal((128, H // 2, W // 2)), om.BF16) for _ in range(n)], om.BF16)
        kw = dict(x1=to_nhwc([q(rng.standard_normal((64, H, W)), om.BF16) for _ in range(n)], om.BF16), cu=128)
        m = om.CONV_UPCAT_RELU
    elif mode == "pool_in":
        x0 = to_nhwc([q(np.abs(rng.standard_normal((C, 2 * H, 2 * W))), om.BF16) for _ in range(n)], om.BF16)
        m = om.CONV_POOL_RELU
    else:
        x0 = to_nhwc([q(rng.standard_normal((C, H, W)), om.BF16) for _ in range(n)], om.BF16)
        m = {"relu": om.CONV_RELU, "res": om.CONV_RES_RELU, "pool_out": om.CONV_RES_RELU,
             "dgrad": om.CONV_DGRAD, "dgrad_res": om.CONV_DGRAD_RES_MASK}[mode]
        if mode == "dgrad_res":
            kw = dict(aux=to_nhwc([q(rng.standard_normal((C, H, W)), om.BF16) for _ in range(n)], om.BF16))
    pool = mode == "pool_out"
    outs = []
    for cfg in (ref_cfg, big, pers, -1):  # -1: the library's default for the layer
        r = om.conv3x3(om.BF16, m, x0, dev(Wt), None if mode.startswith("dgrad") else b, config=cfg, pool=pool,
                       height=H, width=W, **kw)
        outs.append(r if pool else (r,))
    torch.cuda.synchronize()
    for other in outs[1:]:
        for a, c in zip(outs[0], other):
            assert torch.equal(a.view(torch.int16), c.view(torch.int16))
    assert outs[0][0].float().abs().sum() > 0


@pytest.mark.parametrize("case", ["res_pool", "relu_two_blocks", "relu_one_block", "dgrad_res_mask",
                                  "dgrad_three_blocks"])
def test_weight_stationary_form_equals_row_reuse_bit_for_bit(case):
    """Eight-wave launches with 64 input channels and at least 2048 pixel
    blocks run the persistent weight-stationary form (a workgroup per CU
    walking pixel blocks, weights kept in LDS, residual read from the staged
    halo), for forward and data-gradient epilogues and up to four 64-channel
    output blocks.  Its sums are the row-reuse forms' in the same order, so it
    equals the four-wave form (configuration 6) bit for bit, including the
    fused pooled copy."""
    rng = np.random.default_rng(seed_of("ws", case))
    n, H, W = (32, 128, 128) if case in ("relu_two_blocks", "dgrad_three_blocks") else (8, 256, 256)
    cin, cout = {"relu_two_blocks": (64, 128), "dgrad_three_blocks": (192, 64)}.get(case, (64, 64))
    dev = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(DEV)
    Wt = q(rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin)), om.BF16)
    b = dev(rng.standard_normal(cout) * 0.1)
    kw = {}
    if case.startswith("dgrad"):
        # the data gradient: input = the output gradient (cout = 64 channels)
        x = torch.from_numpy(rng.standard_normal((n, H, W, cout)).astype(np.float32)).to(torch.bfloat16).to(DEV)
        if case == "dgrad_res_mask":
            mode = om.CONV_DGRAD_RES_MASK
            kw = dict(aux=torch.from_numpy(rng.standard_normal((n, H, W, cin)).astype(np.float32)).to(torch.bfloat16).to(DEV))
        else:
            mode = om.CONV_DGRAD
            kw = dict(cu=128)
        b = None
    else:
        x = torch.from_numpy(rng.standard_normal((n, H, W, cin)).astype(np.float32)).to(torch.bfloat16).to(DEV)
        mode = om.CONV_RES_RELU if case == "res_pool" else om.CONV_RELU
    pool = case == "res_pool"
    outs = [om.conv3x3(om.BF16, mode, x, dev(Wt), b, config=c, pool=pool, height=H, width=W, **kw) for c in (10, 6)]
    torch.cuda.synchronize()
    outs = [o if isinstance(o, tuple) else (o,) for o in outs]
    for a_, c_ in zip(outs[0], outs[1]):
        assert torch.equal(a_.view(torch.int16), c_.view(torch.int16))
    assert outs[0][0].float().abs().sum() > 0


# ------------------------------------------------------------------ FP8 (E4M3)

def _e4m3_values():
    """Non-negative E4M3 values by code (bit-level decode), code 0x7F (NaN) excluded."""
    v = np.zeros(127)
    for code in range(127):
        e, m = code >> 3, code & 7
        v[code] = (m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
    return v


E4M3 = _e4m3_values()


def fp8_codes(X, scale):
    """[C, H, W] non-negative values -> (codes uint8 of E4M3(X / s), the values those codes stand for)."""
    q = O.round_e4m3(X / scale[:, None, None])
    codes = np.searchsorted(E4M3, q).astype(np.uint8)
    assert np.array_equal(E4M3[codes], q)
    return codes, q * scale[:, None, None]


def to_nhwc_u8(codes_list):
    C, H, W = codes_list[0].shape
    out = np.zeros((len(codes_list), H, W, p32(C)), np.uint8)
    for i, c in enumerate(codes_list):
        out[i, :, :, :C] = np.transpose(c, (1, 2, 0))
    return torch.from_numpy(out).to(DEV)


# The FP8 MFMA (32x32x64 f8f6f4) sums each group of 8 products aligned to
# the group's largest and drops bits below 2^-13 of it (an in-bounds probe of
# one large and many small products: 2^-12 of the largest is kept exactly,
# 2^-14 is lost), so one K = 64 step can lose up to 7 * 2^-13 of each group's
# largest product; FP32 accumulation across taps adds far less.
FP8_MFMA_REL = 7 * 2.0 ** -13 + 3e-5


def check_fp8(got_codes, Yref, Yabs, s_out):
    """GPU codes against the E4M3 encoding of the FP64 result Yref / s_out.
    The GPU's pre-rounding value may differ from Yref by the FP8 MFMA's
    accumulation error, bounded by FP8_MFMA_REL * Yabs (Yabs: the same conv
    on |inputs| and |weights|, the sum of the terms' magnitudes).  Each code
    must be the encoding of some value in [Yref - err, Yref + err];
    mismatches must be rare."""
    got = np.stack([np.transpose(g, (2, 0, 1))[:len(s_out)] for g in got_codes.cpu().numpy()]).astype(np.int64)
    sc = s_out[None, :, None, None]
    v = np.stack(Yref) / sc
    e = FP8_MFMA_REL * np.stack(Yabs) / sc
    code = lambda x: np.searchsorted(E4M3, O.round_e4m3(np.clip(x, 0.0, 448.0)))
    want, lo, hi = code(v), code(v - e), code(v + e)
    assert np.all((got >= lo) & (got <= hi)), np.argwhere((got < lo) | (got > hi))[:5]
    assert (got != want).mean() < 1e-2, (got != want).mean()
    assert np.all(np.transpose(got_codes.cpu().numpy(), (0, 3, 1, 2))[:, len(s_out):] == 0)  # padded channels


def pow2(rng, n, lo=-3, hi=3):
    return 2.0 ** rng.integers(lo, hi + 1, n).astype(np.float64)


def _fp8_case(rng, mode, n, H, W, cin, cout, cu=None):
    """Inputs (codes and the values they stand for), weights, the FP64
    reference and output scales calibrated on it (pow2_scale of each output
    channel's maximum, as the FP8 path derives them)."""
    Wt = (rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin))).astype(np.float32).astype(np.float64)
    b = (rng.standard_normal(cout) * 0.1).astype(np.float32).astype(np.float64)
    s_in = pow2(rng, cin)
    eff = O.fp8_conv_weights(Wt, s_in)[2]
    act = lambda shape, s: fp8_codes(np.abs(rng.standard_normal(shape)) * 50 * s[:, None, None], s)
    kw = {}
    if mode in ("relu", "res"):
        codes, X = zip(*[act((cin, H, W), s_in) for _ in range(n)])
        x0 = to_nhwc_u8(codes)
        Z = X
    elif mode == "pool":
        codes, X = zip(*[act((cin, 2 * H, 2 * W), s_in) for _ in range(n)])
        x0 = to_nhwc_u8(codes)
        Z = [O.maxpool2(x) for x in X]
    else:
        dc, D = zip(*[act((cu, H // 2, W // 2), s_in[:cu]) for _ in range(n)])
        ec, E = zip(*[act((cin - cu, H, W), s_in[cu:]) for _ in range(n)])
        x0 = to_nhwc_u8(dc)
        kw = dict(x1=to_nhwc_u8(ec), cu=cu)
        Z = [np.concatenate([O.up2(d), e]) for d, e in zip(D, E)]
    res = mode == "res"
    ref = [np.maximum(O.conv3x3(z, eff, b) + (z if res else 0), 0) for z in Z]
    mag = [O.conv3x3(z, np.abs(eff), np.abs(b)) + (z if res else 0) for z in Z]
    s_out = O.pow2_scale(np.stack(ref).max(axis=(0, 2, 3)))
    args = [torch.from_numpy(a.astype(np.float32)).to(DEV) for a in (Wt, b, s_in, s_out)]
    m = {"relu": om.CONV_RELU, "res": om.CONV_RES_RELU, "pool": om.CONV_POOL_RELU, "upcat": om.CONV_UPCAT_RELU}[mode]
    return m, x0, args, kw, ref, mag, s_out


FP8_CASES = [(2, 32, 48, 40, 64), (1, 16, 32, 64, 96), (2, 32, 16, 8, 32), (1, 16, 16, 200, 64)]


@pytest.mark.parametrize("n,H,W,cin,cout", FP8_CASES)
@pytest.mark.parametrize("mode", ["relu", "res", "pool", "upcat"])
def test_conv_layer_fp8(n, H, W, cin, cout, mode):
    """One FP8 conv: the oracle's effective weights (fp8_conv_weights) on the
    decoded input codes in FP64, encoded with the output scales, against the
    GPU's output codes."""
    rng = np.random.default_rng(seed_of(n, H, W, cin, cout, mode, "fp8"))
    if mode == "res":
        cin = cout
    m, x0, args, kw, ref, mag, s_out = _fp8_case(rng, mode, n, H, W, cin, cout, cu=max(1, (2 * cin) // 3))
    check_fp8(om.conv3x3_fp8(m, x0, *args, **kw), ref, mag, s_out)


@pytest.mark.parametrize("config", [c for c in range(om.N_CONV_CONFIGS) if om.FP8 in om.conv_config_info(c)[5]])
@pytest.mark.parametrize("mode", ["res", "pool", "upcat"])
def test_every_fp8_tile_configuration(config, mode):
    """Each FP8 tile configuration on a shape with two blocks per axis and
    per channel block."""
    by, bx, bn, wm, wn, _ = om.conv_config_info(config)
    n, H, W = 2, 2 * by, 2 * bx
    cout = 2 * bn
    cin = cout if mode == "res" else 96
    rng = np.random.default_rng(config * 31 + len(mode))
    m, x0, args, kw, ref, mag, s_out = _fp8_case(rng, mode, n, H, W, cin, cout, cu=64)
    check_fp8(om.conv3x3_fp8(m, x0, *args, config=config, **kw), ref, mag, s_out)


# ------------------------------------------------------------------ fused 2x2 max-pool output

@pytest.mark.parametrize("prec,config", [(p, c) for c in range(6, om.N_CONV_CONFIGS) for p in ("bf16", "fp8")
                                         if (om.BF16 if p == "bf16" else om.FP8) in om.conv_config_info(c)[5]])
def test_fused_pool_output(prec, config):
    """The residual conv's pooled copy (the encoder's next input, written by
    the same kernel) equals the 2x2 max of its stored output bit for bit, and
    the output itself matches the oracle."""
    by, bx, bn, wm, wn, _ = om.conv_config_info(config)
    n, H, W = 2, 2 * by, 2 * bx
    C = 2 * bn
    rng = np.random.default_rng(config * 7 + len(prec))
    if prec == "bf16":
        Wt = q(rng.standard_normal((C, C, 3, 3)) * np.sqrt(2.0 / (9 * C)), om.BF16)
        b = rng.standard_normal(C) * 0.1
        X = [q(rng.standard_normal((C, H, W)), om.BF16) for _ in range(n)]
        y, yp = om.conv3x3(om.BF16, om.CONV_RES_RELU, to_nhwc(X, om.BF16), torch.from_numpy(Wt.astype(np.float32)).to(DEV),
                           torch.from_numpy(b.astype(np.float32)).to(DEV), config=config, pool=True)
        check(from_nhwc(y, C), [np.maximum(O.conv3x3(x, Wt, b) + x, 0) for x in X], om.BF16)
        bits = y.view(torch.int16).float()  # non-negative BF16: bit patterns order like values
    else:
        m, x0, args, kw, ref, mag, s_out = _fp8_case(rng, "res", n, H, W, C, C)
        y, yp = om.conv3x3_fp8(m, x0, *args, config=config, pool=True, **kw)
        check_fp8(y, ref, mag, s_out)
        bits = y.float()
    want = torch.nn.functional.max_pool2d(bits.permute(0, 3, 1, 2), 2).permute(0, 2, 3, 1)
    got = yp.view(torch.int16).float() if prec == "bf16" else yp.float()
    assert torch.equal(got, want)

"""The exact BF16 operand splits behind the BF16-MFMA forms of the first conv
and the head's precls (CPU; no GPU).

Both kernels feed FP32 operands to v_mfma_f32_16x16x32_bf16 by splitting them
into BF16 pieces whose sum is the operand exactly, so each MFMA adds exact
products in FP32:
  * an FP32 weight w -> hi = bf16(w), mid = bf16(w - hi), lo = w - hi - mid
    (round to nearest even at each step; lo must itself be a BF16 value);
  * an integer input v < 2^14 (a colour, or a 2^k x 2^k box sum of colours
    for k <= 3) -> v & ~255 and v & 255, each exact in BF16;
  * a product of two BF16 values has at most 16 significant bits, so FP32
    holds it exactly.
These checks restate the bit-level rounding with numpy and test the three
properties exhaustively (inputs) or on a million random weights.
"""

import numpy as np
import pytest


def _bf16_rne_bits(f32):
    """Upper 16 bits of round-to-nearest-even of finite FP32 values to BF16."""
    u = f32.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFFFFFF
    return (u >> 16).astype(np.uint32)


def _bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32)


def _split3(w):
    hi = _bf16_rne_bits(w)
    r1 = (w - _bf16_value(hi)).astype(np.float32)
    mid = _bf16_rne_bits(r1)
    r2 = (r1 - _bf16_value(mid)).astype(np.float32)
    lo = _bf16_rne_bits(r2)
    return hi, mid, lo, r1, r2


def _weights():
    rng = np.random.default_rng(20230523)
    w = np.concatenate([
        rng.standard_normal(1_000_000) * np.sqrt(2.0 / 27.0),  # He-normal first conv
        rng.standard_normal(100_000) * 1e-3,
        rng.uniform(-4.0, 4.0, 100_000),
        [0.0, -0.0, 1.0, -1.0, 1.0 / 3.0, 2.0 ** -60, -(2.0 ** 40), np.pi],
    ])
    return w.astype(np.float32)


def test_three_term_weight_split_is_exact():
    w = _weights()
    hi, mid, lo, r1, r2 = _split3(w)
    # each subtraction is exact in FP32 and the last remainder is a BF16 value
    assert np.all(_bf16_value(lo) == r2)
    total = _bf16_value(hi).astype(np.float64) + _bf16_value(mid) + _bf16_value(lo)
    assert np.array_equal(total, w.astype(np.float64))


def test_two_bf16_terms_are_not_enough():
    # the third term matters: hi + mid alone misses FP32 weights in general
    w = _weights()
    hi, mid, _, _, _ = _split3(w)
    two = _bf16_value(hi).astype(np.float64) + _bf16_value(mid)
    assert np.mean(two != w.astype(np.float64)) > 0.5


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_integer_input_split_is_exact(k):
    vmax = 255 * 4 ** k  # largest box sum of 4^k colours
    v = np.arange(vmax + 1, dtype=np.uint32)
    lo = (v & np.uint32(255)).astype(np.float32)
    hi = (v & ~np.uint32(255)).astype(np.float32)
    for part in (lo, hi):
        assert np.all((part.view(np.uint32) & 0xFFFF) == 0)  # a BF16 value
    assert np.array_equal(lo.astype(np.int64) + hi.astype(np.int64), v.astype(np.int64))
    if k == 0:
        assert np.all(hi == 0)  # at 40x the upper part vanishes


def test_bf16_products_are_exact_in_fp32():
    rng = np.random.default_rng(7)
    a = _bf16_value(_bf16_rne_bits(rng.standard_normal(200_000).astype(np.float32)))
    b = _bf16_value(_bf16_rne_bits((rng.uniform(0, 16383, 200_000)).astype(np.float32)))
    exact = a.astype(np.float64) * b.astype(np.float64)
    assert np.array_equal((a * b).astype(np.float64), exact)

"""Seeded He-normal network weights in one canonical flat FP32 vector.

Canonical flat order (each tensor C-contiguous, weights before biases):
  1. encoder levels l = 0 .. L-1:  conv_a W (C_l, C_in, 3, 3), b (C_l),
                                   conv_b W (C_l, C_l, 3, 3),  b (C_l)
     with C_l = base * 2**l and C_in = 3 at l = 0, else C_{l-1};
  2. decoder levels l = L-2 .. 0:  conv_a W (C_l, 3 C_l, 3, 3), b (C_l),
                                   conv_b W (C_l, C_l, 3, 3),   b (C_l)
     (conv_a input channels: the 2 C_l upsampled channels first, then the
     C_l skip channels);
  3. precls, only when C_0 != 8:   W (8, C_0, 1, 1), b (8);
  4. controller:                   W_c (P, C_{L-1} + n_classes + n_scales),
                                   b_c (P),
     with P = 8*8 + 8*8 + o*8 + 8 + 8 + o for a head with o outputs.

Weights are drawn in FP64 as N(0, 2 / fan_in), fan_in = C_in * kh * kw
(C_{L-1} + n_classes + n_scales for the controller), then rounded once to
FP32.  Biases are zero unless bias_std > 0; they come from a second
generator so that the weight draws do not depend on it.
"""

import numpy as np


def head_param_count(head_out):
    o = int(head_out)
    return 8 * 8 + 8 * 8 + o * 8 + 8 + 8 + o


def weight_layout(base, levels, n_classes, n_scales, head_out):
    """List of (name, shape, fan_in) in canonical flat order."""
    C = [base * 2 ** l for l in range(levels)]
    out = []
    cin = 3
    for l in range(levels):
        out.append((f"enc{l}.a.w", (C[l], cin, 3, 3), cin * 9))
        out.append((f"enc{l}.a.b", (C[l],), None))
        out.append((f"enc{l}.b.w", (C[l], C[l], 3, 3), C[l] * 9))
        out.append((f"enc{l}.b.b", (C[l],), None))
        cin = C[l]
    for l in range(levels - 2, -1, -1):
        out.append((f"dec{l}.a.w", (C[l], 3 * C[l], 3, 3), 3 * C[l] * 9))
        out.append((f"dec{l}.a.b", (C[l],), None))
        out.append((f"dec{l}.b.w", (C[l], C[l], 3, 3), C[l] * 9))
        out.append((f"dec{l}.b.b", (C[l],), None))
    if C[0] != 8:
        out.append(("precls.w", (8, C[0], 1, 1), C[0]))
        out.append(("precls.b", (8,), None))
    P = head_param_count(head_out)
    G = C[levels - 1] + n_classes + n_scales
    out.append(("ctrl.w", (P, G), G))
    out.append(("ctrl.b", (P,), None))
    return out


def he_normal_weights(seed, base, levels, n_classes, n_scales, head_out, bias_std=0.0):
    """Canonical flat FP32 weight vector (numpy float32, 1-D)."""
    layout = weight_layout(base, levels, n_classes, n_scales, head_out)
    rng = np.random.default_rng(seed)
    brng = np.random.default_rng([seed, 1])
    parts = []
    for name, shape, fan_in in layout:
        n = int(np.prod(shape))
        if fan_in is not None:
            parts.append(rng.standard_normal(n) * np.sqrt(2.0 / fan_in))
        elif bias_std > 0:
            parts.append(brng.standard_normal(n) * bias_std)
        else:
            parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def training_init_weights(seed, base, levels, n_classes, n_scales, head_out):
    """Start point for training: the he_normal_weights draw with the second
    (residual) conv of every block set to zero, so each block starts as its
    first conv and activations keep their scale through the depth (the
    He-normal network's logits grow to ~1e5, where BCE gradients are
    useless).  Biases are zero."""
    flat = he_normal_weights(seed, base, levels, n_classes, n_scales, head_out).copy()
    off = 0
    for name, shape, _ in weight_layout(base, levels, n_classes, n_scales, head_out):
        n = int(np.prod(shape))
        if name.endswith(".b.w"):
            flat[off:off + n] = 0.0
        off += n
    return flat


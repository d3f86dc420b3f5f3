"""Plain FP64 CPU oracle of the slide-wise Omni-Seg hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the bench's CPU-baseline
leg do.  It shares no code with the HIP library: its own weight unpacking,
its own padding, resampling, convolution, head, controller and stitch.

Every step is written as its plain definition, in float64 (integers for the
integer steps), with numpy matmul as the only library primitive.  The
paper (arXiv 2305.14566) fixes the pipeline: pad the slide with a colour
taken from its top-left 2x2 corner (Section 2.1), keep only tissue regions
(Section 2.1), run the pre-trained dynamic multi-scale network on
overlapping tiles at several magnifications (Section 2.2), and merge the
overlapping tile predictions back into a per-tissue whole-slide mask
(Sections 2.2 and 2.3; constants in Section 3.2).  The paper does not
define the network, the merge weights, the resampling filter or the tissue
test.  The readings used here are: a residual U-Net with a
controller-generated 1x1 dynamic head, a linear-ramp weighted average of
overlapping tile logits, a box-sum pyramid and a fixed gray threshold on the
coarsest scale; each function states its reading where it is used.

Parity against the paper's own numbers is unpinned: the paper prints no
per-pixel values, masks or weights.  The tests pin every function here to
brute force, closed forms, invariants and independent library routines.
"""

import math

import numpy as np

# --------------------------------------------------------------------------
# configuration
# --------------------------------------------------------------------------


def make_config(base=8, levels=3, head_out=1, n_classes=1, scales=(0,), tile=128,
                stride=64, fg_filter=False, fg_threshold=220, mask_and_fg=False,
                scale_strides=None, merge="ramp", vote_thresholds=None, tissue_method="gray",
                median_kernel=1, min_tissue_area=0):
    """Oracle configuration.

    scales: log2 downsampling factor of each scale slot (0 = 40x, 1 = 20x,
    2 = 10x, 3 = 5x); the scale one-hot indexes this list.
    scale_strides: tile stride of each slot's grid (0 or None = stride);
    Section 3.2 uses 256 at 40x and 64 at 10x and 5x.
    merge: "ramp" (weighted mean of logits) or "vote" (majority vote of the
    binary tile predictions, Section 2.2) with vote_thresholds per slot.
    tissue_method: "gray" (fixed threshold fg_threshold) or "otsu" (with
    median_kernel and min_tissue_area; tissue_map_otsu).
    """
    n = len(scales)
    ss = tuple(int(v) if v else int(stride) for v in (scale_strides or (0,) * n))
    vt = tuple(int(v) for v in (vote_thresholds or (0,) * n))
    return dict(base=int(base), levels=int(levels), head_out=int(head_out),
                n_classes=int(n_classes), scales=tuple(int(s) for s in scales),
                tile=int(tile), stride=int(stride), fg_filter=bool(fg_filter),
                fg_threshold=int(fg_threshold), mask_and_fg=bool(mask_and_fg),
                scale_strides=ss, merge=str(merge), vote_thresholds=vt, tissue_method=str(tissue_method),
                median_kernel=int(median_kernel), min_tissue_area=int(min_tissue_area))


def stride_of(cfg, si):
    """Tile stride of scale slot si."""
    ss = cfg.get("scale_strides")
    return ss[si] if ss else cfg["stride"]


def channels(cfg):
    return [cfg["base"] * 2 ** l for l in range(cfg["levels"])]


def head_params(o):
    """Number of dynamic-head parameters: W1 8x8, W2 8x8, W3 ox8, b1, b2, b3."""
    return 8 * 8 + 8 * 8 + o * 8 + 8 + 8 + o


# --------------------------------------------------------------------------
# weights: the canonical flat order, unpacked independently of the generator
# --------------------------------------------------------------------------


def unpack_weights(flat, cfg):
    """Split the canonical flat vector into named float64 arrays.

    Order: encoder levels 0..L-1 (conv_a W, b, conv_b W, b), decoder levels
    L-2..0 (conv_a W, b, conv_b W, b), precls (only if C_0 != 8), controller
    W_c (P x (C_{L-1} + n_classes + n_scales)) and b_c.
    """
    flat = np.asarray(flat, dtype=np.float64)
    C = channels(cfg)
    L = cfg["levels"]
    pos = [0]
    out = {}

    def take(name, shape):
        n = int(np.prod(shape))
        out[name] = flat[pos[0]:pos[0] + n].reshape(shape)
        pos[0] += n

    cin = 3
    for l in range(L):
        take(f"enc{l}.a.w", (C[l], cin, 3, 3))
        take(f"enc{l}.a.b", (C[l],))
        take(f"enc{l}.b.w", (C[l], C[l], 3, 3))
        take(f"enc{l}.b.b", (C[l],))
        cin = C[l]
    for l in range(L - 2, -1, -1):
        take(f"dec{l}.a.w", (C[l], 3 * C[l], 3, 3))
        take(f"dec{l}.a.b", (C[l],))
        take(f"dec{l}.b.w", (C[l], C[l], 3, 3))
        take(f"dec{l}.b.b", (C[l],))
    if C[0] != 8:
        take("precls.w", (8, C[0], 1, 1))
        take("precls.b", (8,))
    P = head_params(cfg["head_out"])
    take("ctrl.w", (P, C[L - 1] + cfg["n_classes"] + len(cfg["scales"])))
    take("ctrl.b", (P,))
    if pos[0] != flat.size:
        raise ValueError(f"weight vector has {flat.size} values, layout needs {pos[0]}")
    return out


def weight_count(cfg):
    C = channels(cfg)
    L = cfg["levels"]
    n = 0
    cin = 3
    for l in range(L):
        n += C[l] * cin * 9 + C[l] + C[l] * C[l] * 9 + C[l]
        cin = C[l]
    for l in range(L - 1):
        n += C[l] * 3 * C[l] * 9 + C[l] + C[l] * C[l] * 9 + C[l]
    if C[0] != 8:
        n += 8 * C[0] + 8
    P = head_params(cfg["head_out"])
    n += P * (C[L - 1] + cfg["n_classes"] + len(cfg["scales"])) + P
    return n


# --------------------------------------------------------------------------
# O1  pad colour and padded slide (Section 2.1; Section 3.2)
# --------------------------------------------------------------------------


def pad_colour(rgb):
    """Per-channel mean of the top-left 2x2 pixels, rounded half up.

    The paper pads every slide with a colour taken as the mean of the 2x2
    block in its top-left corner (Section 2.1, repeated in Section 3.2).
    Reading: integer mean with round-half-up, floor((sum + 2) / 4).
    """
    rgb = np.asarray(rgb)
    if rgb.shape[0] < 2 or rgb.shape[1] < 2:
        raise ValueError("slide must be at least 2x2")
    s = rgb[:2, :2, :].astype(np.int64).sum(axis=(0, 1))
    return (s + 2) // 4


def padded_slide(rgb, ext_y, ext_x):
    """The slide extended to (ext_y, ext_x) with the pad colour (int64).

    Reading of the pad extent: the slide's (0, 0) stays the grid origin and
    the pad reaches right and down only as far as the tiles need.
    """
    H, W, _ = rgb.shape
    if ext_y < H or ext_x < W:
        raise ValueError("extent smaller than the slide")
    P = np.empty((ext_y, ext_x, 3), np.int64)
    P[:, :, :] = pad_colour(rgb)[None, None, :]
    P[:H, :W, :] = rgb
    return P


# --------------------------------------------------------------------------
# O2  multi-scale pyramid (Section 2.2: 40x, 10x, 5x from the 40x base)
# --------------------------------------------------------------------------


def level_size(n, k):
    """Pixels along one axis at scale k (factor 2**k): ceil(n / 2**k)."""
    f = 2 ** k
    return (n + f - 1) // f


def box_sum(P, f):
    """S(y, x, c) = sum over a, b < f of P(f y + a, f x + b, c)."""
    Hp, Wp, C = P.shape
    if Hp % f or Wp % f:
        raise ValueError("extent must be a multiple of the factor")
    return P.reshape(Hp // f, f, Wp // f, f, C).sum(axis=(1, 3))


def scale_sums(rgb, k, ext_y, ext_x):
    """Integer box sums S_k over [0, ext_y) x [0, ext_x) at scale k."""
    f = 2 ** k
    P = padded_slide(rgb, max(ext_y * f, rgb.shape[0]), max(ext_x * f, rgb.shape[1]))
    P = P[:ext_y * f, :ext_x * f]
    return box_sum(P, f)


# --------------------------------------------------------------------------
# O3  tissue map (Section 2.1 blank-region removal; reading: gray threshold)
# --------------------------------------------------------------------------


def tissue_map(rgb, kc, threshold=220):
    """Coarse foreground map at scale kc: 1000*gray < 1000*threshold.

    gray*1000 = 299 R + 587 G + 114 B of the box mean; in integers on the
    box sums: 299 S_R + 587 S_G + 114 S_B < threshold * 1000 * 4**kc.
    """
    H, W, _ = rgb.shape
    Hc, Wc = level_size(H, kc), level_size(W, kc)
    S = scale_sums(rgb, kc, Hc, Wc)
    g = 299 * S[..., 0] + 587 * S[..., 1] + 114 * S[..., 2]
    return g < threshold * 1000 * 4 ** kc


# --------------------------------------------------------------------------
# O3b  Otsu tissue detection (Section 2.1; Section 3.2: Otsu threshold,
#      median blur, small noise components dropped from the foreground)
# --------------------------------------------------------------------------


def gray8(rgb, kc):
    """Coarse gray map: round((299 S_R + 587 S_G + 114 S_B) / (1000 4^kc)), in [0, 255]."""
    H, W, _ = rgb.shape
    Hc, Wc = level_size(H, kc), level_size(W, kc)
    S = scale_sums(rgb, kc, Hc, Wc).astype(np.int64)
    den = 1000 * 4 ** kc
    return ((299 * S[..., 0] + 587 * S[..., 1] + 114 * S[..., 2] + den // 2) // den).astype(np.int64)


def median_blur(g, m):
    """m x m median (m odd) with replicated borders: the middle element of the
    sorted window."""
    if m == 1:
        return g.copy()
    r = m // 2
    P = np.pad(g, r, mode="edge")
    out = np.empty_like(g)
    for y in range(g.shape[0]):  # one output row at a time keeps the windows small
        win = np.lib.stride_tricks.sliding_window_view(P[y:y + m], (m, m))[0]
        out[y] = np.sort(win.reshape(g.shape[1], m * m), axis=-1)[:, (m * m - 1) // 2]
    return out


def otsu_threshold(g):
    """Otsu's threshold of an integer image in [0, 255].

    For each split {<= t} / {> t} with both classes non-empty the score is
    the between-class variance up to the constant 1/N^2, n0 n1 (mu0 - mu1)^2
    = (N s0 - n0 S)^2 / (n0 n1) with s0 the sum of the class {<= t} and S
    the sum of all pixels; scores are compared exactly (integers,
    cross-multiplied) and the first t of the largest score wins.  -1 when the
    image has a single value.
    """
    h = np.bincount(np.asarray(g).ravel(), minlength=256).astype(np.int64)
    N, S = int(h.sum()), int((h * np.arange(256)).sum())
    best_t, best_a2, best_d = -1, 0, 1
    n0 = s0 = 0
    for t in range(256):
        n0 += int(h[t])
        s0 += t * int(h[t])
        n1 = N - n0
        if n0 == 0 or n1 == 0:
            continue
        a2 = (N * s0 - n0 * S) ** 2
        d = n0 * n1
        if best_t < 0 or a2 * best_d > best_a2 * d:
            best_t, best_a2, best_d = t, a2, d
    return best_t


def components8(mask):
    """8-connected components by breadth-first flood fill.  Returns labels
    (-1 off the mask; each component labelled by its smallest row-major
    index) and the component sizes {label: pixels}."""
    H, W = mask.shape
    lab = -np.ones((H, W), dtype=np.int64)
    sizes = {}
    for y0 in range(H):
        for x0 in range(W):
            if not mask[y0, x0] or lab[y0, x0] >= 0:
                continue
            root = y0 * W + x0  # the first pixel met in row-major order is the smallest
            lab[y0, x0] = root
            queue, n = [(y0, x0)], 0
            while queue:
                y, x = queue.pop()
                n += 1
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < H and 0 <= xx < W and mask[yy, xx] and lab[yy, xx] < 0:
                            lab[yy, xx] = root
                            queue.append((yy, xx))
            sizes[root] = n
    return lab, sizes


def tissue_map_otsu(rgb, kc, median=1, min_area=0):
    """Tissue map by Otsu: gray -> median blur -> threshold t (tissue =
    blurred <= t, the darker class) -> drop 8-connected components below
    min_area pixels.  Returns (map, blurred gray, (t, components, kept))."""
    b = median_blur(gray8(rgb, kc), median)
    t = otsu_threshold(b)
    fg0 = b <= t
    lab, sizes = components8(fg0)
    keep = {r for r, n in sizes.items() if n >= min_area}
    fg = np.isin(lab, list(keep)) & fg0 if keep else np.zeros_like(fg0)
    return fg, b, (t, len(sizes), len(keep))


def tissue_of(rgb, cfg):
    """The tissue map a configuration asks for, at the coarsest scale."""
    kc = max(cfg["scales"])
    if cfg.get("tissue_method", "gray") == "otsu":
        return tissue_map_otsu(rgb, kc, cfg["median_kernel"], cfg["min_tissue_area"])[0]
    return tissue_map(rgb, kc, cfg["fg_threshold"])


# --------------------------------------------------------------------------
# O4  tile grid and foreground tile list (Section 2.2 overlap tiling)
# --------------------------------------------------------------------------


def grid_count(n_k, T, s):
    """Tiles along one axis: the origins 0, s, 2s, ... until the tiles cover n_k."""
    if n_k <= T:
        return 1
    return -(-(n_k - T) // s) + 1


def grid_extent(n_k, T, s):
    return (grid_count(n_k, T, s) - 1) * s + T


def tile_keeps(fg, kc, k, T, s, jy, jx):
    """Keep the tile iff a coarse foreground pixel overlaps its 40x footprint.

    Coarse row r covers 40x rows [r f_kc, (r+1) f_kc); the tile covers
    [jy s f_k, (jy s + T) f_k).  Same on columns.
    """
    fk, fc = 2 ** k, 2 ** kc
    r = np.arange(fg.shape[0])
    c = np.arange(fg.shape[1])
    rows = (r * fc < (jy * s + T) * fk) & ((r + 1) * fc > jy * s * fk)
    cols = (c * fc < (jx * s + T) * fk) & ((c + 1) * fc > jx * s * fk)
    return bool(fg[np.ix_(rows, cols)].any())


def tile_list(slides_hw, cfg, fg_maps=None):
    """Ordered list of kept tiles (slide, scale slot, jy, jx).

    Order: slide, scale slot ascending, tile row, tile column.
    """
    T = cfg["tile"]
    kc = max(cfg["scales"])
    out = []
    for n, (H, W) in enumerate(slides_hw):
        for si, k in enumerate(cfg["scales"]):
            s = stride_of(cfg, si)
            ny = grid_count(level_size(H, k), T, s)
            nx = grid_count(level_size(W, k), T, s)
            for jy in range(ny):
                for jx in range(nx):
                    if cfg["fg_filter"] and not tile_keeps(fg_maps[n], kc, k, T, s, jy, jx):
                        continue
                    out.append((n, si, jy, jx))
    return out


def tile_input(rgb, k, T, s, jy, jx):
    """The network input of one tile: x = S_k / (255 * 4**k), channels first."""
    H, W, _ = rgb.shape
    ey = grid_extent(level_size(H, k), T, s)
    ex = grid_extent(level_size(W, k), T, s)
    S = scale_sums(rgb, k, ey, ex)[jy * s:jy * s + T, jx * s:jx * s + T]
    return np.transpose(S, (2, 0, 1)).astype(np.float64) / (255.0 * 4 ** k)


# --------------------------------------------------------------------------
# O5-O6  residual U-Net backbone
# --------------------------------------------------------------------------


def conv3x3(X, Wt, b):
    """3x3 cross-correlation, stride 1, zero padding 1.

    Y[o, y, x] = b[o] + sum_{c, i, j} W[o, c, i, j] X[c, y + i - 1, x + j - 1]
    with X taken as 0 outside the tile.
    """
    Cin, H, W = X.shape
    Xp = np.zeros((Cin, H + 2, W + 2))
    Xp[:, 1:H + 1, 1:W + 1] = X
    Y = np.zeros((Wt.shape[0], H * W))
    for i in range(3):
        for j in range(3):
            # contiguous operands keep numpy on its BLAS path
            Wij = np.ascontiguousarray(Wt[:, :, i, j])
            Y += Wij @ Xp[:, i:i + H, j:j + W].reshape(Cin, H * W)
    return Y.reshape(-1, H, W) + b[:, None, None]


def relu(x):
    return np.maximum(x, 0.0)


def round_bf16(x):
    """Round to bfloat16 (1 sign, 8 exponent, 7 fraction bits), ties to even.

    bfloat16 keeps the upper 16 bits of an IEEE float32.  Values are first
    rounded to float32, then the low 16 bits are rounded away: add 0x7FFF
    plus the lowest kept bit and truncate.  Used only to emulate a path that
    stores activations and weights in bfloat16.
    """
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


E4M3_MAX = 448.0


def round_e4m3(x):
    """Round to the OCP FP8 E4M3 format (1 sign, 4 exponent bits with bias
    7, 3 fraction bits, subnormals below 2^-6, largest finite value 448),
    ties to even, after saturating magnitudes above 448 to 448.

    Inside a binade [2^e, 2^(e+1)) the representable values are spaced
    2^(e-3); below 2^-6 the spacing stays at 2^-9 (subnormals).  So the
    value is rounded to a multiple of 2^(max(e, -6) - 3).  Used only to
    emulate a path that stores activations and weights in FP8.
    """
    x = np.asarray(x, np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    _, ex = np.frexp(a)  # a = m 2^ex with m in [0.5, 1): binade exponent ex - 1
    e = np.maximum(ex - 1, -6)
    step = np.ldexp(1.0, e - 3)
    q = np.rint(a / step) * step  # rint: ties to even
    return np.where(x < 0, -q, q)


def pow2_scale(amax):
    """Power-of-two scale 2^ceil(log2(amax / 448)) that maps [0, amax] into
    the E4M3 range; 1 for amax = 0.  Powers of two keep every rescaling
    exact."""
    amax = np.asarray(amax, np.float64)
    out = np.ones_like(amax)
    pos = amax > 0
    r = amax[pos] / E4M3_MAX
    m, ex = np.frexp(r)  # r = m 2^ex, m in [0.5, 1): ceil(log2 r) = ex - 1 if m == 0.5 else ex
    out[pos] = np.ldexp(1.0, np.where(m == 0.5, ex - 1, ex))
    return out


def fp8_activation(X, scale):
    """An activation [C, H, W] as an FP8 path stores it: channel c as
    E4M3(X_c / s_c), read back as s_c E4M3(X_c / s_c)."""
    s = np.asarray(scale, np.float64)[:, None, None]
    return s * round_e4m3(X / s)


def fp8_conv_weights(Wt, s_in):
    """Weights of a 3x3 conv [Cout, Cin, 3, 3] as an FP8 path uses them.

    The input's channel scale s_in[c] folds into column c (W'[o, c] =
    W[o, c] s_in[c]); each output channel o then gets the power-of-two scale
    w_o = pow2_scale(max |W'[o]|) and W' is stored as E4M3(W'[o] / w_o).
    Returns the stored codes' values (q), the output scales w and the
    effective weights w_o q[o, c] / s_in[c] that act on the real-valued
    input, so that conv(fp8_activation(X), effective) is what the path
    computes (up to its FP32 accumulation)."""
    s_in = np.asarray(s_in, np.float64)
    Wf = Wt * s_in[None, :, None, None]
    w = pow2_scale(np.abs(Wf).reshape(Wf.shape[0], -1).max(axis=1))
    q = round_e4m3(Wf / w[:, None, None, None])
    eff = q * w[:, None, None, None] / s_in[None, :, None, None]
    return q, w, eff


def maxpool2(X):
    C, H, W = X.shape
    return X.reshape(C, H // 2, 2, W // 2, 2).max(axis=(2, 4))


def up2(X):
    """Nearest upsampling by 2: up2(D)(y, x) = D(y // 2, x // 2)."""
    return np.repeat(np.repeat(X, 2, axis=1), 2, axis=2)


def bf16_weights(wts):
    """Weights as a bfloat16 backbone stores them: every 3x3 conv except the
    first (3 -> C_0) in bfloat16; first conv, precls and controller in FP32."""
    out = dict(wts)
    for k, v in wts.items():
        if k.endswith(".w") and (k.startswith("enc") or k.startswith("dec")) and k != "enc0.a.w":
            out[k] = round_bf16(v)
    return out


def unet_forward(x, wts, cfg, keep=False, store=None, act_scales=None):
    """Residual U-Net on one tile.

    Encoder level l: A = ReLU(conv_a(X_l)); E_l = ReLU(conv_b(A) + A);
    X_{l+1} = maxpool2(E_l).  Decoder level l = L-2..0:
    Z = concat(up2(D_{l+1}), E_l); A = ReLU(conv_a(Z)); D_l = ReLU(conv_b(A) + A),
    with D_{L-1} = E_{L-1}.  Head input F = ReLU(W_p D_0 + b_p) if C_0 != 8,
    else D_0.  Returns (F, g) with g the pixel mean of E_{L-1}; with keep,
    also a dict of every intermediate for the reverse pass.  `store`, if
    given, rounds every conv output as a reduced-precision path stores it;
    `act_scales` (tensor name -> per-channel scale, names as in
    activation_names) instead stores each conv output as FP8 with its
    channel scales (fp8_activation).
    """
    L = cfg["levels"]
    C = channels(cfg)
    saved = {}

    def q(name, v):
        if act_scales is not None:
            return fp8_activation(v, act_scales[name])
        return store(v) if store is not None else v

    X = x
    E = []
    for l in range(L):
        if l > 0:
            X = maxpool2(E[l - 1])
        A = q(f"enc{l}.A", relu(conv3x3(X, wts[f"enc{l}.a.w"], wts[f"enc{l}.a.b"])))
        El = q(f"enc{l}.E", relu(conv3x3(A, wts[f"enc{l}.b.w"], wts[f"enc{l}.b.b"]) + A))
        if keep:
            saved[f"enc{l}.X"] = X
            saved[f"enc{l}.A"] = A
        E.append(El)
    D = E[L - 1]
    for l in range(L - 2, -1, -1):
        Z = np.concatenate([up2(D), E[l]], axis=0)
        A = q(f"dec{l}.A", relu(conv3x3(Z, wts[f"dec{l}.a.w"], wts[f"dec{l}.a.b"])))
        D = q(f"dec{l}.D", relu(conv3x3(A, wts[f"dec{l}.b.w"], wts[f"dec{l}.b.b"]) + A))
        if keep:
            saved[f"dec{l}.Z"] = Z
            saved[f"dec{l}.A"] = A
            saved[f"dec{l}.D"] = D
    if C[0] != 8:
        Wp = wts["precls.w"][:, :, 0, 0]
        pre = np.tensordot(Wp, D, axes=(1, 0)) + wts["precls.b"][:, None, None]
        F = relu(pre)
    else:
        F = D
    g = E[L - 1].mean(axis=(1, 2))
    if keep:
        saved["E"] = E
        saved["D0"] = D
        saved["F"] = F
        saved["g"] = g
        return F, g, saved
    return F, g


# --------------------------------------------------------------------------
# O7-O8  controller and dynamic head
# --------------------------------------------------------------------------


def controller_input(g, c, si, n_classes, n_scales):
    """[g; onehot_C(c); onehot_S(si)]."""
    v = np.zeros(g.size + n_classes + n_scales)
    v[:g.size] = g
    v[g.size + c] = 1.0
    v[g.size + n_classes + si] = 1.0
    return v


def controller(g, c, si, wts, cfg):
    """theta = W_c [g; onehot_C(c); onehot_S(si)] + b_c (P head parameters)."""
    v = controller_input(g, c, si, cfg["n_classes"], len(cfg["scales"]))
    return wts["ctrl.w"] @ v + wts["ctrl.b"]


def split_theta(theta, o):
    """theta -> W1 (8x8), W2 (8x8), W3 (o x 8), b1 (8), b2 (8), b3 (o)."""
    p = 0
    W1 = theta[p:p + 64].reshape(8, 8); p += 64
    W2 = theta[p:p + 64].reshape(8, 8); p += 64
    W3 = theta[p:p + 8 * o].reshape(o, 8); p += 8 * o
    b1 = theta[p:p + 8]; p += 8
    b2 = theta[p:p + 8]; p += 8
    b3 = theta[p:p + o]; p += o
    return W1, W2, W3, b1, b2, b3


def head(F, theta, o):
    """Dynamic head: three 1x1 convs whose weights are theta.

    h1 = ReLU(W1 F + b1); h2 = ReLU(W2 h1 + b2); z = W3 h2 + b3.
    Logit: z_0 for one output, z_1 - z_0 for two (the foreground
    probability of a two-way softmax is sigmoid(z_1 - z_0)).
    """
    W1, W2, W3, b1, b2, b3 = split_theta(theta, o)
    h1 = relu(np.tensordot(W1, F, axes=(1, 0)) + b1[:, None, None])
    h2 = relu(np.tensordot(W2, h1, axes=(1, 0)) + b2[:, None, None])
    z = np.tensordot(W3, h2, axes=(1, 0)) + b3[:, None, None]
    return z[0] if o == 1 else z[1] - z[0]


def tile_logits(x, wts, cfg, si, classes, store=None, act_scales=None):
    """Logits of one tile for the given classes (all at the tile's scale slot)."""
    F, g = unet_forward(x, wts, cfg, store=store, act_scales=act_scales)
    return np.stack([head(F, controller(g, c, si, wts, cfg), cfg["head_out"]) for c in classes])


# --------------------------------------------------------------------------
# FP8 form of the backbone: per-channel power-of-two scales
# --------------------------------------------------------------------------


def activation_names(cfg):
    """Names of the stored backbone activations: the output of every conv_a
    (enc{l}.A, dec{l}.A) and of every residual block (enc{l}.E, dec{l}.D)."""
    L = cfg["levels"]
    return ([f"enc{l}.A" for l in range(L)] + [f"enc{l}.E" for l in range(L)] +
            [f"dec{l}.A" for l in range(L - 1)] + [f"dec{l}.D" for l in range(L - 1)])


def conv_input_scale(name, cfg, act_scales):
    """Per-channel scale of the stored input of backbone conv `name`
    ("enc{l}.a", "enc{l}.b", "dec{l}.a", "dec{l}.b"); None for the first
    conv, which reads the RGB tile.  Max-pooling keeps the channel scales
    (a positive per-channel factor commutes with max); the decoder's concat
    input takes the upsampled tensor's scales, then the skip's."""
    L = cfg["levels"]
    part, l, ab = name[:3], int(name[3:-2]), name[-1]
    if part == "enc":
        if ab == "a":
            return None if l == 0 else act_scales[f"enc{l - 1}.E"]
        return act_scales[f"enc{l}.A"]
    if ab == "a":
        below = act_scales[f"enc{L - 1}.E"] if l + 1 == L - 1 else act_scales[f"dec{l + 1}.D"]
        return np.concatenate([below, act_scales[f"enc{l}.E"]])
    return act_scales[f"dec{l}.A"]


def fp8_weights(wts, cfg, act_scales):
    """Weights as the FP8 backbone uses them: every 3x3 conv except the
    first gets the effective weights of fp8_conv_weights for its input's
    channel scales; first conv, precls and controller stay as they are."""
    out = dict(wts)
    L = cfg["levels"]
    convs = [f"enc{l}.{ab}" for l in range(L) for ab in "ab"] + [f"dec{l}.{ab}" for l in range(L - 1) for ab in "ab"]
    for name in convs:
        s_in = conv_input_scale(name, cfg, act_scales)
        if s_in is not None:
            out[name + ".w"] = fp8_conv_weights(wts[name + ".w"], s_in)[2]
    return out


def fp8_calibrate(tiles_x, wts, cfg):
    """Per-channel activation scales from the exact forward pass over the
    given tile inputs: pow2_scale of each stored tensor's per-channel
    maximum (activations are ReLU outputs, so the maximum is the amax)."""
    return {k: pow2_scale(v) for k, v in activation_amax(tiles_x, wts, cfg).items()}


def activation_amax(tiles_x, wts, cfg):
    """Per-channel maximum of every stored backbone activation (names as in
    activation_names) over the exact forward passes of the given tiles."""
    L = cfg["levels"]
    amax = {}

    def take(name, V):
        m = V.reshape(V.shape[0], -1).max(axis=1)
        amax[name] = m if name not in amax else np.maximum(amax[name], m)

    for x in tiles_x:
        _, _, sv = unet_forward(x, wts, cfg, keep=True)
        for l in range(L):
            take(f"enc{l}.A", sv[f"enc{l}.A"])
            take(f"enc{l}.E", sv["E"][l])
        for l in range(L - 1):
            take(f"dec{l}.A", sv[f"dec{l}.A"])
            take(f"dec{l}.D", sv[f"dec{l}.D"])
    return amax


# --------------------------------------------------------------------------
# O10  overlap-weighted stitch (Sections 2.2-2.3; reading: linear ramp)
# --------------------------------------------------------------------------


def ramp(T):
    """r(i) = min(i + 1, T - i): positive, peaked in the tile centre."""
    i = np.arange(T)
    return np.minimum(i + 1, T - i).astype(np.float64)


def stitch(tiles, logits, H_k, W_k, T, s):
    """Weighted average of overlapping tile logits.

    tiles: list of (jy, jx) of the kept tiles; logits: matching list of TxT
    arrays.  N(p) = sum_t w_t(p) l_t(p - o_t), D(p) = sum_t w_t(p) with
    w(i, j) = r(i) r(j); Lambda = N / D where D > 0, else 0.
    Returns (Lambda, N, D) over [0, H_k) x [0, W_k).
    """
    ey, ex = grid_extent(H_k, T, s), grid_extent(W_k, T, s)
    N = np.zeros((ey, ex))
    D = np.zeros((ey, ex))
    w = np.outer(ramp(T), ramp(T))
    for (jy, jx), l in zip(tiles, logits):
        N[jy * s:jy * s + T, jx * s:jx * s + T] += w * l
        D[jy * s:jy * s + T, jx * s:jx * s + T] += w
    N, D = N[:H_k, :W_k], D[:H_k, :W_k]
    Lam = np.where(D > 0, N / np.where(D > 0, D, 1.0), 0.0)
    return Lam, N, D


# --------------------------------------------------------------------------
# O10b  majority vote (Section 2.2 overlap testing; thresholds in Section 3.2)
# --------------------------------------------------------------------------


def vote(tiles, logits, H_k, W_k, T, s):
    """Votes of overlapping binary tile predictions.

    Each kept tile predicts the class at a pixel where its logit is positive
    (probability above one half).  V(p) counts the covering tiles that
    predict the class, C(p) counts all covering tiles.  The mask of a slot
    with threshold v is V >= v.  Returns (V, C) over [0, H_k) x [0, W_k).
    """
    ey, ex = grid_extent(H_k, T, s), grid_extent(W_k, T, s)
    V = np.zeros((ey, ex), dtype=np.int64)
    C = np.zeros((ey, ex), dtype=np.int64)
    for (jy, jx), l in zip(tiles, logits):
        V[jy * s:jy * s + T, jx * s:jx * s + T] += (np.asarray(l) > 0)
        C[jy * s:jy * s + T, jx * s:jx * s + T] += 1
    return V[:H_k, :W_k], C[:H_k, :W_k]


def fg_at_scale(fg, kc, k, H_k, W_k):
    """Nearest lookup of the coarse map at scale k: fg(y >> (kc-k), x >> (kc-k))."""
    sh = kc - k
    ys = np.arange(H_k) >> sh
    xs = np.arange(W_k) >> sh
    return fg[np.ix_(ys, xs)]


# --------------------------------------------------------------------------
# O12  merge to the 40x base and colour mapping (Section 2.3; per-class
#      magnifications in Section 1)
# --------------------------------------------------------------------------


def upsample_nearest(mask_k, k, H, W):
    """40x mask from a scale-k mask: each value covers its 2^k x 2^k block."""
    f = 2 ** k
    return np.repeat(np.repeat(np.asarray(mask_k) != 0, f, axis=0), f, axis=1)[:H, :W]


def upsample_bilinear(lam_k, k, H, W):
    """Bilinear sample of a scale-k plane at the 40x pixel centres: source
    coordinate max(0, (y + 0.5) / 2^k - 0.5), the upper neighbour clamped to
    the plane; FP64."""
    f = 2.0 ** k
    L = np.asarray(lam_k, dtype=np.float64)
    Hk, Wk = L.shape

    def axis(n, nk):
        src = np.maximum(0.0, (np.arange(n) + 0.5) / f - 0.5)
        i0 = np.floor(src).astype(np.int64)
        i1 = np.minimum(i0 + 1, nk - 1)
        return i0, i1, src - i0

    y0, y1, ly = axis(H, Hk)
    x0, x1, lx = axis(W, Wk)
    ly, lx = ly[:, None], lx[None, :]
    top = (1 - lx) * L[np.ix_(y0, x0)] + lx * L[np.ix_(y0, x1)]
    bot = (1 - lx) * L[np.ix_(y1, x0)] + lx * L[np.ix_(y1, x1)]
    return (1 - ly) * top + ly * bot


def overlay(rgb, classes):
    """Colour mapping: for every class (mask at scale k, colour, alpha in
    [0, 256]) whose mask is on, in order: out = (out (256 - a) + c a + 128) >> 8."""
    H, W, _ = rgb.shape
    out = rgb.astype(np.int64)
    for (mask_k, k, col, a) in classes:
        on = upsample_nearest(mask_k, k, H, W)
        blended = (out * (256 - a) + np.asarray(col, np.int64) * a + 128) >> 8
        out = np.where(on[..., None], blended, out)
    return out.astype(np.uint8)


def map_10x(img):
    """The 10x map from the 40x one: the rounded (half up) mean of each 4 x 4
    block, over the block's pixels that lie inside the image."""
    H, W, C = img.shape
    Hb, Wb = -(-H // 4), -(-W // 4)
    out = np.zeros((Hb, Wb, C), np.uint8)
    for by in range(Hb):
        for bx in range(Wb):
            blk = img[4 * by:4 * by + 4, 4 * bx:4 * bx + 4].astype(np.int64).reshape(-1, C)
            n = blk.shape[0]
            out[by, bx] = (blk.sum(axis=0) + n // 2) // n
    return out


# --------------------------------------------------------------------------
# whole path
# --------------------------------------------------------------------------


def segment(slides, flat_weights, cfg, pairs, tile_subset=None, keep_tiles=False, emulate=None, fp8_scales=None):
    """Masks and stitched logits for every (slide, pair).

    slides: list of uint8 HWC arrays; pairs: list of (class, scale slot).
    Returns dict with 'mask'[n][p] (bool H_k x W_k), 'logit'[n][p] (float64),
    'tiles' (the kept tile list), 'pad' per slide, 'fg' per slide, and with
    keep_tiles the per-tile logits {(n, si, jy, jx): {class: TxT}}.  With
    merge "vote" the 'logit' planes hold the vote counts V.
    emulate="bf16" rounds weights and stored activations as a bfloat16
    backbone does (round_bf16); emulate="fp8" stores them as the FP8
    backbone does, with the channel scales `fp8_scales` (from
    fp8_calibrate); the default is exact FP64.
    """
    wts = unpack_weights(flat_weights, cfg)
    store = None
    act_scales = None
    if emulate == "bf16":
        wts = bf16_weights(wts)
        store = round_bf16
    elif emulate == "fp8":
        act_scales = fp8_scales
        wts = fp8_weights(wts, cfg, act_scales)
    T = cfg["tile"]
    kc = max(cfg["scales"])
    need_fg = cfg["fg_filter"] or cfg["mask_and_fg"]
    fgs = [tissue_of(r, cfg) if need_fg else None for r in slides]
    tl = tile_list([r.shape[:2] for r in slides], cfg, fgs)
    if tile_subset is not None:
        tl = [t for t in tl if t in set(tile_subset)]
    per_tile = {}
    for (n, si, jy, jx) in tl:
        classes = [c for (c, sj) in pairs if sj == si]
        if not classes:
            continue
        k = cfg["scales"][si]
        x = tile_input(slides[n], k, T, stride_of(cfg, si), jy, jx)
        lg = tile_logits(x, wts, cfg, si, classes, store=store, act_scales=act_scales)
        per_tile[(n, si, jy, jx)] = {c: lg[i] for i, c in enumerate(classes)}
    masks, logits = [], []
    for n, rgb in enumerate(slides):
        H, W, _ = rgb.shape
        mrow, lrow = [], []
        for (c, si) in pairs:
            k = cfg["scales"][si]
            Hk, Wk = level_size(H, k), level_size(W, k)
            ts = [(jy, jx) for (m, sj, jy, jx) in tl if m == n and sj == si]
            ls = [per_tile[(n, si, jy, jx)][c] for (jy, jx) in ts]
            if cfg.get("merge", "ramp") == "vote":
                V, _ = vote(ts, ls, Hk, Wk, T, stride_of(cfg, si))
                M = V >= cfg["vote_thresholds"][si]
                Lam = V.astype(np.float64)
            else:
                Lam, N, D = stitch(ts, ls, Hk, Wk, T, stride_of(cfg, si))
                M = (N > 0) & (D > 0)
            if cfg["mask_and_fg"]:
                M &= fg_at_scale(fgs[n], kc, k, Hk, Wk)
            mrow.append(M)
            lrow.append(Lam)
        masks.append(mrow)
        logits.append(lrow)
    out = dict(mask=masks, logit=logits, tiles=tl, pad=[pad_colour(r) for r in slides], fg=fgs)
    if keep_tiles:
        out["tile_logits"] = per_tile
    return out


# --------------------------------------------------------------------------
# O11  loss and hand-written reverse pass
# --------------------------------------------------------------------------


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def soft_target(gt_mask, k):
    """Box mean of the 40x ground-truth mask over each 2**k block (padded with 0)."""
    f = 2 ** k
    H, W = gt_mask.shape
    Hk, Wk = level_size(H, k), level_size(W, k)
    m = np.zeros((Hk * f, Wk * f))
    m[:H, :W] = gt_mask
    return m.reshape(Hk, f, Wk, f).mean(axis=(1, 3))


def bce_terms(Lam, y):
    """max(L, 0) - y L + log1p(exp(-|L|)), the BCE-with-logits term."""
    return np.maximum(Lam, 0.0) - y * Lam + np.log1p(np.exp(-np.abs(Lam)))


def conv3x3_backward(X, Wt, dY):
    """Gradients of conv3x3 w.r.t. its input, weight and bias."""
    Cin, H, W = X.shape
    Cout = Wt.shape[0]
    Xp = np.zeros((Cin, H + 2, W + 2))
    Xp[:, 1:H + 1, 1:W + 1] = X
    dXp = np.zeros_like(Xp)
    dY2 = dY.reshape(Cout, H * W)
    dW = np.zeros_like(Wt)
    for i in range(3):
        for j in range(3):
            sl = Xp[:, i:i + H, j:j + W].reshape(Cin, H * W)
            dW[:, :, i, j] = dY2 @ sl.T
            dXp[:, i:i + H, j:j + W] += (np.ascontiguousarray(Wt[:, :, i, j].T) @ dY2).reshape(Cin, H, W)
    return dXp[:, 1:H + 1, 1:W + 1], dW, dY2.sum(axis=1)


def maxpool2_backward(X, dY):
    """Route each gradient to the first maximum of its 2x2 window (row-major)."""
    C, H, W = X.shape
    win = X.reshape(C, H // 2, 2, W // 2, 2).transpose(0, 1, 3, 2, 4).reshape(C, H // 2, W // 2, 4)
    first = np.argmax(win, axis=-1)  # argmax returns the first maximum
    dwin = np.zeros_like(win)
    np.put_along_axis(dwin, first[..., None], dY[..., None], axis=-1)
    return dwin.reshape(C, H // 2, W // 2, 2, 2).transpose(0, 1, 3, 2, 4).reshape(C, H, W)


def up2_backward(dY):
    C, H, W = dY.shape
    return dY.reshape(C, H // 2, 2, W // 2, 2).sum(axis=(2, 4))


def head_backward(F, theta, o, dl):
    """Gradients of the head logit w.r.t. theta and F, given dL/dlogit (TxT)."""
    W1, W2, W3, b1, b2, b3 = split_theta(theta, o)
    h1 = relu(np.tensordot(W1, F, axes=(1, 0)) + b1[:, None, None])
    h2 = relu(np.tensordot(W2, h1, axes=(1, 0)) + b2[:, None, None])
    if o == 1:
        dz = dl[None]
    else:
        dz = np.stack([-dl, dl])
    dW3 = np.tensordot(dz, h2, axes=([1, 2], [1, 2]))
    db3 = dz.sum(axis=(1, 2))
    dh2 = np.tensordot(W3, dz, axes=(0, 0)) * (h2 > 0)
    dW2 = np.tensordot(dh2, h1, axes=([1, 2], [1, 2]))
    db2 = dh2.sum(axis=(1, 2))
    dh1 = np.tensordot(W2, dh2, axes=(0, 0)) * (h1 > 0)
    dW1 = np.tensordot(dh1, F, axes=([1, 2], [1, 2]))
    db1 = dh1.sum(axis=(1, 2))
    dF = np.tensordot(W1, dh1, axes=(0, 0))
    dtheta = np.concatenate([dW1.ravel(), dW2.ravel(), dW3.ravel(), db1, db2, db3])
    return dtheta, dF


def unet_backward(wts, cfg, saved, dF, dg):
    """Reverse pass of unet_forward; returns a dict of weight gradients."""
    L = cfg["levels"]
    C = channels(cfg)
    grads = {}
    E = saved["E"]
    if C[0] != 8:
        D0 = saved["D0"]
        F = saved["F"]
        dpre = dF * (F > 0)
        grads["precls.w"] = np.tensordot(dpre, D0, axes=([1, 2], [1, 2]))[:, :, None, None]
        grads["precls.b"] = dpre.sum(axis=(1, 2))
        dD = np.tensordot(wts["precls.w"][:, :, 0, 0], dpre, axes=(0, 0))
    else:
        dD = dF.copy()
    dE = [np.zeros_like(e) for e in E]
    hb, wb = E[L - 1].shape[1:]
    dE[L - 1] += dg[:, None, None] / (hb * wb)
    for l in range(0, L - 1):
        Dl = saved[f"dec{l}.D"]
        A = saved[f"dec{l}.A"]
        Z = saved[f"dec{l}.Z"]
        dpre_b = dD * (Dl > 0)
        dA, grads[f"dec{l}.b.w"], grads[f"dec{l}.b.b"] = conv3x3_backward(A, wts[f"dec{l}.b.w"], dpre_b)
        dA = dA + dpre_b
        dpre_a = dA * (A > 0)
        dZ, grads[f"dec{l}.a.w"], grads[f"dec{l}.a.b"] = conv3x3_backward(Z, wts[f"dec{l}.a.w"], dpre_a)
        nu = 2 * C[l]
        dE[l] += dZ[nu:]
        dD = up2_backward(dZ[:nu])
    dE[L - 1] += dD
    for l in range(L - 1, -1, -1):
        El = E[l]
        A = saved[f"enc{l}.A"]
        X = saved[f"enc{l}.X"]
        dpre_b = dE[l] * (El > 0)
        dA, grads[f"enc{l}.b.w"], grads[f"enc{l}.b.b"] = conv3x3_backward(A, wts[f"enc{l}.b.w"], dpre_b)
        dA = dA + dpre_b
        dpre_a = dA * (A > 0)
        dX, grads[f"enc{l}.a.w"], grads[f"enc{l}.a.b"] = conv3x3_backward(X, wts[f"enc{l}.a.w"], dpre_a)
        if l > 0:
            dE[l - 1] += maxpool2_backward(E[l - 1], dX)
    return grads


def pack_grads(grads, cfg):
    """Gradients in the canonical flat order (float64)."""
    C = channels(cfg)
    L = cfg["levels"]
    names = []
    for l in range(L):
        names += [f"enc{l}.a.w", f"enc{l}.a.b", f"enc{l}.b.w", f"enc{l}.b.b"]
    for l in range(L - 2, -1, -1):
        names += [f"dec{l}.a.w", f"dec{l}.a.b", f"dec{l}.b.w", f"dec{l}.b.b"]
    if C[0] != 8:
        names += ["precls.w", "precls.b"]
    names += ["ctrl.w", "ctrl.b"]
    return np.concatenate([np.asarray(grads[n]).ravel() for n in names])


def train_loss(rgb, gt, flat_weights, cfg, pairs, batch, with_grad=True):
    """BCE loss of the stitched logits over the pixels a tile batch covers.

    batch: list of (scale slot, jy, jx) tiles of one slide.  For each pair
    (c, si) the batch tiles at scale slot si are stitched; the loss is the
    mean of the BCE terms over every (pair, pixel) with D > 0 against the
    soft target (box mean of the 40x mask of class c).  Returns (loss, flat
    gradient in canonical order or None, dict of per-pair Lambda).
    """
    wts = unpack_weights(flat_weights, cfg)
    T, s = cfg["tile"], cfg["stride"]
    o = cfg["head_out"]
    H, W, _ = rgb.shape
    fwd = {}
    for (si, jy, jx) in batch:
        k = cfg["scales"][si]
        x = tile_input(rgb, k, T, s, jy, jx)
        F, g, saved = unet_forward(x, wts, cfg, keep=True)
        fwd[(si, jy, jx)] = (F, g, saved)
    terms = 0.0
    n_terms = 0
    stitched = {}
    for (c, si) in pairs:
        k = cfg["scales"][si]
        Hk, Wk = level_size(H, k), level_size(W, k)
        ts = [(jy, jx) for (sj, jy, jx) in batch if sj == si]
        ls = []
        for (jy, jx) in ts:
            F, g, _ = fwd[(si, jy, jx)]
            ls.append(head(F, controller(g, c, si, wts, cfg), o))
        Lam, N, D = stitch(ts, ls, Hk, Wk, T, s)
        y = soft_target(gt[c], k)
        cov = D > 0
        terms += bce_terms(Lam, y)[cov].sum()
        n_terms += int(cov.sum())
        stitched[(c, si)] = (Lam, D, y, cov, ts)
    loss = terms / n_terms
    if not with_grad:
        return loss, None, {p: v[0] for p, v in stitched.items()}
    w = np.outer(ramp(T), ramp(T))
    grads = {}
    dWc = np.zeros_like(wts["ctrl.w"])
    dbc = np.zeros_like(wts["ctrl.b"])
    dF_all = {key: np.zeros_like(v[0]) for key, v in fwd.items()}
    dg_all = {key: np.zeros_like(v[1]) for key, v in fwd.items()}
    G = channels(cfg)[-1]
    for (c, si), (Lam, D, y, cov, ts) in stitched.items():
        k = cfg["scales"][si]
        dLam = np.where(cov, (sigmoid(Lam) - y) / n_terms, 0.0)
        ey, ex = grid_extent(Lam.shape[0], T, s), grid_extent(Lam.shape[1], T, s)
        dL_ext = np.zeros((ey, ex))
        D_ext = np.ones((ey, ex))
        dL_ext[:Lam.shape[0], :Lam.shape[1]] = dLam
        D_ext[:Lam.shape[0], :Lam.shape[1]] = np.where(cov, D, 1.0)
        for (jy, jx) in ts:
            F, g, _ = fwd[(si, jy, jx)]
            sl = (slice(jy * s, jy * s + T), slice(jx * s, jx * s + T))
            dl = dL_ext[sl] * w / D_ext[sl]
            theta = controller(g, c, si, wts, cfg)
            dtheta, dF = head_backward(F, theta, o, dl)
            v = controller_input(g, c, si, cfg["n_classes"], len(cfg["scales"]))
            dWc += np.outer(dtheta, v)
            dbc += dtheta
            dg_all[(si, jy, jx)] += wts["ctrl.w"][:, :G].T @ dtheta
            dF_all[(si, jy, jx)] += dF
    for key, (F, g, saved) in fwd.items():
        gk = unet_backward(wts, cfg, saved, dF_all[key], dg_all[key])
        for name, v in gk.items():
            grads[name] = grads.get(name, 0.0) + v
    grads["ctrl.w"] = dWc
    grads["ctrl.b"] = dbc
    return loss, pack_grads(grads, cfg), {p: v[0] for p, v in stitched.items()}

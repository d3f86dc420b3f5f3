"""Seeded synthetic whole-slide images (uint8 RGB, HWC) with ground-truth masks.

Stand-ins for the kidney biopsy slides of the paper's data section (40x base,
six tissue classes, pale background, pink stain).  No dataset item is
reproduced: every slide is drawn from a seeded numpy generator.

Colour and noise model (shared by every generator here):
  * background level B ~ U{235..245} on all three channels;
  * shapes are rasterised at pixel centres, later shapes overwrite earlier ones;
  * Gaussian noise N(0, 4^2) per pixel and channel is added last, then the
    image is rounded, clipped to [0, 255] and cast to uint8.
"""

import numpy as np

# The paper's six annotated tissue types (data section), in a fixed order.
CLASS_NAMES = ("TUFT", "CAP", "PT", "DT", "PTC", "VES")
TUFT, CAP, PT, DT, PTC, VES = range(6)

_NOISE_SIGMA = 4.0
_NOISE_ROWS = 512  # rows of noise drawn per block (bounds host memory)


def _finish(canvas, rng):
    """Add N(0, 4^2) noise block by block, round, clip, cast to uint8 (in place)."""
    H, W, _ = canvas.shape
    for y0 in range(0, H, _NOISE_ROWS):
        y1 = min(H, y0 + _NOISE_ROWS)
        noise = rng.standard_normal((y1 - y0, W, 3), dtype=np.float32) * np.float32(_NOISE_SIGMA)
        blk = canvas[y0:y1].astype(np.float32) + noise
        np.rint(blk, out=blk)
        np.clip(blk, 0, 255, out=blk)
        canvas[y0:y1] = blk.astype(np.uint8)
    return canvas


def _bbox(cy, cx, r, H, W):
    y0 = max(0, int(np.floor(cy - r)))
    y1 = min(H, int(np.ceil(cy + r)) + 1)
    x0 = max(0, int(np.floor(cx - r)))
    x1 = min(W, int(np.ceil(cx + r)) + 1)
    return y0, y1, x0, x1


def _ellipse_mask(cy, cx, a, b, ang, y0, y1, x0, x1):
    yy = np.arange(y0, y1, dtype=np.float64)[:, None] + 0.5 - cy
    xx = np.arange(x0, x1, dtype=np.float64)[None, :] + 0.5 - cx
    ca, sa = np.cos(ang), np.sin(ang)
    u = xx * ca + yy * sa
    v = -xx * sa + yy * ca
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def _disc_dist(cy, cx, y0, y1, x0, x1):
    yy = np.arange(y0, y1, dtype=np.float64)[:, None] + 0.5 - cy
    xx = np.arange(x0, x1, dtype=np.float64)[None, :] + 0.5 - cx
    return np.sqrt(yy * yy + xx * xx)


def ellipse_slide(seed, H=256, W=256, n_ellipses=6):
    """White slide with pink ellipses: the tiny one-class instance.

    Returns (rgb uint8 [H, W, 3], gt bool [1, H, W]); class 0 is the union of
    the ellipses.  Semi-axes U(20, 40) px, angle U(0, pi), colour
    (200, 120, 170) + U{-15..15} per channel.
    """
    rng = np.random.default_rng(seed)
    bg = int(rng.integers(235, 246))
    canvas = np.full((H, W, 3), bg, np.uint8)
    gt = np.zeros((1, H, W), bool)
    for _ in range(n_ellipses):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        a, b = rng.uniform(20, 40, size=2)
        ang = rng.uniform(0, np.pi)
        col = np.array([200, 120, 170]) + rng.integers(-15, 16, size=3)
        r = max(a, b)
        y0, y1, x0, x1 = _bbox(cy, cx, r, H, W)
        if y1 <= y0 or x1 <= x0:
            continue
        m = _ellipse_mask(cy, cx, a, b, ang, y0, y1, x0, x1)
        canvas[y0:y1, x0:x1][m] = col
        gt[0, y0:y1, x0:x1][m] = True
    return _finish(canvas, rng), gt


def tiny_slide(seed, H=64, W=64):
    """Small white slide with a few pink discs (gradient-check instance).

    Returns (rgb, gt bool [6, H, W]); every class gets a seeded disc so each
    class has both positive and negative pixels.
    """
    rng = np.random.default_rng(seed)
    bg = int(rng.integers(235, 246))
    canvas = np.full((H, W, 3), bg, np.uint8)
    gt = np.zeros((6, H, W), bool)
    for c in range(6):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        r = rng.uniform(0.08, 0.2) * min(H, W)
        col = np.array([200, 120, 170]) + rng.integers(-30, 31, size=3)
        y0, y1, x0, x1 = _bbox(cy, cx, r, H, W)
        m = _disc_dist(cy, cx, y0, y1, x0, x1) <= r
        canvas[y0:y1, x0:x1][m] = col
        gt[c, y0:y1, x0:x1][m] = True
    return _finish(canvas, rng), gt


def strip_slide(seed, H, W, fg_frac=0.30, with_gt=True, density=1.0):
    """Needle-biopsy style slide: a sinusoidal tissue band on a pale background.

    Inside the band (half-width fg_frac*H/2 about the centreline
    y_c(x) = H/2 + A sin(2 pi x / period + phase), A = U(0.05, 0.15) H,
    period = U(0.5, 1.5) W) the tissue base colour (225, 165, 205) +- 10 is
    painted and then, in this order:
      * glomeruli: ellipses with semi-axes U(60, 200), colour (200, 120, 170)
        +- 15 (class CAP), each with a concentric 0.8x tuft (170, 80, 150)
        +- 15 (class TUFT, a subset of CAP); about 1 per 2 Mpx of band;
      * tubule rings: outer radius U(20, 50), wall U(4, 10), coin-split into
        PT (210, 130, 180) and DT (180, 130, 200); about 1 per 20 kpx;
      * capillary dots: radius U(4, 10), colour (150, 60, 120), class PTC;
        about 1 per 5 kpx;
      * vessel rings: radius U(40, 80), wall U(12, 20), colour
        (190, 70, 100), class VES; about 1 per 20 Mpx (at least one).
    `density` scales the shape counts.  Returns (rgb, gt bool [6, H, W] or None).
    """
    rng = np.random.default_rng(seed)
    bg = int(rng.integers(235, 246))
    canvas = np.full((H, W, 3), bg, np.uint8)
    gt = np.zeros((6, H, W), bool) if with_gt else None

    amp = rng.uniform(0.05, 0.15) * H
    period = rng.uniform(0.5, 1.5) * W
    phase = rng.uniform(0, 2 * np.pi)
    hw = fg_frac * H / 2.0
    base = np.array([225, 165, 205]) + rng.integers(-10, 11, size=3)
    xs = np.arange(W, dtype=np.float64) + 0.5
    yc = H / 2.0 + amp * np.sin(2 * np.pi * xs / period + phase)
    for y0 in range(0, H, 1024):
        y1 = min(H, y0 + 1024)
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] + 0.5
        band = np.abs(yy - yc[None, :]) <= hw
        canvas[y0:y1][band] = base

    band_area = float(2 * hw * W)

    def centre():
        x = rng.uniform(0, W)
        y = H / 2.0 + amp * np.sin(2 * np.pi * x / period + phase) + rng.uniform(-hw, hw)
        return y, x

    def paint(mask, y0, y1, x0, x1, col, cls):
        canvas[y0:y1, x0:x1][mask] = col
        if gt is not None:
            # a later shape replaces the labels of whatever it covers
            for c in range(6):
                if c != cls and not (cls == TUFT and c == CAP):
                    gt[c, y0:y1, x0:x1][mask] = False
            gt[cls, y0:y1, x0:x1][mask] = True

    n_glom = max(1, int(round(density * band_area / 2e6)))
    for _ in range(n_glom):
        cy, cx = centre()
        a, b = rng.uniform(60, 200, size=2)
        ang = rng.uniform(0, np.pi)
        col_cap = np.array([200, 120, 170]) + rng.integers(-15, 16, size=3)
        col_tuft = np.array([170, 80, 150]) + rng.integers(-15, 16, size=3)
        y0, y1, x0, x1 = _bbox(cy, cx, max(a, b), H, W)
        if y1 <= y0 or x1 <= x0:
            continue
        m = _ellipse_mask(cy, cx, a, b, ang, y0, y1, x0, x1)
        paint(m, y0, y1, x0, x1, col_cap, CAP)
        m2 = _ellipse_mask(cy, cx, 0.8 * a, 0.8 * b, ang, y0, y1, x0, x1)
        paint(m2, y0, y1, x0, x1, col_tuft, TUFT)

    n_tub = int(round(density * band_area / 2e4))
    for _ in range(n_tub):
        cy, cx = centre()
        r = rng.uniform(20, 50)
        wall = rng.uniform(4, 10)
        is_pt = rng.uniform() < 0.5
        col = np.array([210, 130, 180]) if is_pt else np.array([180, 130, 200])
        y0, y1, x0, x1 = _bbox(cy, cx, r, H, W)
        if y1 <= y0 or x1 <= x0:
            continue
        d = _disc_dist(cy, cx, y0, y1, x0, x1)
        paint((d <= r) & (d >= r - wall), y0, y1, x0, x1, col, PT if is_pt else DT)

    n_cap = int(round(density * band_area / 5e3))
    for _ in range(n_cap):
        cy, cx = centre()
        r = rng.uniform(4, 10)
        y0, y1, x0, x1 = _bbox(cy, cx, r, H, W)
        if y1 <= y0 or x1 <= x0:
            continue
        d = _disc_dist(cy, cx, y0, y1, x0, x1)
        paint(d <= r, y0, y1, x0, x1, np.array([150, 60, 120]), PTC)

    n_ves = max(1, int(round(density * band_area / 2e7)))
    for _ in range(n_ves):
        cy, cx = centre()
        r = rng.uniform(40, 80)
        wall = rng.uniform(12, 20)
        y0, y1, x0, x1 = _bbox(cy, cx, r, H, W)
        if y1 <= y0 or x1 <= x0:
            continue
        d = _disc_dist(cy, cx, y0, y1, x0, x1)
        paint((d <= r) & (d >= r - wall), y0, y1, x0, x1, np.array([190, 70, 100]), VES)

    return _finish(canvas, rng), gt


def strip_crop_origin(seed, H, W, size, align=128):
    """Top-left corner of a size x size window of strip_slide(seed, H, W)
    centred on the tissue band at the slide's middle column, rounded to a
    multiple of `align` and kept inside the slide.  Repeats the generator's
    first draws (background level, band amplitude, period, phase)."""
    rng = np.random.default_rng(seed)
    rng.integers(235, 246)
    amp = rng.uniform(0.05, 0.15) * H
    period = rng.uniform(0.5, 1.5) * W
    phase = rng.uniform(0, 2 * np.pi)
    xc = W / 2.0
    yc = H / 2.0 + amp * np.sin(2 * np.pi * xc / period + phase)
    y0 = int(round((yc - size / 2.0) / align)) * align
    x0 = int(round((xc - size / 2.0) / align)) * align
    return min(max(0, y0), H - size), min(max(0, x0), W - size)


def batch_slide_specs(seed=99, n=16, h_range=(2000, 8000), w_range=(4000, 40000),
                      fg_range=(0.10, 0.60)):
    """Sizes and foreground fractions of an uneven multi-slide batch.

    Returns a list of dicts {seed, H, W, fg_frac}; slide i uses seed 100 + i.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        H = int(rng.integers(h_range[0], h_range[1] + 1))
        W = int(rng.integers(w_range[0], w_range[1] + 1))
        fg = float(rng.uniform(*fg_range))
        specs.append(dict(seed=100 + i, H=H, W=W, fg_frac=fg))
    return specs


def soft_targets(gt, scale_log2, pairs):
    """Per-pair training targets, concatenated in pair order (float32).

    Target of pair (class c, scale slot si) at scale k = scale_log2[si]: the
    mean of the 40x ground-truth mask of class c over each 2^k x 2^k block,
    blocks reaching past the slide counting as background.
    """
    out = []
    H, W = gt.shape[1:]
    for (c, si) in pairs:
        f = 1 << scale_log2[si]
        Hk, Wk = -(-H // f), -(-W // f)
        m = np.zeros((Hk * f, Wk * f), np.float64)
        m[:H, :W] = gt[c]
        out.append(m.reshape(Hk, f, Wk, f).mean(axis=(1, 3)).ravel())
    return np.concatenate(out).astype(np.float32)

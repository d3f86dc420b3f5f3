"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package draws random numbers and rasterises shapes; it holds none of the
segmentation method's arithmetic (no padding, resampling, convolution, head,
controller or stitch).  Both sides of every parity check take their inputs
from here, so the only thing they share is the input itself.
"""

from .slides import (
    ellipse_slide,
    strip_slide,
    strip_crop_origin,
    tiny_slide,
    batch_slide_specs,
    soft_targets,
    CLASS_NAMES,
)
from .weights import weight_layout, he_normal_weights, head_param_count, training_init_weights

__all__ = [
    "ellipse_slide",
    "strip_slide",
    "strip_crop_origin",
    "tiny_slide",
    "batch_slide_specs",
    "soft_targets",
    "CLASS_NAMES",
    "weight_layout",
    "he_normal_weights",
    "head_param_count",
    "training_init_weights",
]

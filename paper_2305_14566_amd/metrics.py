"""Host-side comparison metrics for segmentation outputs (numpy).

  * normwise logit error  max_p |a - b| / max_p |b| over covered pixels;
  * Dice                  2 |A & B| / (|A| + |B|), 1 when both masks are empty;
  * disagreement          |A xor B| / #pixels;
  * at-risk fraction      share of pixels whose reference logit is within the
                          measured error of the threshold (either mask value
                          is then within the path's error bound).
"""

import numpy as np


def normwise_error(a, ref, covered=None):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    if covered is not None:
        a, ref = a[covered], ref[covered]
    den = np.abs(ref).max() if ref.size else 0.0
    if den == 0:
        return float(np.abs(a - ref).max()) if a.size else 0.0
    return float(np.abs(a - ref).max() / den)


def dice(a, b):
    a = np.asarray(a, bool)
    b = np.asarray(b, bool)
    s = a.sum() + b.sum()
    if s == 0:
        return 1.0
    return float(2.0 * (a & b).sum() / s)


def disagreement(a, b):
    a = np.asarray(a, bool)
    b = np.asarray(b, bool)
    return float((a ^ b).mean()) if a.size else 0.0


def at_risk_fraction(ref_logit, max_abs_err):
    ref = np.asarray(ref_logit, np.float64)
    return float((np.abs(ref) <= max_abs_err).mean()) if ref.size else 0.0

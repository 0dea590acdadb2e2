"""Error metrics between a computed field and the oracle's (test infrastructure only).

Readings for "max and RMS relative error", which are undefined pointwise near zero:
* rel_rms  = ||x - x_o||_2 / ||x_o||_2 over all points;
* rel_max  = max |x - x_o| / max |x_o|;
* rel_pointwise_max = max |x - x_o| / |x_o| over points with |x_o| >= 0.1 rms(x_o);
* radius mismatch = fraction of points whose radius index differs.
"""

import numpy as np


def rel_rms(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sqrt(np.sum(ref * ref))
    return float(np.sqrt(np.sum((x - ref) ** 2)) / den) if den > 0 else float(np.max(np.abs(x)))


def rel_max(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(x - ref)) / den) if den > 0 else float(np.max(np.abs(x)))


def rel_pointwise_max(x, ref, floor=0.1):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = np.sqrt(np.mean(ref * ref))
    sel = np.abs(ref) >= floor * rms
    if not np.any(sel):
        return 0.0
    return float(np.max(np.abs(x[sel] - ref[sel]) / np.abs(ref[sel])))


def mismatch_fraction(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.count_nonzero(a != b)) / a.size


def report(x, ref):
    return {"rel_rms": rel_rms(x, ref), "rel_max": rel_max(x, ref),
            "rel_pointwise_max": rel_pointwise_max(x, ref)}

"""The parity metric: error of a result relative to the reference, per result.

For one q with results over frequencies w, the error of each result is
|got(q, w) - ref(q, w)| / max(|ref(q, w)|, 1e-3 * max_w |ref(q, .)|): relative to the result
itself, with a floor so that frequencies where the reference nearly vanishes (the tails of Im chi0)
do not turn rounding into large ratios.  A q is summarised by the max and the mean over its
frequencies.  For a single static value per q this is |got - ref| / |ref|.
"""
import numpy as np

FLOOR = 1e-3


def per_result(got, ref):
    """Errors per result (same shape as ref, last axis = frequencies)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    mag = np.abs(ref)
    floor = FLOOR * np.max(mag, axis=-1, keepdims=True)
    den = np.maximum(np.maximum(mag, floor), 1e-300)
    return np.abs(got - ref) / den


def max_err(got, ref) -> float:
    return float(np.max(per_result(got, ref)))


def mean_err(got, ref) -> float:
    return float(np.mean(per_result(got, ref)))

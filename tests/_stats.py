"""Statistical acceptance rules shared by the tests.

Scalars: |a - b| <= k * sqrt(se_a^2 + se_b^2) (k = 3 unless stated).
Histograms: z-scores over slots that hold enough mass on both sides; accept when
the chi-square of the z-scores is below its 0.999 quantile and the largest
|z| is at most 5.  Fixed seeds make every outcome deterministic.

Same random numbers: where both sides replay the same Philox streams, their
difference comes only from paths whose FP32 and FP64 replays part at a
threshold (a Fresnel or roulette draw, a boundary test, a bin edge within
about 1e-6 of it), so the estimates agree to a small fraction of their
standard error: |z| <= SAME_STREAM_Z.
"""

from __future__ import annotations

import numpy as np
from scipy import stats

SAME_STREAM_Z = 0.5


def mean_se(sum_x, sum_x2, n):
    sum_x = np.asarray(sum_x, np.float64)
    sum_x2 = np.asarray(sum_x2, np.float64)
    n = np.asarray(n, np.float64)
    mean = sum_x / n
    var = np.maximum(sum_x2 - sum_x * sum_x / n, 0.0) / np.maximum(n - 1.0, 1.0)
    return mean, np.sqrt(var / n)


def zscore(a, se_a, b, se_b=0.0):
    se = np.sqrt(np.asarray(se_a, np.float64) ** 2 + np.asarray(se_b, np.float64) ** 2)
    return (np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.where(se > 0, se, np.inf)


def histogram_z(mean_a, se_a, mean_b, se_b, min_rel_se=None, mask=None):
    """z-scores per slot where both sides have nonzero SE (or the mask says so)."""
    mean_a = np.asarray(mean_a, np.float64)
    mean_b = np.asarray(mean_b, np.float64)
    se = np.sqrt(np.asarray(se_a, np.float64) ** 2 + np.asarray(se_b, np.float64) ** 2)
    ok = se > 0
    if mask is not None:
        ok &= mask
    if min_rel_se is not None:
        ok &= se <= min_rel_se * np.maximum(np.abs(mean_a), np.abs(mean_b))
    z = (mean_a[ok] - mean_b[ok]) / se[ok]
    return z


def accept_histogram(z, quantile=0.999, zmax=5.0):
    z = np.asarray(z)
    if z.size == 0:
        return True, 0.0, 0.0
    chi2 = float(np.sum(z * z))
    lim = float(stats.chi2.ppf(quantile, z.size))
    return (chi2 <= lim and float(np.max(np.abs(z))) <= zmax), chi2, lim

"""Flyvbjerg-Petersen blocking of a per-step (numerator, denominator) series and
the delta-method error of the ratio of their means (test helper)."""
import numpy as np


def ratio_se(num, den, min_blocks=16):
    num = np.asarray(num, float)
    den = np.asarray(den, float)
    n = len(num)
    best = 0.0
    a, b = num.copy(), den.copy()
    while len(a) >= min_blocks:
        ma, mb = a.mean(), b.mean()
        r = ma / mb
        # variance of the ratio of means by the delta method on block means
        g = (a - r * b) / mb
        se = np.sqrt(g.var(ddof=1) / len(g))
        best = max(best, se)
        m = len(a) // 2
        a = 0.5 * (a[:2 * m:2] + a[1:2 * m:2])
        b = 0.5 * (b[:2 * m:2] + b[1:2 * m:2])
    return num.mean() / den.mean(), best, n

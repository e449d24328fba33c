"""Structural similarity (Wang, Bovik, Sheikh and Simoncelli, IEEE TIP 2004)
for the curvature-flow study: local means, variances and covariance over a
7x7 uniform window (valid region only), dynamic range 1, K1 = 0.01,
K2 = 0.03, the mean of the SSIM map.  Test infrastructure, FP64 numpy."""
import numpy as np


def _box(a, k):
    c = np.cumsum(np.cumsum(np.pad(a, ((1, 0), (1, 0))), axis=0), axis=1)
    return (c[k:, k:] - c[:-k, k:] - c[k:, :-k] + c[:-k, :-k]) / (k * k)


def ssim(x, y, win=7):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    c1, c2 = (0.01) ** 2, (0.03) ** 2
    n = win * win
    mx, my = _box(x, win), _box(y, win)
    # unbiased local (co)variances
    vx = (_box(x * x, win) - mx * mx) * n / (n - 1)
    vy = (_box(y * y, win) - my * my) * n / (n - 1)
    cxy = (_box(x * y, win) - mx * my) * n / (n - 1)
    m = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return float(m.mean())

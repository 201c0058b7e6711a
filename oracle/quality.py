"""Quality metrics of the paper's evaluation, plain float64 numpy -- TEST
INFRASTRUCTURE ONLY (tests/, the smoke check and the benchmark's CPU-baseline
leg may use it).  Shares nothing with the GPU library.

SSIM (Eq. 3, Section III-C): for two fields D1 (original) and D2
(decompressed), per window

    SSIM = (2 mu1 mu2 + c1)(2 s12 + c2) / ((mu1^2 + mu2^2 + c1)(s1^2 + s2^2 + c2))

with the sample means mu, sample variances s^2 and sample covariance s12 of
the window's voxels, c1 = 1e-4 and c2 = 9e-4; the field's SSIM is the mean over
all windows of a sliding window of 7 voxels per axis moved by a stride of 2.
PSNR (Eq. 4): 20 log10((max D1 - min D1) / sqrt(MSE(D1, D2))).

Readings taken where the paper is silent:
* both fields are first normalised by the original's range,
  (D - min D1) / (max D1 - min D1), so that the constants c1, c2 (which assume
  values in [0, 1]) apply to any field;
* "sample" variance and covariance divide by m - 1 (m voxels per window);
* an axis shorter than 7 voxels takes its whole extent as the window (one
  position along it); only whole windows are used (starts 0, 2, 4, ... while
  the window fits).
"""
from __future__ import annotations

import numpy as np

C1, C2 = 1e-4, 9e-4
WINDOW, STRIDE = 7, 2


def _as3(a):
    a = np.asarray(a)
    while a.ndim < 3:
        a = a[None]
    return a


def window_starts(n, window=WINDOW, stride=STRIDE):
    """Start indices of the windows along an axis of extent n, and the window
    extent used along it."""
    w = min(window, n)
    return list(range(0, n - w + 1, stride)), w


def window_stats(d1, d2, window=WINDOW, stride=STRIDE):
    """Per-window (mu1, mu2, s1^2, s2^2, s12) of the range-normalised fields,
    arrays indexed by window position (z, y, x)."""
    a, b = _as3(d1).astype(np.float64), _as3(d2).astype(np.float64)
    if a.shape != b.shape:
        raise ValueError("fields differ in shape")
    lo, hi = a.min(), a.max()
    rng = hi - lo
    if not rng > 0:
        raise ValueError("the original field is constant: SSIM normalisation undefined")
    a = (a - lo) / rng
    b = (b - lo) / rng
    (sz, wz), (sy, wy), (sx, wx) = (window_starts(n, window, stride) for n in a.shape)
    m = wz * wy * wx
    if m < 2:
        raise ValueError("a window needs at least two voxels")
    out = np.empty((5, len(sz), len(sy), len(sx)))
    for i, z in enumerate(sz):
        for j, y in enumerate(sy):
            for k, x in enumerate(sx):
                u = a[z:z + wz, y:y + wy, x:x + wx].ravel()
                v = b[z:z + wz, y:y + wy, x:x + wx].ravel()
                mu, mv = u.mean(), v.mean()
                out[0, i, j, k] = mu
                out[1, i, j, k] = mv
                out[2, i, j, k] = ((u - mu) ** 2).sum() / (m - 1)
                out[3, i, j, k] = ((v - mv) ** 2).sum() / (m - 1)
                out[4, i, j, k] = ((u - mu) * (v - mv)).sum() / (m - 1)
    return out


def ssim_map(d1, d2, window=WINDOW, stride=STRIDE):
    mu1, mu2, v1, v2, cv = window_stats(d1, d2, window, stride)
    return ((2 * mu1 * mu2 + C1) * (2 * cv + C2)) / ((mu1 ** 2 + mu2 ** 2 + C1) * (v1 + v2 + C2))


def ssim(d1, d2, window=WINDOW, stride=STRIDE):
    """Mean SSIM over all window positions (Eq. 3)."""
    return float(ssim_map(d1, d2, window, stride).mean())


def psnr(d1, d2):
    """Eq. 4; +inf when the fields are equal."""
    a, b = np.asarray(d1, np.float64), np.asarray(d2, np.float64)
    mse = float(((a - b) ** 2).mean())
    rng = float(a.max() - a.min())
    return float("inf") if mse == 0.0 else 20.0 * np.log10(rng / np.sqrt(mse))


def mse(d1, d2):
    a, b = np.asarray(d1, np.float64), np.asarray(d2, np.float64)
    return float(((a - b) ** 2).mean())

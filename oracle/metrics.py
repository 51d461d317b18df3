"""Restoration quality measures of Sec. 5.5, float64.

RE   = ||X_true - X||_F / ||X_true||_F.
PSNR = 10 log10( ||X_true - E(X_true)||_F^2 / ||X - X_true||_F^2 ), where
       E(X_true) is the mean intensity: the paper's definition uses the
       variance of the true image in the numerator, not a peak value.
peak_psnr is the usual 10 log10(n peak^2 / ||X - X_true||^2) for reference.
"""
from __future__ import annotations

import math

import numpy as np


def relative_error(x_true, x) -> float:
    x_true = np.asarray(x_true, np.float64)
    x = np.asarray(x, np.float64)
    return float(np.linalg.norm((x_true - x).ravel()) / np.linalg.norm(x_true.ravel()))


def psnr_paper(x_true, x) -> float:
    x_true = np.asarray(x_true, np.float64)
    x = np.asarray(x, np.float64)
    num = float(np.sum((x_true - x_true.mean()) ** 2))
    den = float(np.sum((x - x_true) ** 2))
    return 10.0 * math.log10(num / den)


def psnr_peak(x_true, x, peak=None) -> float:
    x_true = np.asarray(x_true, np.float64)
    x = np.asarray(x, np.float64)
    peak = float(x_true.max()) if peak is None else float(peak)
    mse = float(np.mean((x - x_true) ** 2))
    return 10.0 * math.log10(peak * peak / mse)

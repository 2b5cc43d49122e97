"""Restoration quality measures used to report results (host-side NumPy,
not part of the restoration itself).

psnr:        peak signal-to-noise ratio with the root-mean-square error and
             peak 255 (Section 5), no clipping of the estimate;
edge_map:    pixels whose Sobel gradient magnitude exceeds a threshold;
edge_error:  fraction of pixels where two edge maps disagree;
edge_recall: fraction of the true image's edge pixels that are edge pixels
             of the estimate (Section 5's edge experiment in a number).
"""
from __future__ import annotations

import numpy as np


def psnr(u_true, u_hat) -> float:
    a = np.asarray(u_true, dtype=np.float64)
    b = np.asarray(u_hat, dtype=np.float64)
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(255.0 ** 2 / mse)


def edge_map(u, threshold: float = 60.0) -> np.ndarray:
    """|Sobel gradient| > threshold (gray levels per pixel, replicated
    border)."""
    x = np.pad(np.asarray(u, dtype=np.float64), 1, mode="edge")
    gx = (x[:-2, 2:] + 2 * x[1:-1, 2:] + x[2:, 2:]) - (x[:-2, :-2] + 2 * x[1:-1, :-2] + x[2:, :-2])
    gy = (x[2:, :-2] + 2 * x[2:, 1:-1] + x[2:, 2:]) - (x[:-2, :-2] + 2 * x[:-2, 1:-1] + x[:-2, 2:])
    return np.hypot(gx, gy) > threshold


def edge_error(u_true, u_hat, threshold: float = 60.0) -> float:
    return float(np.mean(edge_map(u_true, threshold) != edge_map(u_hat, threshold)))


def edge_recall(u_true, u_hat, threshold: float = 60.0) -> float:
    e = edge_map(u_true, threshold)
    n = int(e.sum())
    return 1.0 if n == 0 else float((e & edge_map(u_hat, threshold)).sum() / n)

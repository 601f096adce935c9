"""Peak positions of a spectrum on the energy grid (host-side post-processing).

The paper identifies the vibrational levels with the peaks of I(E) but gives
no rule; the one used for every comparison here: local maxima with
I >= frac * max I, a maximum within `sep` of a higher one is dropped (the
finite-time window has side lobes at 4.7 % and 1.6 % of the main lobe, spaced
2 pi / T), and each position is refined by the vertex of the parabola through
the maximum and its two neighbours.
"""
from __future__ import annotations

import math

import numpy as np


def find_peaks(E: np.ndarray, I: np.ndarray, T: float, frac: float = 0.05, sep_windows: float = 3.0):
    """Return [(E_peak, I_peak)] sorted by energy; T is the total propagation time."""
    E = np.asarray(E, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    if I.size < 3 or not np.any(I > 0):
        return []
    top = float(I.max())
    cand = [k for k in range(1, I.size - 1) if I[k] >= I[k - 1] and I[k] > I[k + 1] and I[k] >= frac * top]
    cand.sort(key=lambda k: -I[k])
    sep = sep_windows * 2.0 * math.pi / T
    kept = []
    for k in cand:
        if all(abs(E[k] - E[m]) > sep for m in kept):
            kept.append(k)
    out = []
    dE = E[1] - E[0]
    for k in sorted(kept):
        y0, y1, y2 = I[k - 1], I[k], I[k + 1]
        den = y0 - 2.0 * y1 + y2
        off = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        out.append((float(E[k] + off * dE), float(y1)))
    return out


def peak_errors(ref, test, tol: float):
    """Match each reference peak to the nearest test peak within `tol`;
    return (max |dE| over matched peaks, number of reference peaks unmatched)."""
    worst = 0.0
    missing = 0
    for e, _ in ref:
        if not test:
            missing += 1
            continue
        d = min(abs(e - t) for t, _ in test)
        if d > tol:
            missing += 1
        else:
            worst = max(worst, d)
    return worst, missing


def smooth(E: np.ndarray, I: np.ndarray, sigma: float) -> np.ndarray:
    """I convolved with a normalised Gaussian of standard deviation sigma
    (hartree) on the uniform grid E, truncated at 4 sigma, edges renormalised:
    a band of many close levels then has a peak that Monte Carlo ripples at
    the 2 pi / T scale do not move."""
    E = np.asarray(E, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    de = E[1] - E[0]
    h = int(math.ceil(4.0 * sigma / de))
    x = np.arange(-h, h + 1) * de
    g = np.exp(-0.5 * (x / sigma) ** 2)
    num = np.convolve(I, g, mode="same")
    den = np.convolve(np.ones_like(I), g, mode="same")
    return num / den


def centroid(E: np.ndarray, I: np.ndarray, lo: float, hi: float) -> float:
    """First moment of I over the window [lo, hi] (hartree)."""
    E = np.asarray(E, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    m = (E >= lo) & (E <= hi)
    return float(np.sum(E[m] * I[m]) / np.sum(I[m]))

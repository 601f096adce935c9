"""Comparison rules between the HIP path and the oracle.

State parity: for every trajectory that is good on both sides and whose
monodromy matrix stays moderate (||M~(T)||_F <= 1e3 in the scaled coordinates
x = (p / sqrt(gamma), sqrt(gamma) q), where a harmonic flow is a rotation;
i.e. not chaotic enough to amplify rounding differences beyond the tolerance),
the scaled state (sqrt(gamma) q, p / sqrt(gamma), S, phi) and M~ agree to 1e-9
relative to max(1, |x|).  Flags agree for every trajectory whose largest |det(M)^2 - 1|
(on either side) lies outside the band [1e-7, 1e-5], a decade either side of
the 1e-6 threshold: the deviation the monitor measures is FP64 rounding stored
in M (what the monitor after Eq. (5) catches, shown by the binary128 and long
double probes), and each side stores its own rounding, so near the threshold
the two sides' values are independent draws of one noise; over 4096 steps at
F = 9 they differ by factors up to about 5.
"""
from __future__ import annotations

import numpy as np

STATE_TOL = 1e-9
M_NORM_CAP = 1e3
FLAG_BAND = (1e-7, 1e-5)


def scaled_monodromy(prob, M):
    """D M D^-1 with D = diag(1/sqrt(gamma) for p rows, sqrt(gamma) for q rows)."""
    sg = np.sqrt(prob.gamma)
    d = np.concatenate([1 / sg, sg])
    return M * d[:, None] / d[None, :]


def compare_states(prob, gpu: dict, ora, tol: float = STATE_TOL):
    """Return (n_compared, worst error, list of failures)."""
    F = prob.F
    sg = np.sqrt(prob.gamma)
    n = gpu["S"].shape[0]
    fails = []
    worst = 0.0
    compared = 0
    for j in range(n):
        so = ora.state(j)
        gg = bool(gpu["good"][j])
        if gg != so.good:
            md = max(so.maxdev, gpu["maxdev"][j])
            if not (FLAG_BAND[0] <= md <= FLAG_BAND[1]):
                fails.append((j, "flag", gg, so.good, so.maxdev, gpu["maxdev"][j]))
            continue
        if not gg:
            continue
        Mo = scaled_monodromy(prob, so.M)
        if np.linalg.norm(Mo) > M_NORM_CAP:
            continue
        xg = np.concatenate([sg * gpu["q"][:, j], gpu["p"][:, j] / sg, [gpu["S"][j], gpu["phi"][j]]])
        xo = np.concatenate([sg * so.q, so.p / sg, [so.S, so.phi]])
        err = np.max(np.abs(xg - xo) / np.maximum(1.0, np.abs(xo)))
        mg = scaled_monodromy(prob, gpu["M"][j])
        errM = np.max(np.abs(mg - Mo)) / max(1.0, np.max(np.abs(Mo)))
        e = max(err, errM)
        worst = max(worst, e)
        compared += 1
        if not (e <= tol):
            fails.append((j, "state", e))
    return compared, worst, fails


def flag_differences(gpu: dict, ora) -> list:
    """Indices whose stability flag differs between the two sides."""
    n = gpu["S"].shape[0]
    return [j for j in range(n) if bool(gpu["good"][j]) != ora.state(j).good]

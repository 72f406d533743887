"""Diagnostics of a sweep (oracle side): per-slice field and beam moments and
the windowed quantities the paper plots.

TEST INFRASTRUCTURE ONLY (see oracle/qsa_pic.py).  Plain definitions in
float64 (numpy):

  * transverse mean squares of the fields E_x, E_y, E_z, B_x, B_y, B_z per
    xi slice (E_perp from the stored psi derivatives and B_perp, as
    qsa_pic.output_fields defines them);
  * root-mean-square amplitudes <F^2>^(1/2) averaged over windows of xi
    (the field amplitudes of the paper's comparison with full PIC, Fig. 2);
  * field energies as fractions of the beam energy density,
    eps_F = <F^2>/(4 n_b gamma_b) in the normalized units (k_p = omega_p = 1,
    n_p = 1, so n_b = alpha): the paper's saturation estimates define
    eps_Bz and eps_Ey that way (discussion of Fig. 3);
  * per-slice sums of the beam weight and of its first and second momentum
    moments, and from them the weighted root-mean-square momentum spreads
    along and across the beam per window (Fig. 3f).

A beam particle belongs to slice floor(xi/dxi) when that lies in
[0, nxi) and its weight is non-zero.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

FIELDS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
BEAM_SUMS = ("w", "wux", "wuy", "wuz", "wux2", "wuy2", "wuz2")


def field_slice_means(out: Dict[str, np.ndarray]) -> np.ndarray:
    """[nxi, 6]: transverse means of the squares of FIELDS, from output
    fields [nxi, ny, nx] each."""
    return np.stack([np.mean(np.asarray(out[f], dtype=np.float64) ** 2, axis=(1, 2)) for f in FIELDS], axis=1)


def beam_slice_sums(beam: Dict[str, np.ndarray], dxi: float, nxi: int) -> np.ndarray:
    """[nxi, 7]: per-slice sums of BEAM_SUMS over the particles of each slice."""
    xi = np.asarray(beam["xi"], dtype=np.float64)
    w = np.asarray(beam["w"], dtype=np.float64)
    j = np.floor(xi / dxi)
    keep = (w != 0) & (j >= 0) & (j < nxi)
    j = j[keep].astype(np.int64)
    w = w[keep]
    u = [np.asarray(beam[k], dtype=np.float64)[keep] for k in ("ux", "uy", "uz")]
    cols = [w] + [w * c for c in u] + [w * c * c for c in u]
    out = np.zeros((nxi, len(cols)))
    for k, c in enumerate(cols):
        np.add.at(out[:, k], j, c)
    return out


def windows(per_slice: np.ndarray, dxi: float, window: float) -> np.ndarray:
    """Sums of per-slice rows over consecutive windows of round(window/dxi)
    slices (the last window may be shorter): [n_windows, ...]."""
    m = max(1, int(round(window / dxi)))
    n = per_slice.shape[0]
    return np.stack([per_slice[a:a + m].sum(axis=0) for a in range(0, n, m)])


def window_counts(nxi: int, dxi: float, window: float) -> np.ndarray:
    m = max(1, int(round(window / dxi)))
    return np.array([min(m, nxi - a) for a in range(0, nxi, m)], dtype=np.float64)


def field_rms(per_slice: np.ndarray, dxi: float, window: float) -> np.ndarray:
    """[n_windows, 6]: <F^2>^(1/2) over each window."""
    nxi = per_slice.shape[0]
    return np.sqrt(windows(per_slice, dxi, window) / window_counts(nxi, dxi, window)[:, None])


def energy_fraction(per_slice: np.ndarray, dxi: float, window: float, alpha: float, gamma_b: float) -> np.ndarray:
    """[n_windows, 6]: eps_F = <F^2>/(4 n_b gamma_b), n_b = alpha."""
    nxi = per_slice.shape[0]
    mean = windows(per_slice, dxi, window) / window_counts(nxi, dxi, window)[:, None]
    return mean / (4.0 * alpha * gamma_b)


def momentum_spread(sums: np.ndarray, dxi: float, window: float) -> np.ndarray:
    """[n_windows, 3]: weighted RMS spreads of u_x, u_y, u_z per window
    (sqrt(<u^2> - <u>^2)); NaN where a window holds no particle."""
    s = windows(sums, dxi, window)
    w = s[:, 0:1]
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = s[:, 1:4] / w
        var = s[:, 4:7] / w - mean * mean
    return np.sqrt(np.maximum(var, 0.0))

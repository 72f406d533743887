"""Pins of the diagnostics oracle: closed forms on constructed fields and
beams (no GPU)."""
import math

import numpy as np
import torch

from oracle import diagnostics as D
from oracle import qsa_pic as O


def _stored(nxi, ny, nx):
    return torch.zeros(7, nxi, ny, nx, dtype=torch.float64)


def test_field_means_of_analytic_fields():
    """E_x = -d_x psi + B_y and E_y = -d_y psi - B_x as the oracle stores
    them: a sine of amplitude A averages to A^2/2 over whole periods, a
    constant c to c^2, and the two parts of E_x add before squaring."""
    nxi, ny, nx = 3, 8, 16
    F = _stored(nxi, ny, nx)
    x = torch.arange(nx, dtype=torch.float64)
    A, b, c = 0.7, 0.25, -1.5
    F[O.DXPSI] = A * torch.sin(2 * math.pi * 3 * x / nx)   # E_x = -A sin(...)
    F[O.BZ] = c
    F[O.BX, 1] = b                                           # E_y = -b and B_x = b on slice 1
    F[O.EZ, 2] = torch.cos(2 * math.pi * torch.arange(ny, dtype=torch.float64) / ny)[:, None]
    F[O.BY, 2] = b                                           # E_x = b - A sin on slice 2
    m = D.field_slice_means({k: v.numpy() for k, v in O.output_fields(F).items()})
    ex, ey, ez, bx, by, bz = (m[:, k] for k in range(6))
    assert np.allclose(ex[:2], A * A / 2, rtol=0, atol=1e-15)
    assert math.isclose(ex[2], b * b + A * A / 2, abs_tol=1e-15)   # the cross term averages out
    assert np.allclose(ey, [0.0, b * b, 0.0], atol=1e-15)
    assert np.allclose(bx, [0.0, b * b, 0.0], atol=1e-15)
    assert np.allclose(ez, [0.0, 0.0, 0.5], atol=1e-15)
    assert np.allclose(by, [0.0, 0.0, b * b], atol=1e-15)
    assert np.allclose(bz, c * c, atol=1e-15)


def test_windows_rms_and_energy_fraction():
    """Windows of round(window/dxi) slices, the last one shorter; the RMS is
    the root of the window mean of the slice means; eps = <F^2>/(4 alpha
    gamma_b)."""
    dxi = 0.5
    per = np.zeros((10, 6))
    per[:, 5] = np.arange(10.0)                         # <Bz^2> = j on slice j
    rms = D.field_rms(per, dxi, window=2.0)             # 4 slices per window
    assert rms.shape == (3, 6)
    assert np.allclose(rms[:, 5], np.sqrt([1.5, 5.5, 8.5]))
    eps = D.energy_fraction(per, dxi, 2.0, alpha=1e-2, gamma_b=100.0)
    assert np.allclose(eps[:, 5], np.array([1.5, 5.5, 8.5]) / 4.0)


def test_beam_sums_and_spreads():
    """Particles binned by floor(xi/dxi); weightless ones and those outside
    [0, nxi) slices are left out; the weighted spread of u = m +- a is a."""
    dxi, nxi = 0.1, 4
    rng = np.random.default_rng(3)
    n = 1000
    j = rng.integers(0, nxi, n)
    xi = (j + rng.uniform(0.01, 0.99, n)) * dxi
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    # pairs (2k, 2k+1) share a slice and a weight, so each slice's u_z is
    # exactly m +- a with equal weight on both signs
    j[1::2] = j[0::2]
    xi[1::2] = xi[0::2]
    w = np.repeat(rng.uniform(0.5, 2.0, n // 2), 2)
    beam = {"xi": xi, "w": w, "ux": 0.3 * sign, "uy": np.full(n, 2.0), "uz": 1000.0 + 4.0 * sign}
    extra = {"xi": np.array([-0.05, nxi * dxi + 0.01, 0.15]), "w": np.array([1.0, 1.0, 0.0]),
             "ux": np.ones(3), "uy": np.ones(3), "uz": np.ones(3)}
    allb = {k: np.concatenate([beam[k], extra[k]]) for k in beam}
    s = D.beam_slice_sums(allb, dxi, nxi)
    ref_w = np.array([w[j == k].sum() for k in range(nxi)])
    assert np.allclose(s[:, 0], ref_w, rtol=1e-14)
    assert np.allclose(s[:, 2], 2.0 * ref_w, rtol=1e-14)
    sp = D.momentum_spread(s, dxi, window=dxi)        # one slice per window
    assert np.allclose(sp[:, 0], 0.3, rtol=1e-9)
    assert np.allclose(sp[:, 1], 0.0, atol=1e-6)
    assert np.allclose(sp[:, 2], 4.0, rtol=1e-9)

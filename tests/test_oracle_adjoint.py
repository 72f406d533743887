"""Pins of the oracle's gradient of the transverse magnetic energy with
respect to beam-amplitude bins: central finite differences of the same
scheme, and Euler's relation for a degree-2 homogeneous objective in the
linear-response limit."""
import numpy as np
import pytest

import qsa_workloads as W
from oracle import adjoint as A


def _case(alpha=0.1, nb=4, nxi=12, uth=0.01):
    return W.small_3d(16, 16, nxi).with_(
        n_bins=nb, dt=5.0, plasma_uth=uth, species=(W.Species(Z=-1, alpha=alpha, ppc=2, sigma_par=1e-3),))


def test_gradient_matches_central_differences():
    wl = _case()
    plasma, beams = W.plasma_template(wl), W.beam(wl)
    amps = np.array([1.0, 0.8, 1.2, 1.0])
    L, g = A.energy_and_gradient(wl, plasma, beams, 2, amps)
    eps = 1e-4
    for b in range(4):
        ap, am = amps.copy(), amps.copy()
        ap[b] += eps
        am[b] -= eps
        fd = (A.energy(wl, plasma, beams, 2, ap) - A.energy(wl, plasma, beams, 2, am)) / (2 * eps)
        assert abs(fd - g[b]) <= 1e-6 * np.abs(g).max(), (b, g[b], fd)


def test_linear_limit_euler_relation():
    """Cold plasma (no fields without the beam), alpha = 1e-4, no beam push:
    fields are linear in the amplitudes to O(alpha), the energy quadratic, so
    sum_b a_b dL/da_b = 2 L."""
    wl = _case(alpha=1e-4, uth=0.0)
    plasma, beams = W.plasma_template(wl), W.beam(wl)
    amps = np.array([1.0, 0.5, 1.5, 0.9])
    L, g = A.energy_and_gradient(wl, plasma, beams, 0, amps)
    assert float(np.dot(amps, g)) == pytest.approx(2.0 * L, rel=2e-3)

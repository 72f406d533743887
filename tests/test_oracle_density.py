"""Pins of the oracle's plasma density profile (the paper's conclusion lists
plasma inhomogeneity in its outlook): the electrons carry the density in
their weights, the immobile ions match it at the nodes.

* A uniform plasma of density n0 behind a wide, weak electron beam rings at
  its own plasma frequency sqrt(n0): the 1D wake equation
  psi'' = alpha beta + (n0/2)((1 + psi)^-2 - 1) (the k_perp = 0 limit of the
  linear response behind Eqs. (1)-(2), with the plasma current scaled by n0)
  has the small-amplitude solution psi = (alpha beta/n0)(1 - cos(sqrt(n0) xi)).
  Leaving the ions at density 1 (or scaling only the electrons) breaks it.
* A neutral, cold, transversely modulated plasma with no beam is an
  equilibrium: the fields vanish as the grid is refined, at second order (the
  electrons' deposit matches the ions' node density up to O(dx^2)); ions laid
  along the wrong axis leave O(1) fields."""
import math

import numpy as np
import torch
from scipy.integrate import solve_ivp

import qsa_workloads as W
from oracle import qsa_pic as O


def _wake(h, n0, alpha=1e-4, length=8.0):
    n = 4
    nxi = int(round(length / h)) + 1
    wl = W.Workload(name="wake1d_n0", nx=n, ny=n, nxi=nxi, dx=0.25, dy=0.25, dxi=h,
                    gamma_b=100.0, species=(W.Species(Z=-1, alpha=alpha, ppc=8),),
                    plasma_mx=2, plasma_my=2, beam_loading="lattice", seed=1, plasma_n0=n0)
    pl = W.plasma_template(wl)
    s = O.Sim(wl, pl, W.beam(wl))
    return wl, pl, s.sweep()


def test_uniform_density_rings_at_its_plasma_frequency():
    n0 = 2.25
    beta = math.sqrt(1 - 1e-4)
    wl, pl, f = _wake(0.05, n0)
    assert np.allclose(pl["ion"], n0)
    psi = f[O.PSI, :, 0, 0].numpy()
    xis = np.arange(wl.nxi) * wl.dxi
    lin = 1e-4 * beta / n0 * (1.0 - np.cos(math.sqrt(n0) * xis))
    # O(h^2) phase error and O(alpha) nonlinearity, both far below the
    # difference a density of 1 would make
    assert np.abs(psi - lin).max() < 5e-3 * 1e-4
    wrong = 1e-4 * beta * (1.0 - np.cos(xis))
    assert np.abs(psi - wrong).max() > 0.5e-4


def test_uniform_density_nonlinear_wake_follows_the_scaled_ode():
    n0, alpha = 0.64, 0.05
    beta = math.sqrt(1 - 1e-4)

    def rhs(t, s):
        return [s[1], alpha * beta + 0.5 * n0 * ((1.0 + s[0]) ** -2 - 1.0)]
    errs = []
    for h in (0.1, 0.05):
        wl, _, f = _wake(h, n0, alpha=alpha)
        xis = np.arange(wl.nxi) * h
        ref = solve_ivp(rhs, (0, xis[-1]), [0.0, 0.0], t_eval=xis, rtol=1e-12, atol=1e-14,
                        method="DOP853").y[0]
        errs.append(np.abs(f[O.PSI, :, 0, 0].numpy() - ref).max())
    order = math.log2(errs[0] / errs[1])
    assert 1.8 < order < 2.2, errs


def _equilibrium(nx, ions_transposed=False):
    L = 6.4
    wl = W.small_3d(nx, nx, 6, dx=L / nx, dy=L / nx, dxi=0.1, plasma_uth=0.0,
                    plasma_n0=1.3, plasma_mod=0.4, plasma_mod_mx=1, plasma_mod_my=0,
                    species=(W.Species(Z=-1, alpha=0.0, ppc=1),))
    pl = O.to_torch(W.plasma_template(wl))
    if ions_transposed:
        pl["ion"] = pl["ion"].t().contiguous()
    g = O.Grid.of(wl)
    src = torch.zeros((4, wl.nxi, wl.ny, wl.nx), dtype=O.F64)
    return O.slice_sweep(g, pl, src, 3, 0.75)


def test_modulated_neutral_plasma_is_an_equilibrium():
    e16 = float(_equilibrium(16)[O.PSI].abs().max())
    e32 = float(_equilibrium(32)[O.PSI].abs().max())
    order = math.log2(e16 / e32)
    assert e16 < 2e-2 and 1.8 < order < 2.2, (e16, e32, order)
    # ions along y against electrons modulated along x: a net charge of
    # O(0.5) whose response drives 1 + psi through the breakdown threshold
    try:
        bad = float(_equilibrium(16, ions_transposed=True)[O.PSI].abs().max())
    except O.QSABreakdown:
        bad = math.inf
    assert bad > 20 * e16, (bad, e16)

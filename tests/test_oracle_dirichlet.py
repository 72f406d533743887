"""Pins of the Dirichlet (conducting-wall) sine-transform solve of the oracle:
a single wall mode is solved exactly by its eigenvalue; the transform equals
scipy's DST-I and is its own inverse up to 2/(N+1); a superposition of modes
and kappa^2 > 0 (Helmholtz) divide mode by mode; the discrete solution of a
smooth source converges to the closed-form continuous solution; the slab
(ny = 1) case reduces to the 1D problem."""
import math

import numpy as np
import pytest
import scipy.fft as sf

from oracle import dirichlet as D


@pytest.mark.parametrize("nx,ny", [(7, 15), (31, 31), (63, 1)])
@pytest.mark.parametrize("kappa2", [0.0, 0.75])
def test_single_wall_mode_is_exact(nx, ny, kappa2):
    dx, dy = 0.1, 0.07
    Lx, Ly = (nx + 1) * dx, (ny + 1) * dy
    x = np.arange(1, nx + 1) * dx
    y = np.arange(1, ny + 1) * dy
    m = 3
    n = 2 if ny > 1 else 0
    fx = np.sin(m * math.pi * x / Lx)
    fy = np.sin(n * math.pi * y / Ly) if ny > 1 else np.ones(1)
    f = np.outer(fy, fx)
    lam = (m * math.pi / Lx) ** 2 + ((n * math.pi / Ly) ** 2 if ny > 1 else 0.0) + kappa2
    u = D.dirichlet_solve(f, dx, dy, kappa2)
    assert np.abs(u - f / lam).max() <= 1e-13 * np.abs(f / lam).max()


def test_transform_matches_scipy_dst1_and_inverts():
    rng = np.random.default_rng(3)
    for n in (1, 7, 31, 255):
        f = rng.standard_normal(n)
        S = D.dst1_matrix(n) @ f
        ref = sf.dst(f, type=1) / 2.0   # scipy's DST-I is 2 sum f sin(...)
        assert np.abs(S - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        back = D.dst1_matrix(n) @ S * 2.0 / (n + 1)
        assert np.abs(back - f).max() <= 1e-12


def test_superposition_and_helmholtz_divide_mode_by_mode():
    nx, ny, dx, dy, k2 = 15, 31, 0.2, 0.1, 0.3
    Lx, Ly = (nx + 1) * dx, (ny + 1) * dy
    x = np.arange(1, nx + 1) * dx
    y = np.arange(1, ny + 1) * dy
    modes = [(1, 1, 0.7), (4, 9, -1.3), (15, 31, 0.25)]   # the highest modes included
    f = np.zeros((ny, nx))
    want = np.zeros((ny, nx))
    for m, n, a in modes:
        phi = a * np.outer(np.sin(n * math.pi * y / Ly), np.sin(m * math.pi * x / Lx))
        f += phi
        want += phi / ((m * math.pi / Lx) ** 2 + (n * math.pi / Ly) ** 2 + k2)
    u = D.dirichlet_solve(f, dx, dy, k2)
    assert np.abs(u - want).max() <= 1e-13 * np.abs(want).max()
    # batched: leading dimensions are independent grids
    fb = np.stack([f, 2.0 * f, -f])
    ub = D.dirichlet_solve(fb, dx, dy, k2)
    for s, c in enumerate((1.0, 2.0, -1.0)):
        assert np.abs(ub[s] - c * want).max() <= 1e-13 * np.abs(want).max()


def test_converges_to_the_continuous_solution():
    """-u'' = 1 on (0, L) with u(0) = u(L) = 0 has u = x (L - x)/2: the
    slab solve of the constant source on N interior nodes (the sine series
    truncated at N modes) converges to it at second order in the spacing."""
    L = 1.0
    errs = []
    for N in (15, 31, 63, 127):
        dx = L / (N + 1)
        x = np.arange(1, N + 1) * dx
        u = D.dirichlet_solve(np.ones((1, N)), dx, 1.0)[0]
        errs.append(np.abs(u - x * (L - x) / 2.0).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) >= 1.8, (errs, orders)
    assert errs[-1] < 1e-4

"""Oracle of the conducting-wall (Dirichlet) transverse solves: the sine-
transform counterpart of the periodic Fourier solves of the field equations.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline use it; the library never does.

The transverse field equations of the quasistatic model (the pseudo-
potential's Poisson equation, Eq. (2) of the paper in its linear form, and the
Helmholtz-shifted B_perp iteration) are solved in a box whose walls at
x = 0, L_x and y = 0, L_y are perfect conductors where the potential
vanishes.  On nx x ny interior nodes x_i = i dx (i = 1..nx, L_x = (nx+1) dx),
y_l = l dy (l = 1..ny, L_y = (ny+1) dy) the solution is expanded in the wall
modes sin(m pi x/L_x) sin(n pi y/L_y), m = 1..nx, n = 1..ny, which vanish on
the walls; the operator -lap_perp + kappa^2 is diagonal in them with
eigenvalue (m pi/L_x)^2 + (n pi/L_y)^2 + kappa^2 (the continuous Laplacian's,
as the periodic solves use the exact |k|^2).  A slab (ny = 1) has only the x
walls and the x modes.

DST-I, the transform to those modes on the interior nodes, and its inverse:
    S[m] = sum_{i=1..N} f[i] sin(pi i m/(N+1)),
    f[i] = 2/(N+1) sum_{m=1..N} S[m] sin(pi i m/(N+1)).
Written out here as a plain matrix product in float64.

Parity of this module is pinned by tests/test_oracle_dirichlet.py: single wall
modes are reproduced exactly, the transform matches scipy's DST-I and its
inverse, and refinement converges to the continuous solution of a problem
with a closed form.
"""
from __future__ import annotations

import numpy as np


def dst1_matrix(n: int) -> np.ndarray:
    """[m-1, i-1] = sin(pi i m/(n+1)), i, m = 1..n."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return np.sin(np.pi * np.outer(k, k) / (n + 1))


def wall_eigenvalues(n: int, d: float) -> np.ndarray:
    """(m pi/L)^2 for m = 1..n, L = (n+1) d."""
    L = (n + 1) * d
    return (np.pi * np.arange(1, n + 1, dtype=np.float64) / L) ** 2


def dirichlet_solve(f: np.ndarray, dx: float, dy: float, kappa2: float = 0.0) -> np.ndarray:
    """Solve (-lap_perp + kappa2) u = f with u = 0 on the walls.

    f: [..., ny, nx] values at the interior nodes (ny = 1: a slab, x walls
    only).  Returns u of the same shape, float64."""
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape[-2], f.shape[-1]
    Sx = dst1_matrix(nx)
    lam = wall_eigenvalues(nx, dx)[None, :]
    if ny == 1:
        # transform along x, divide, transform back
        F = f @ Sx.T                                   # [..., 1, m]
        U = F / (lam + kappa2)
        return (U @ Sx) * (2.0 / (nx + 1))
    Sy = dst1_matrix(ny)
    lam = lam + wall_eigenvalues(ny, dy)[:, None]      # [n, m]
    F = Sy @ f @ Sx.T                                  # [..., n, m]
    U = F / (lam + kappa2)
    return (Sy.T @ U @ Sx) * (2.0 / (nx + 1)) * (2.0 / (ny + 1))

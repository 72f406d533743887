"""Linear quasistatic theory of the beam-plasma instabilities (oracle side).

TEST INFRASTRUCTURE ONLY.  Closed forms and a numerical solver of the
paper's single-mode equation, used to check growth rates measured in
particle runs.  Normalized units: k_p = omega_p = 1.

  * beam plasma frequency omega_bs^2 = Z_s^2 alpha_s/(gamma_b M_s) ("Quasistatic
    model" section; only the square is used, so the sign of Z_s is irrelevant);
  * temporal CFI rate Gamma = (sum_s omega_bs^2 k^2/(k^2+1))^(1/2), the
    definition after Eq. (5);
  * temporal OTSI rate Gamma_OTSI = (sqrt 3/2^(4/3)) Gamma^(2/3) (after Eq. (6),
    omega_p-normalized);
  * the asymptotic exponents of Eqs. (6) and (7), the transition ray
    xi = 2 Gamma tau/sqrt(27) and the rate (4/3) sqrt(2/3) Gamma seen along it
    (text after Eq. (7));
  * Eq. (5) itself, [(d_xi^2 + 1) d_tau^2 - Gamma^2] dPsi = 0, solved as the
    pair n = (d_xi^2 + 1) dPsi, dPsi(xi) = int_0^xi sin(xi - xi') n(xi') dxi'
    (the causal inverse: no perturbation ahead of the beam front), with
    d_tau^2 n = Gamma^2 dPsi advanced by classical RK4 in tau.
"""
from __future__ import annotations

import math
from typing import Iterable, Tuple

import numpy as np


def omega_b2(alpha: float, gamma_b: float, Z: int = -1, M: float = 1.0) -> float:
    return Z * Z * alpha / (gamma_b * M)


def gamma_cfi(k: float, species: Iterable[Tuple[int, float, float]], gamma_b: float) -> float:
    """Temporal CFI growth rate at transverse wavenumber k (definition after Eq. (5)).

    species: iterable of (Z, M, alpha)."""
    s = sum(omega_b2(a, gamma_b, Z, M) for Z, M, a in species)
    return math.sqrt(s * k * k / (k * k + 1.0))


def gamma_otsi(gamma: float) -> float:
    """Temporal OTSI rate from the CFI rate (text after Eq. (6))."""
    return math.sqrt(3.0) / 2.0 ** (4.0 / 3.0) * gamma ** (2.0 / 3.0)


def eq6_exponent(gt: float, xi: float) -> float:
    """Real exponent of Eq. (6): (3 sqrt 3/4)(Gamma tau)^(2/3) xi^(1/3)."""
    return 3.0 * math.sqrt(3.0) / 4.0 * gt ** (2.0 / 3.0) * xi ** (1.0 / 3.0)


def eq7_exponent(gt: float, xi: float) -> float:
    """Exponent of Eq. (7): 2 sqrt(Gamma tau xi) (1 - xi/(4 Gamma tau))."""
    return 2.0 * math.sqrt(gt * xi) * (1.0 - xi / (4.0 * gt))


RAY_SLOPE = 2.0 / math.sqrt(27.0)                     # xi_t = RAY_SLOPE * Gamma tau
RAY_RATE = 4.0 / 3.0 * math.sqrt(2.0 / 3.0)           # growth rate along the ray / Gamma


def solve_eq5(gamma, xi: np.ndarray, n0: np.ndarray, taus: np.ndarray,
              dtau: float) -> Tuple[np.ndarray, np.ndarray]:
    """Solve Eq. (5) for a seed n(xi, 0) = n0, d_tau n(xi, 0) = 0.

    gamma: a number, or Gamma(xi) on the grid (an arbitrary longitudinal
    beam profile, for which the paper generalizes Eq. (5) through Gamma(xi):
    d_tau^2 n = Gamma(xi)^2 Psi point by point).
    xi: uniform grid starting at 0.  Returns (n, Psi) sampled at the requested
    taus, arrays [len(taus), len(xi)].  The xi integral uses the trapezoid
    rule; tau uses classical RK4 with step dtau (taus must be multiples).
    """
    d = xi[1] - xi[0]
    nxi = xi.size
    A = np.sin(xi[:, None] - xi[None, :]) * d
    A = np.tril(A)
    A[:, 0] *= 0.5          # trapezoid end weight (the diagonal term is sin 0 = 0)
    g2 = np.asarray(gamma, dtype=np.float64) ** 2

    def rhs(state):
        n, v = state
        return np.stack([v, g2 * (A @ n)])

    st = np.stack([n0.astype(np.float64), np.zeros(nxi)])
    out_n, out_p = [], []
    t = 0.0
    for target in taus:
        nsteps = int(round((target - t) / dtau))
        for _ in range(nsteps):
            k1 = rhs(st)
            k2 = rhs(st + 0.5 * dtau * k1)
            k3 = rhs(st + 0.5 * dtau * k2)
            k4 = rhs(st + dtau * k3)
            st = st + dtau / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        t += nsteps * dtau
        out_n.append(st[0].copy())
        out_p.append(A @ st[0])
    return np.array(out_n), np.array(out_p)


def ray_rate(gamma: float, xi: np.ndarray, amp: np.ndarray, taus: np.ndarray,
             gt0: float, gt1: float) -> float:
    """Growth rate d ln|amp| / d tau along xi = RAY_SLOPE Gamma tau, fitted by
    least squares over Gamma tau in [gt0, gt1]; amp is [len(taus), len(xi)]."""
    sel = [(i, t) for i, t in enumerate(taus) if gt0 <= gamma * t <= gt1]
    ts, ls = [], []
    for i, t in sel:
        xr = RAY_SLOPE * gamma * t
        a = np.interp(xr, xi, np.abs(amp[i]))
        ts.append(t)
        ls.append(math.log(a))
    return float(np.polyfit(ts, ls, 1)[0])

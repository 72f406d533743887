"""Pins of the oracle's linear-theory module against numbers the paper prints
and against limits the mathematics fixes."""
import json
import math
import os

import numpy as np
import pytest

from oracle import linear_theory as L

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_cfi_rate_fig1_worked_number():
    g = GOLD["cfi_rate_fig1"]
    sp = [tuple(s) for s in g["species"]]
    val = L.gamma_cfi(g["k"], sp, g["gamma_b"])
    # printed to two significant digits: 1.7e-3
    assert round(val, 4) == pytest.approx(g["value"], abs=0.5e-4)


def test_cfi_rate_large_k_limit():
    # k >> k_p: Gamma -> sqrt(sum alpha/gamma) (cold-beam filamentation rate)
    sp = [(-1, 1.0, 0.05), (1, 1.0, 0.05)]
    assert L.gamma_cfi(1e4, sp, 100.0) == pytest.approx(math.sqrt(0.1 / 100.0), rel=1e-7)
    # and the k^2/(k^2+1) factor at k = 1 halves the square
    assert L.gamma_cfi(1.0, sp, 100.0) ** 2 == pytest.approx(0.5 * 0.1 / 100.0, rel=1e-12)
    # the sign of Z does not matter, the mass does
    assert L.gamma_cfi(2.0, [(1, 1.0, 0.1)], 10.0) == L.gamma_cfi(2.0, [(-1, 1.0, 0.1)], 10.0)
    assert L.gamma_cfi(2.0, [(1, 4.0, 0.1)], 10.0) == pytest.approx(
        0.5 * L.gamma_cfi(2.0, [(1, 1.0, 0.1)], 10.0), rel=1e-12)


def test_otsi_rate_formula():
    # (sqrt 3/2^(4/3)) (alpha/gamma)^(1/3) for Gamma = sqrt(alpha/gamma)
    a, g = 1e-2, 1e3
    G = math.sqrt(a / g)
    assert L.gamma_otsi(G) == pytest.approx(math.sqrt(3) / 2 ** (4 / 3) * (a / g) ** (1 / 3), rel=1e-12)


def test_transition_ray_and_rate():
    assert L.RAY_SLOPE == pytest.approx(GOLD["transition_ray"]["slope"], abs=5e-5)
    assert round(L.RAY_RATE, 2) == GOLD["ray_rate"]["value"]
    # the CFI extent after N_e e-folds: xi_t = slope * Gamma tau ~ 0.4 N_e
    assert round(L.RAY_SLOPE, 1) == GOLD["cfi_extent"]["value"]
    # Eq. (7)'s exponent is maximal in tau-derivative terms at the ray only
    # asymptotically; at the ray the two asymptotes bracket the exact rate
    gt = 100.0
    xi = L.RAY_SLOPE * gt
    d7 = (L.eq7_exponent(gt * (1 + 1e-6), xi * (1 + 1e-6)) - L.eq7_exponent(gt, xi)) / (gt * 1e-6)
    d6 = (L.eq6_exponent(gt * (1 + 1e-6), xi * (1 + 1e-6)) - L.eq6_exponent(gt, xi)) / (gt * 1e-6)
    assert d6 < L.RAY_RATE < d7


def test_blazar_saturation_estimates():
    """Arithmetic of the blazar-section estimates, using gamma_cfi for Gamma."""
    b = GOLD["blazar_saturation"]
    sp = [(-1, 1.0, b["alpha"]), (1, 1.0, b["alpha"])]
    G = L.gamma_cfi(1.0, sp, b["gamma_b"])          # k_y ~ k_p
    eps_bz = (b["xi"] / b["tau_sat"]) ** 2 / 4.0
    assert eps_bz == pytest.approx(b["eps_Bz"], rel=0.05)
    gst = math.sqrt(G * b["xi"] / b["tau_sat"])
    assert b["gamma_b"] * gst == pytest.approx(b["dpy_cfi"], rel=0.08)
    o = GOLD["blazar_otsi"]
    eps_ey = 9.0 / 64.0 * (o["alpha"] / o["gamma_b"]) ** (1 / 3) * (o["xi"] / o["tau_sat"]) ** (4 / 3)
    assert eps_ey == pytest.approx(o["eps_Ey"], rel=0.05)
    gst = math.sqrt(3) / 2 * G ** (2 / 3) * (o["xi"] / o["tau_sat"]) ** (1 / 3)
    assert o["gamma_b"] * gst == pytest.approx(o["dpy_otsi"], rel=0.03)


def test_eq5_solver_flat_seed_short_time():
    """Series in tau: n = 1 + (tau^2/2) P[1] + (tau^4/24) P[P[1]] + O(tau^6), with
    P[1] = 1 - cos xi and P[P[1]] = (1 - cos xi) - (xi/2) sin xi."""
    xi = np.arange(0, 6.0, 0.01)
    t = 0.1
    n, p = L.solve_eq5(1.0, xi, np.ones_like(xi), np.array([t]), 0.01)
    p1 = 1 - np.cos(xi)
    p2 = p1 - 0.5 * xi * np.sin(xi)
    expect = 1.0 + 0.5 * t * t * p1 + t ** 4 / 24.0 * p2
    assert np.max(np.abs(n[0] - expect)) < 2e-7
    # Psi = int_0^xi sin(xi - s) n ds = 1 - cos xi at tau = 0 (to the rule's error)
    n0, p0 = L.solve_eq5(1.0, xi, np.ones_like(xi), np.array([0.0]), 0.01)
    assert np.max(np.abs(p0[0] - (1 - np.cos(xi)))) < 1e-4


def test_eq5_ray_rate_tends_to_saddle_value():
    """Along the transition ray the growth rate tends to (4/3) sqrt(2/3) Gamma."""
    xi = np.arange(0, 13.0, 0.02)
    taus = np.arange(0, 31.0, 0.5)
    n, p = L.solve_eq5(1.0, xi, np.ones_like(xi), taus, 0.02)
    r = L.ray_rate(1.0, xi, p, taus, 20.0, 30.0)
    assert r == pytest.approx(L.RAY_RATE, rel=0.01)
    # Gamma scaling: the same problem at Gamma = 0.5 gives half the rate
    n2, p2 = L.solve_eq5(0.5, xi, np.ones_like(xi), taus * 2, 0.04)
    r2 = L.ray_rate(0.5, xi, p2, taus * 2, 20.0, 30.0)
    assert r2 == pytest.approx(0.5 * r, rel=1e-3)


def test_eq5_solver_with_a_longitudinal_profile():
    """Gamma(xi) a step (0 ahead of xi0 = 1.5, 1 behind): nothing grows
    where Gamma = 0, and behind the step the short-time series holds,
    n = 1 + (tau^2/2) P[1] + (tau^4/24) P[g P[1]] with g the step and
    P[f](xi) = int_0^xi sin(xi - s) f(s) ds evaluated by adaptive quadrature."""
    from scipy.integrate import quad
    xi = np.arange(0, 4.0, 0.005)
    g = np.where(xi >= 1.5, 1.0, 0.0)
    t = 0.1
    n, _ = L.solve_eq5(g, xi, np.ones_like(xi), np.array([t, 2 * t]), 0.005)
    ahead = xi < 1.5
    assert np.array_equal(n[:, ahead], np.ones((2, ahead.sum())))
    # the constant profile is the scalar solver
    nc, pc = L.solve_eq5(np.full_like(xi, 0.7), xi, np.ones_like(xi), np.array([t]), 0.005)
    ns, ps = L.solve_eq5(0.7, xi, np.ones_like(xi), np.array([t]), 0.005)
    assert np.array_equal(nc, ns) and np.array_equal(pc, ps)

    def p_gp1(x):
        if x <= 1.5:
            return 0.0
        return quad(lambda s: np.sin(x - s) * (1 - np.cos(s)), 1.5, x, epsabs=1e-13, epsrel=1e-12)[0]

    for x in (2.0, 2.7, 3.5):
        i = int(round(x / 0.005))
        expect = 1.0 + 0.5 * t * t * (1 - np.cos(xi[i])) + t ** 4 / 24.0 * p_gp1(xi[i])
        assert abs(n[0, i] - expect) < 1e-6, (x, n[0, i], expect)

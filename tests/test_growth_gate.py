"""Growth-rate gates: current filamentation along the transition ray, and
the oblique two-stream region behind it (second half of this file).

Filamentation: the pair-beam slab with a single
seeded transverse mode (lattice-loaded e- and e+ beams, weights modulated
+-1e-3 at mode m = 5), |B_y(k_m)| sampled along the ray xi = (2/sqrt 27)
Gamma tau, growth rate fitted over Gamma tau in [4, 7.75].

Reference: the linear model of the paper (Eq. (5), solved numerically for a
uniform seed) over the same window.  The beam current, hence B_y, follows
the beam density perturbation n of that model, whose rate along the ray is
1.04 Gamma there; the asymptotic value (4/3) sqrt(2/3) Gamma = 1.0887 Gamma
of the saddle-point analysis is only approached at much larger Gamma tau.
Gate: the measured rate within 5% of the model's.
"""
import math

import numpy as np
import pytest

import qsa_workloads as W
from oracle import linear_theory as LT

M = 5
NXI = 40                         # the ray stays below xi = 3.1 over the window
STEPS = 52                       # Gamma tau up to 8.06 at dt = 5
WINDOW = (4.0, 7.75)


def _workload():
    return W.slab_pair(seeded_mode=True, m=M).with_(nxi=NXI)


def _gamma(wl):
    km = 2.0 * math.pi * M / (wl.nx * wl.dx)
    sp = [(s.Z, s.M, s.alpha) for s in wl.species]
    return LT.gamma_cfi(km, sp, wl.gamma_b)


def _ray_amplitude(wl, by_slices, tau, gamma):
    """|B_y(k_m)| (physical amplitude) interpolated at the ray's xi."""
    xi = LT.RAY_SLOPE * gamma * tau
    jf = xi / wl.dxi
    j0 = int(math.floor(jf))
    f = jf - j0
    amp = np.abs(np.fft.rfft(by_slices, axis=1)[:, M]) * 2.0 / wl.nx
    return (1.0 - f) * amp[j0] + f * amp[j0 + 1]


def _fit_rate(gts, amps):
    gts, amps = np.asarray(gts), np.asarray(amps)
    sel = (gts >= WINDOW[0]) & (gts <= WINDOW[1])
    assert sel.sum() >= 8
    return float(np.polyfit(gts[sel], np.log(amps[sel]), 1)[0])


def _model_rate(gamma):
    xi = np.arange(0.0, 4.0 + 1e-12, 0.02)
    dtau = 1.0
    taus = np.arange(0.0, (WINDOW[1] + 0.5) / gamma, 5.0)
    taus = np.round(taus / dtau) * dtau
    n, _ = LT.solve_eq5(gamma, xi, np.ones_like(xi), taus, dtau)
    return LT.ray_rate(gamma, xi, n, taus, *WINDOW) / gamma


def test_model_rate_over_the_window():
    """The model's density rate over the window (the gate's reference) lies
    between the window's start-up value and the asymptotic ray rate."""
    r = _model_rate(_gamma(_workload()))
    assert 1.0 < r < LT.RAY_RATE


def test_oracle_cfi_growth_gate():
    from oracle import qsa_pic as O
    wl = _workload()
    gamma = _gamma(wl)
    sim = O.Sim(wl, O.to_torch(W.plasma_template(wl)), [O.to_torch(b) for b in W.beam(wl)])
    gts, amps = [], []
    for n in range(STEPS + 1):
        sim.sweep()
        by = O.output_fields(sim.fields)["By"].numpy()[:, 0, :]
        gts.append(gamma * n * wl.dt)
        amps.append(_ray_amplitude(wl, by, n * wl.dt, gamma))
        if n < STEPS:
            sim.push()
    rate = _fit_rate(gts, amps)
    model = _model_rate(gamma)
    print(f"[gate] oracle rate {rate:.4f} Gamma, model {model:.4f} Gamma", flush=True)
    assert abs(rate / model - 1.0) <= 0.05, (rate, model)


@pytest.mark.gpu
def test_gpu_cfi_growth_gate_and_history():
    """The same run on the GPU (float64): the gate, and the amplitude history
    along the ray against the oracle's (the linear phase amplifies rounding
    differences only mildly)."""
    import paper_2607_24214_amd as Q
    from oracle import qsa_pic as O
    wl = _workload()
    gamma = _gamma(wl)
    plasma, beams = W.plasma_template(wl), W.beam(wl)
    sg = Q.Sim(Q.params_from_workload(wl, precision="f64"))
    sg.load_plasma(plasma)
    for s, b in enumerate(beams):
        sg.load_beam(s, b)
    so = O.Sim(wl, O.to_torch(plasma), [O.to_torch(b) for b in beams])
    gts, ag, ao = [], [], []
    for n in range(STEPS + 1):
        # a beam step sweeps at tau_n and then pushes: its fields are tau_n's
        if n < STEPS:
            sg.beam_step(1)
        else:
            sg.slice_sweep()
        so.sweep()
        tau = n * wl.dt
        gts.append(gamma * tau)
        ag.append(_ray_amplitude(wl, sg.fields("By")[:, 0, :], tau, gamma))
        ao.append(_ray_amplitude(wl, O.output_fields(so.fields)["By"].numpy()[:, 0, :], tau, gamma))
        if n < STEPS:
            so.push()
    rate = _fit_rate(gts, ag)
    model = _model_rate(gamma)
    rel = max(abs(a / b - 1.0) for a, b in zip(ag, ao))
    print(f"[gate] GPU rate {rate:.4f} Gamma, model {model:.4f}; history vs oracle {rel:.2e}", flush=True)
    assert abs(rate / model - 1.0) <= 0.05, (rate, model)
    assert rel <= 1e-8, rel


# ---------------------------------------------------------------------------
# Behind the transition ray (k_p xi >> 2 Gamma tau / sqrt 27: the region of
# the spatiotemporal oblique two-stream growth of Eq. (6)) the seeded mode
# oscillates along xi like exp(i k_p xi), so its growth is measured on the
# envelope: the largest |B_y(k_m)| over one plasma wavelength centred on
# xi0.  The whole 12.8-long slab, a seed of 1e-8 (the 1e-3 seed of the gate
# above is nonlinear there by Gamma tau ~ 5), the same window and reference
# model; gate: within 5% at xi0 = 8 and 9.5 (envelope windows wholly behind
# the ray, which stays below xi = 3).

OTSI_XI0 = (8.0, 9.5)


def _otsi_workload():
    return W.slab_pair(seeded_mode=True, m=M, eps=1e-8)


def _envelope(amp, x, x0):
    sel = (x >= x0 - math.pi) & (x <= x0 + math.pi)
    return np.abs(amp[..., sel]).max(axis=-1)


def _otsi_model_rates(gamma, gts):
    xm = np.arange(0.0, 12.8 + 1e-12, 0.02)
    taus = np.round(np.asarray(gts) / gamma)
    n, _ = LT.solve_eq5(gamma, xm, np.ones_like(xm), taus, 1.0)
    return [_fit_rate(gts, _envelope(n, xm, x0)) for x0 in OTSI_XI0]


def _mode_amplitudes(wl, by_slices):
    return np.abs(np.fft.rfft(by_slices, axis=1)[:, M]) * 2.0 / wl.nx


def _otsi_check(wl, gamma, gts, hist, who):
    xs = np.arange(wl.nxi) * wl.dxi
    hist = np.asarray(hist)
    model = _otsi_model_rates(gamma, gts)
    for x0, mr in zip(OTSI_XI0, model):
        r = _fit_rate(gts, _envelope(hist, xs, x0))
        print(f"[gate] {who} envelope rate at xi0 = {x0}: {r:.4f} Gamma, model {mr:.4f} Gamma", flush=True)
        assert abs(r / mr - 1.0) <= 0.05, (x0, r, mr)


# ---------------------------------------------------------------------------
# Front region (G2): behind the beam head and ahead of the transition ray
# (0.5 <= xi < 2 Gamma tau/sqrt 27, Gamma tau in [1, 6]) the seeded mode's
# |psi(k_m)| is fitted by least squares in log amplitude to the linear
# model's potential U(xi, Gamma tau) (Eq. (5) for a uniform seed depends on
# xi and Gamma tau only), with the growth rate Gamma and an amplitude free.
# Gate: the fitted Gamma within 5% of the model's Gamma for this beam.

FRONT_WINDOW = (1.0, 6.0)


def _front_model(gmax):
    """Potential of Eq. (5) with Gamma = 1 on xi in [0, 4], Gamma tau in
    [0, gmax] (step 0.05): [len(s), len(xi)]."""
    xi = np.arange(0.0, 4.0 + 1e-12, 0.02)
    s = np.arange(0.0, gmax + 1e-9, 0.05)
    _, psi = LT.solve_eq5(1.0, xi, np.ones_like(xi), s, 0.05)
    return xi, s, np.abs(psi)


def _front_fit(wl, gts, psi_hist, gamma):
    """Gamma_fit / gamma from the least-squares fit of ln|psi(k_m)| over
    the front region."""
    xs = np.arange(wl.nxi) * wl.dxi
    taus = np.asarray(gts) / gamma
    pts = [(i, j) for i, gt in enumerate(gts) if FRONT_WINDOW[0] <= gt <= FRONT_WINDOW[1]
           for j, x in enumerate(xs) if 0.5 <= x < LT.RAY_SLOPE * gt]
    assert len(pts) >= 40, len(pts)
    lv = np.array([math.log(psi_hist[i][j]) for i, j in pts])
    xm, sm, U = _front_model(1.3 * FRONT_WINDOW[1])

    def resid(g):
        # the model at (xi, g tau): bilinear in the tabulated (s, xi)
        m = []
        for i, j in pts:
            s = g * taus[i]
            a = min(int(s / 0.05), len(sm) - 2)
            fa = s / 0.05 - a
            u = (1 - fa) * np.interp(xs[j], xm, U[a]) + fa * np.interp(xs[j], xm, U[a + 1])
            m.append(math.log(u))
        d = lv - np.array(m)
        return float(np.sum((d - d.mean()) ** 2))     # the amplitude fitted out

    # golden-section search for the rate over [0.7, 1.3] Gamma
    lo, hi = 0.7 * gamma, 1.3 * gamma
    r = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = hi - r * (hi - lo), lo + r * (hi - lo)
    fa, fb = resid(a), resid(b)
    for _ in range(40):
        if fa < fb:
            hi, b, fb = b, a, fa
            a = hi - r * (hi - lo)
            fa = resid(a)
        else:
            lo, a, fa = a, b, fb
            b = lo + r * (hi - lo)
            fb = resid(b)
    return 0.5 * (lo + hi) / gamma


def _front_check(wl, gamma, gts, psi_hist, who):
    g = _front_fit(wl, gts, psi_hist, gamma)
    print(f"[gate] {who} front-region fit of |psi(k_m)|: Gamma_fit = {g:.4f} Gamma", flush=True)
    assert abs(g - 1.0) <= 0.05, g


def test_oracle_growth_behind_the_ray():
    """The envelope gate behind the ray and, on the same run, the
    front-region least-squares fit of |psi(k_m)| to the linear model."""
    from oracle import qsa_pic as O
    wl = _otsi_workload()
    gamma = _gamma(wl)
    sim = O.Sim(wl, O.to_torch(W.plasma_template(wl)), [O.to_torch(b) for b in W.beam(wl)])
    gts, hist, phist = [], [], []
    for n in range(STEPS + 1):
        sim.sweep()
        gts.append(gamma * n * wl.dt)
        of = O.output_fields(sim.fields)
        hist.append(_mode_amplitudes(wl, of["By"].numpy()[:, 0, :]))
        phist.append(_mode_amplitudes(wl, of["psi"].numpy()[:, 0, :]))
        if n < STEPS:
            sim.push()
    _otsi_check(wl, gamma, gts, hist, "oracle")
    _front_check(wl, gamma, gts, phist, "oracle")


@pytest.mark.gpu
def test_gpu_growth_behind_the_ray():
    import paper_2607_24214_amd as Q
    wl = _otsi_workload()
    gamma = _gamma(wl)
    sg = Q.Sim(Q.params_from_workload(wl, precision="f64"))
    sg.load_plasma(W.plasma_template(wl))
    for s, b in enumerate(W.beam(wl)):
        sg.load_beam(s, b)
    gts, hist, phist = [], [], []
    for n in range(STEPS + 1):
        if n < STEPS:
            sg.beam_step(1)
        else:
            sg.slice_sweep()
        gts.append(gamma * n * wl.dt)
        hist.append(_mode_amplitudes(wl, sg.fields("By")[:, 0, :]))
        phist.append(_mode_amplitudes(wl, sg.fields("psi")[:, 0, :]))
    _otsi_check(wl, gamma, gts, hist, "GPU")
    _front_check(wl, gamma, gts, phist, "GPU")


# ---------------------------------------------------------------------------
# Noise-seeded run (G3, reported): the pair slab as specified (random
# positions, longitudinal spread 1e-3, no seeded mode), the growth of the
# RMS E_x and B_y over windows of width 2 centred on xi = 2 and xi = 10 (the
# paper's window method), from the device diagnostics after every step.
# The rates are printed next to the gates above; the check is only that the
# noise grows at rates of the order of Gamma in the linear window.

G3_XI0 = (2.0, 10.0)


@pytest.mark.gpu
def test_gpu_noise_seeded_window_rates_report():
    import paper_2607_24214_amd as Q
    wl = W.slab_pair(seeded_mode=False)
    gamma = _gamma(wl)
    sg = Q.Sim(Q.params_from_workload(wl, precision="f64"))
    sg.load_plasma(W.plasma_template(wl))
    for s, b in enumerate(W.beam(wl)):
        sg.load_beam(s, b)
    half = int(round(1.0 / wl.dxi))          # windows of 1 c/omega_p, paired around xi0
    gts, ex, by = [], [], []
    for n in range(STEPS + 1):
        if n < STEPS:
            sg.beam_step(1)
        else:
            sg.slice_sweep()
        fm = sg.field_moments(half)            # [windows, (Ex^2, Ey^2, Ez^2, Bx^2, By^2, Bz^2)]
        gts.append(gamma * n * wl.dt)
        ex.append([math.sqrt(0.5 * (fm[int(x0) - 1, 0] + fm[int(x0), 0])) for x0 in G3_XI0])
        by.append([math.sqrt(0.5 * (fm[int(x0) - 1, 4] + fm[int(x0), 4])) for x0 in G3_XI0])
    ex, by = np.asarray(ex), np.asarray(by)
    rates = []
    for k, x0 in enumerate(G3_XI0):
        rex, rby = _fit_rate(gts, ex[:, k]), _fit_rate(gts, by[:, k])
        print(f"[gate] noise-seeded RMS rates at xi0 = {x0}: E_x {rex:.3f} Gamma, B_y {rby:.3f} Gamma", flush=True)
        rates += [rex, rby]
    assert all(math.isfinite(r) and r < 3.0 for r in rates), rates
    assert max(rates) > 0.3, rates   # the noise grows

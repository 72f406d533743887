"""Pins of the oracle's external guide field (a uniform B_0 along the
propagation axis; the paper's conclusion lists external magnetic fields in
its outlook).

A static field along z exerts the force -v x B_0 z^ on an electron: in the
transverse plane it turns u_perp at the cyclotron rate B_0/gamma per unit
time, which is B_0/G per unit xi since d xi/dt = 1 - v_z = G/gamma; with no
wake (G = 1) that is u_perp(xi) = u0 (cos B_0 xi, sin B_0 xi) and the orbit
x(xi) = x0 + (u0/B_0) sin B_0 xi, y(xi) = y0 + (u0/B_0)(1 - cos B_0 xi).  A
beam particle (charge Z, mass M) in the same field turns by the Boris angle
-2 atan(Z B_0 dt/(2 M gamma)) per step, at constant |u|.  Both are fixed here
with the wake made negligible (plasma and beam weights of 1e-13): the closed
forms come from the Lorentz force, not from the oracle's code."""
import math

import numpy as np
import torch

import qsa_workloads as W
from oracle import qsa_pic as O


def _gyrating_plasma(h, nxi, b0, u0):
    g = O.Grid(8, 8, nxi, 0.2, 0.2, h)
    wl = W.small_3d(8, 8, nxi, dx=0.2, dy=0.2, dxi=h, plasma_uth=0.0)
    pl = O.to_torch(W.plasma_template(wl))
    x0, y0 = pl["x"].clone(), pl["y"].clone()
    pl["ux"] = torch.full_like(x0, u0)
    pl["uy"] = torch.zeros_like(x0)
    pl["w"] = 1e-13          # the plasma's own wake is negligible
    src = torch.zeros((4, nxi, 8, 8), dtype=O.F64)
    st = {}
    f = O.slice_sweep(g, pl, src, 3, 0.75, stats=st, b0z=b0)
    x, y, ux, uy = st["plasma"]
    return g, f, x0, y0, x, y, ux, uy


def _orbit_error(h, b0=0.8, u0=0.05, length=6.4):
    nxi = int(round(length / h))
    g, f, x0, y0, x, y, ux, uy = _gyrating_plasma(h, nxi, b0, u0)
    xi = nxi * h
    ph = b0 * xi
    ex = torch.remainder(x0 + (u0 / b0) * math.sin(ph), g.lx)
    ey = torch.remainder(y0 + (u0 / b0) * (1.0 - math.cos(ph)), g.ly)
    dx = torch.remainder(x - ex + 0.5 * g.lx, g.lx) - 0.5 * g.lx
    dy = torch.remainder(y - ey + 0.5 * g.ly, g.ly) - 0.5 * g.ly
    eu = max(float((ux - u0 * math.cos(ph)).abs().max()), float((uy - u0 * math.sin(ph)).abs().max())) / u0
    ep = max(float(dx.abs().max()), float(dy.abs().max())) / (u0 / b0)
    return eu, ep, f


def test_plasma_gyrates_in_the_guide_field_at_second_order():
    e1u, e1p, f = _orbit_error(0.1)
    e2u, e2p, _ = _orbit_error(0.05)
    # the wake stays at the level of the negligible weights
    assert float(f.abs().max()) < 1e-9
    # midpoint-rule phase error: about xi B_0^3 h^2 / 6 = 5.5e-3 here
    assert e1u < 7e-3 and e1p < 7e-3, (e1u, e1p)
    for a, b in ((e1u, e2u), (e1p, e2p)):
        order = math.log2(a / b)
        assert 1.8 <= order <= 2.2, (a, b, order)


def test_guide_field_turns_electrons_counterclockwise():
    # the sense of rotation: an electron moving along +x in B_0 z^ is pushed
    # towards +y (force -v x B = -B_0 (v_y, -v_x, 0))
    _, _, _, _, _, _, ux, uy = _gyrating_plasma(0.05, 4, 0.5, 0.05)
    assert float(uy.min()) > 0.0


def test_beam_turns_by_the_boris_angle_in_the_guide_field():
    b0, dt, n = 0.6, 2.0, 7
    wl = W.small_3d(16, 8, 24, gamma_b=10.0, dt=dt, b0z=b0, seed=11, plasma_uth=0.0,
                    species=(W.Species(Z=-1, alpha=1e-13, ppc=1, sigma_perp=0.05),
                             W.Species(Z=+1, M=3.0, alpha=1e-13, ppc=1, sigma_perp=0.05)))
    beams = W.beam(wl)
    s = O.Sim(wl, W.plasma_template(wl), beams)
    start = [dict(b) for b in s.beams]
    s.beam_step(n)
    for b0_, b1, sp in zip(start, s.beams, wl.species):
        keep = b1["w"] > 0
        u = torch.sqrt(b0_["ux"] ** 2 + b0_["uy"] ** 2 + b0_["uz"] ** 2)
        gam = torch.sqrt(1.0 + u * u)
        phi = -2.0 * torch.atan(sp.Z * b0 * dt / (2.0 * sp.M * gam))
        ang0 = torch.atan2(b0_["uy"], b0_["ux"])
        want_x = torch.sqrt(b0_["ux"] ** 2 + b0_["uy"] ** 2) * torch.cos(ang0 + n * phi)
        want_y = torch.sqrt(b0_["ux"] ** 2 + b0_["uy"] ** 2) * torch.sin(ang0 + n * phi)
        scale = float(torch.sqrt(b0_["ux"] ** 2 + b0_["uy"] ** 2).max())
        assert float((b1["ux"] - want_x)[keep].abs().max()) <= 1e-9 * scale
        assert float((b1["uy"] - want_y)[keep].abs().max()) <= 1e-9 * scale
        assert float((b1["uz"] - b0_["uz"])[keep].abs().max()) <= 1e-9 * float(b0_["uz"].abs().max())


def test_zero_guide_field_changes_nothing():
    wl = W.small_3d(16, 8, 12, seed=5)
    a = O.Sim(wl, W.plasma_template(wl), W.beam(wl))
    b = O.Sim(wl.with_(b0z=0.0), W.plasma_template(wl), W.beam(wl))
    a.beam_step(1)
    b.beam_step(1)
    assert torch.equal(a.sweep(), b.sweep())
    wl2 = wl.with_(b0z=0.3)
    c = O.Sim(wl2, W.plasma_template(wl2), W.beam(wl2))
    c.beam_step(1)
    assert float((c.sweep() - a.fields).abs().max()) > 0.0

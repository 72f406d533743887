"""Pins of the oracle's beam coupling and of E_z, independent of the oracle.

* The beam's four source channels (rho - J_z, J_x, J_y, J_z) of a warm beam
  (u_perp != 0, gamma ~ 10) against a brute-force loop over the nodes of the
  3D linear shape, with 1 - v_z and v = u/gamma taken from their definitions
  in 50-digit decimal arithmetic ("Quasistatic model" section: each beam
  species carries charge Z_s and moves with the common drift; sources of the
  field equations whose linear form is Eqs. (1)-(2)).
* B_z of the first slice for a beam whose transverse current is a single
  transverse mode: lap B_z = d_y J_x - d_x J_y has the closed form
  B_z = -(A/k_y) cos(k_y y) + (A'/k_x) cos(k_x x) for J_x = A sin(k_y y),
  J_y = A' sin(k_x x) (the plasma enters cold, so the beam is the only
  current there).
* E_z = d_xi psi (the quasistatic gauge identity that carries charge
  continuity d_xi(rho - J_z) + div J_perp = 0): the stored E_z against the
  centred xi-difference of the stored psi, and the continuity residual
  itself, converging at second order under joint refinement in the linear
  regime.
* The 3D gather of the Boris push in fields that vary in x, y and xi: the
  linear shape reproduces a trilinear function exactly, so pure-E kicks and
  pure-B rotations follow from the field at the particle in closed form.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
import torch

import qsa_workloads as W
from oracle import qsa_pic as O

F64 = torch.float64


def _hat(d, h, L=None):
    """Linear shape weight of a node at signed distance d (minimum image when
    the axis is periodic with length L)."""
    if L is not None:
        d = (d + 0.5 * L) % L - 0.5 * L
    return max(0.0, 1.0 - abs(d) / h)


# ------------------------------------------------------- beam source channels
def _brute_sources(g, parts):
    """[4, nxi, ny, nx] by a loop over every node and particle; parts: list of
    (Z, x, y, xi, ux, uy, uz, w).  Velocities from 50-digit decimals."""
    getcontext().prec = 50
    out = np.zeros((4, g.nxi, g.ny, g.nx))
    dv = g.dx * g.dy * g.dxi
    for Z, x, y, xi, ux, uy, uz, w in parts:
        U = [Decimal(repr(v)) for v in (ux, uy, uz)]
        gam = (1 + U[0] * U[0] + U[1] * U[1] + U[2] * U[2]).sqrt()
        v = [float(u / gam) for u in U]
        one_m_vz = float(1 - U[2] / gam)
        chan = (one_m_vz, v[0], v[1], v[2])
        for j in range(g.nxi):
            wz = _hat(j * g.dxi - xi, g.dxi)          # no wrap in xi; nodes outside are absent
            if wz == 0.0:
                continue
            for l in range(g.ny):
                wy = _hat(l * g.dy - y, g.dy, g.ly)
                for i in range(g.nx):
                    wx = _hat(i * g.dx - x, g.dx, g.lx)
                    wt = Z * w * wx * wy * wz / dv
                    for c in range(4):
                        out[c, j, l, i] += wt * chan[c]
    return out


def test_beam_sources_brute_force_warm_beam():
    g = O.Grid(6, 5, 4, 0.3, 0.4, 0.25)
    # species 0 (electrons): one particle at the x wrap, one inside; species 1
    # (positrons): one in the last cell row of xi, whose upper xi node (4)
    # lies outside the grid and is dropped
    s0 = [(-1, 0.05, 1.93, 0.10, 1.3, -0.7, 9.5, 0.8),
          (-1, 1.10, 0.50, 0.62, -2.2, 0.4, 12.0, 1.7)]
    s1 = [(+1, 0.90, 0.05, 0.80, 0.6, 2.5, 7.0, 1.1)]

    def spec(ps):
        cols = list(zip(*ps))
        return {k: torch.tensor(cols[i + 1], dtype=F64)
                for i, k in enumerate(("x", "y", "xi", "ux", "uy", "uz", "w"))}

    got = O.beam_sources(g, [spec(s0), spec(s1)], [-1, +1]).numpy()
    ref = _brute_sources(g, s0 + s1)
    for c in range(4):
        scale = np.abs(ref[c]).max()
        assert scale > 0
        assert np.abs(got[c] - ref[c]).max() <= 1e-13 * scale, c
    # the transverse currents are first order in u_perp/gamma and carry the
    # charge sign: the electron particle at the wrap sits alone on node
    # (j=0, l=4, i=0) with a positive u_x, so its J_x there is negative
    assert ref[1, 0, 4, 0] < 0


def test_bz_of_a_single_mode_beam_current():
    nx = ny = 16
    d, h = 0.2, 0.2
    g = O.Grid(nx, ny, 3, d, d, h)
    Lx, Ly = nx * d, ny * d
    kx, ky = 2 * math.pi * 3 / Lx, 2 * math.pi * 2 / Ly
    a, b, gam0, alpha = 0.6, -0.9, 10.0, 0.01
    # one particle per cell at the cell centre, in xi cells 0 and 1; u_x a
    # mode in y, u_y a mode in x, u_z chosen so that every gamma is gam0
    ii, ll, jj = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(2), indexing="ij")
    x = (ii.ravel() + 0.5) * d
    y = (ll.ravel() + 0.5) * d
    xi = (jj.ravel() + 0.5) * h
    ux = a * np.sin(ky * y)
    uy = b * np.sin(kx * x)
    uz = np.sqrt(gam0 ** 2 - 1 - ux ** 2 - uy ** 2)
    w = np.full(x.size, alpha * d * d * h)
    beam = {k: torch.as_tensor(v, dtype=F64) for k, v in
            dict(x=x, y=y, xi=xi, ux=ux, uy=uy, uz=uz, w=w).items()}
    src = O.beam_sources(g, [beam], [-1])
    # node slice 0 takes half of each cell-0 particle; the four particles
    # around a node average a mode sin(k y) to sin(k y_node) cos(k d/2)
    A = -alpha * 0.5 * a * math.cos(ky * d / 2) / gam0
    Ap = -alpha * 0.5 * b * math.cos(kx * d / 2) / gam0
    X, Y = np.meshgrid(np.arange(nx) * d, np.arange(ny) * d)
    assert np.abs(src[1, 0].numpy() - A * np.sin(ky * Y)).max() < 1e-15
    assert np.abs(src[2, 0].numpy() - Ap * np.sin(kx * X)).max() < 1e-15
    wl = W.Workload(name="bzmode", nx=nx, ny=ny, nxi=3, dx=d, dy=d, dxi=h, gamma_b=gam0,
                    species=(W.Species(Z=-1, alpha=alpha, ppc=1),), plasma_mx=2, plasma_my=2)
    plasma = O.to_torch(W.plasma_template(wl))
    f = O.slice_sweep(g, plasma, src)
    bz_ref = -(A / ky) * np.cos(ky * Y) + (Ap / kx) * np.cos(kx * X)
    bz = f[O.BZ, 0].numpy()
    assert np.abs(bz - bz_ref).max() < 1e-13 * np.abs(bz_ref).max()
    # div J_perp = 0 for these modes: E_z has no transverse structure
    ez = f[O.EZ, 0].numpy()
    assert np.abs(ez - ez.mean()).max() < 1e-16


def test_ez_from_jy_manufactured():
    """lap E_z = d_y J_y for J_y a single mode (the y half of div J_perp)."""
    g = O.Grid(16, 8, 1, 0.25, 0.3, 0.1)
    sp = O.Spectral(g)
    x = torch.arange(g.nx, dtype=F64) * g.dx
    y = torch.arange(g.ny, dtype=F64) * g.dy
    X, Y = x[None, :].expand(g.ny, g.nx), y[:, None].expand(g.ny, g.nx)
    kx, ky = 2 * math.pi * 1 / g.lx, 2 * math.pi * 3 / g.ly
    th = kx * X + ky * Y
    k2 = kx * kx + ky * ky
    Jy = torch.cos(th)
    bz, ez = O.solve_bz_ez(sp, torch.zeros_like(Jy, dtype=torch.complex128), torch.fft.fft2(Jy), -0.2)
    assert torch.allclose(ez, ky * torch.sin(th) / k2 - 0.2, atol=1e-14, rtol=0)
    assert torch.allclose(bz, -kx * torch.sin(th) / k2, atol=1e-14, rtol=0)


# ------------------------------------------------- P6: E_z = d_xi psi, continuity
def _p6_residuals(n, L=3.2, xi_len=3.0, alpha=1e-6, eps=0.3):
    h = L / n
    nxi = int(round(xi_len / h)) + 1
    wl = W.Workload(name="p6", nx=n, ny=1, nxi=nxi, dx=L / n, dy=L / n, dxi=h, gamma_b=1000.0,
                    species=(W.Species(Z=-1, alpha=alpha, ppc=8, mod_eps=eps, mod_m=1),),
                    plasma_mx=4, plasma_my=1, beam_loading="lattice", seed=1)
    f = O.Sim(wl, W.plasma_template(wl), W.beam(wl)).sweep()
    psi = f[O.PSI, :, 0, :].numpy()
    ez = f[O.EZ, :, 0, :].numpy()
    dpsi = (psi[2:] - psi[:-2]) / (2 * h)          # centred d_xi psi at slices 1 .. nxi-2
    e = ez[1:-1]
    xis = np.arange(1, nxi - 1) * h
    sel = (xis >= 1.0) & (xis <= xi_len - 0.2)       # behind the head, before the tail
    # transverse structure only (the k = 0 parts follow the leapfrog by construction)
    r = np.fft.rfft(dpsi[sel] - e[sel], axis=1)[:, 1:]
    ref = np.fft.rfft(e[sel], axis=1)[:, 1:]
    k2 = (2 * np.pi * np.arange(1, n // 2 + 1) / L) ** 2
    res_ez = np.linalg.norm(r) / np.linalg.norm(ref)
    # continuity: d_xi S + div J_perp, with S = -lap psi and div J_perp = lap E_z
    res_cont = np.linalg.norm(r * k2) / np.linalg.norm(ref * k2)
    return res_ez, res_cont


def test_ez_is_dxi_psi_and_continuity_converge_at_second_order():
    """Weak seeded mode (alpha = 1e-6): E_z - d_xi psi and the continuity
    residual shrink at order >= 1.8 as h and dx halve together.  (At finite
    amplitude a lattice plasma deposited with the linear shape keeps a floor
    proportional to the amplitude: its density is linear in the particle
    displacements until they cross a node, so the second-order density
    change is missing; that is a property of the discretization, not
    checked here.)"""
    res = [_p6_residuals(n) for n in (16, 32, 64)]
    for k in range(2):
        e = [r[k] for r in res]
        o1, o2 = math.log2(e[0] / e[1]), math.log2(e[1] / e[2])
        assert o1 >= 1.8 and o2 >= 1.8, (k, e)
    assert res[-1][0] < 1e-4 and res[-1][1] < 1e-4, res


# ----------------------------------------------- P8: 3D gather in varying fields
def _node_field(g, fn):
    z = torch.arange(g.nxi, dtype=F64)[:, None, None] * g.dxi
    y = torch.arange(g.ny, dtype=F64)[None, :, None] * g.dy
    x = torch.arange(g.nx, dtype=F64)[None, None, :] * g.dx
    return fn(x, y, z).expand(g.nxi, g.ny, g.nx).clone()


def _trilin(x, y, z):
    return 0.011 + 0.004 * x - 0.006 * y + 0.003 * z + 0.002 * x * y * z


def _one(**kw):
    d = dict(x=1.37, y=1.11, xi=0.95, ux=0.3, uy=-0.2, uz=40.0, w=1.0)
    d.update(kw)
    return {k: torch.tensor([v], dtype=F64) for k, v in d.items()}


def test_boris_gathers_trilinear_fields_exactly():
    g = O.Grid(8, 8, 8, 0.5, 0.4, 0.3)
    dt, Z = 2.0, -1
    b0 = _one()
    xp, yp, zp = 1.37, 1.11, 0.95
    fp = _trilin(xp, yp, zp)
    F = _node_field(g, _trilin)
    # pure E along each axis: u changes by (Z/M) E(x_p) dt exactly
    for slot, comp, sign in ((O.EZ, "uz", 1.0), (O.DXPSI, "ux", -1.0), (O.DYPSI, "uy", -1.0)):
        fields = torch.zeros(7, g.nxi, g.ny, g.nx, dtype=F64)
        fields[slot] = F
        b = O.boris_push(g, b0, Z, 1.0, fields, dt)
        assert float(b[comp]) == pytest.approx(float(b0[comp]) + Z * sign * fp * dt, abs=1e-14), slot
    # pure B_z (varying): |u| kept, rotation in the x-y plane by 2 atan|t|
    fields = torch.zeros(7, g.nxi, g.ny, g.nx, dtype=F64)
    fields[O.BZ] = F
    b = O.boris_push(g, b0, Z, 1.0, fields, dt)
    u0 = np.array([float(b0[k]) for k in ("ux", "uy", "uz")])
    u1 = np.array([float(b[k]) for k in ("ux", "uy", "uz")])
    gam = math.sqrt(1 + (u0 ** 2).sum())
    t = 0.5 * dt * Z * fp / gam
    assert np.linalg.norm(u1) == pytest.approx(np.linalg.norm(u0), rel=1e-15)
    ang = math.atan2(u1[1], u1[0]) - math.atan2(u0[1], u0[0])
    assert ang == pytest.approx(-2 * math.atan(t), abs=1e-13)
    # pure B_y (E_x = -d_x psi + B_y cancelled): rotation in the z-x plane
    fields = torch.zeros(7, g.nxi, g.ny, g.nx, dtype=F64)
    fields[O.BY] = F
    fields[O.DXPSI] = F
    b = O.boris_push(g, b0, Z, 1.0, fields, dt)
    u1 = np.array([float(b[k]) for k in ("ux", "uy", "uz")])
    ang = math.atan2(u1[0], u1[2]) - math.atan2(u0[0], u0[2])
    assert ang == pytest.approx(-2 * math.atan(t), abs=1e-13)
    assert u1[1] == pytest.approx(u0[1], abs=1e-15)
    # pure B_x (E_y = -d_y psi - B_x cancelled): rotation in the y-z plane
    fields = torch.zeros(7, g.nxi, g.ny, g.nx, dtype=F64)
    fields[O.BX] = F
    fields[O.DYPSI] = -F
    b = O.boris_push(g, b0, Z, 1.0, fields, dt)
    u1 = np.array([float(b[k]) for k in ("ux", "uy", "uz")])
    ang = math.atan2(u1[2], u1[1]) - math.atan2(u0[2], u0[1])
    assert ang == pytest.approx(-2 * math.atan(t), abs=1e-13)
    assert u1[0] == pytest.approx(u0[0], abs=1e-15)


def test_boris_gather_drops_nodes_behind_the_grid():
    """In the last cell row of xi only the lower node slice exists: the
    gathered field is (1 - f_xi) times its bilinear value there."""
    g = O.Grid(8, 8, 4, 0.5, 0.4, 0.3)
    F = _node_field(g, _trilin)
    fields = torch.zeros(7, g.nxi, g.ny, g.nx, dtype=F64)
    fields[O.EZ] = F
    zp = 0.98                     # cell 3 (the last node slice), f = 0.98/0.3 - 3
    fz = zp / g.dxi - 3
    b0 = _one(xi=zp, uz=2.0)
    b = O.boris_push(g, b0, -1, 1.0, fields, 1.0)
    ez = (1 - fz) * _trilin(1.37, 1.11, 3 * g.dxi)
    assert float(b["uz"]) == pytest.approx(2.0 - ez, abs=1e-14)

"""Reference QSA particle-in-cell step in float64 on the CPU.

TEST INFRASTRUCTURE ONLY.  This is the oracle: a plain, slow, readable
implementation of what the GPU library computes, used by the tests, by the
package's smoke check and by the benchmark's CPU-baseline leg.  Nothing in
the product path may import it.

Physics (paper, "Quasistatic model" section): plasma electrons (charge -1,
mass 1) over immobile ions, a beam of species s (charge Z_s, mass M_s, density
alpha_s) drifting at v_b ~ c along the propagation axis.  The quasistatic
approximation changes to comoving coordinates (xi, tau) = (ct - z, t) and
treats the plasma/field response as a function of xi at fixed tau, while the
beam evolves slowly in tau.  Normalized units c = omega_p = m_e = e = 1.  The
propagation axis is called z here (the paper's x); the transverse plane is
(x, y); the pseudo-potential psi = phi - A_z equals minus the paper's Psi
(definition after Eq. (2)).

Field equations used (Maxwell's equations in Lorenz gauge with d_t -> d_xi,
d_z -> -d_xi; the linearized forms are the paper's Eqs. (1)-(2)):
  -lap psi = rho - J_z                 E_z = d_xi psi
  lap B_z  = d_y J_x - d_x J_y         lap E_z = div J_perp
  lap B_x  = -d_y J_z - d_xi J_y       lap B_y = d_x J_z + d_xi J_x
  E_x = -d_x psi + B_y,  E_y = -d_y psi - B_x.
A uniform external magnetic field B_0 along the propagation axis (the
guide field of a magnetized plasma, one of the paper's outlook items) adds
to B_z wherever a particle is pushed; it is static and curl-free, so it is
no source of the wake, and it exerts no force along z, so the invariant
below still holds.
Mobile ions (charge Z, mass M in m_e, momenta in units of M c), when the
plasma has them, follow the same equations with G = 1 - (Z/M) psi and the
accelerations scaled by -Z/M, and carry +Z w and Z w u/G.
Plasma electrons conserve gamma - u_z = 1 + psi =: G, so in xi
  dx_perp/dxi = u_perp/G,
  du_x/dxi = gamma d_x psi/G - B_y - u_y B_z/G,
  du_y/dxi = gamma d_y psi/G + B_x + u_x B_z/G,
  gamma = (1 + |u_perp|^2 + G^2)/(2G),
and a macro-particle of weight w contributes -w to rho - J_z and -w u/G to J.

The discretization (the paper defers its code's scheme to a companion
paper) is fixed here and mirrored by the GPU library:
  * periodic transverse grid, nodes x_i = i dx, y_l = l dy; linear
    (cloud-in-cell) shape; cell index floor(x/dx) taken modulo N;
  * spectral solves with the forward FFT unnormalized and the inverse scaled
    by 1/N; every i*k multiplier is zero on that axis's Nyquist index;
    |k|^2 uses the exact wavenumbers; the k = 0 modes of psi and E_z come
    from the transverse-mean equations d_xi <E_z> = -<J_z>, d_xi psi0 = <E_z>
    integrated by leapfrog; B_z(k=0) = 0;
  * B_perp from K fixed-point iterations of the Helmholtz-shifted equations
    (-|k|^2 - kappa^2) B_new = RHS(B_old) - kappa^2 B_old, the xi-derivative
    of J_perp taken as the centred difference of a predicted J_perp at j+1
    and the stored J_perp at j-1.  The predicted J_perp responds to B_perp
    through the push with dD/dB = (3/4) n (the midpoint stage sees
    (3/2) B over a step h, differenced over 2h), so kappa^2 = 3/4 makes the
    iteration's gain (kappa^2 - 3n/4)/(|k|^2 + kappa^2) vanish for unit
    plasma density; K = 3 iterations are taken;
  * the plasma advanced from slice j to j+1 by RK2 (midpoint) with fields
    F^j and the extrapolation F^{j+1/2} = (3F^j - F^{j-1})/2;
  * beam sources from a 3D linear shape in (x, y, xi); the beam advanced in
    tau by a Boris step of length dt in the stored 3D fields.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import torch

F64 = torch.float64
BREAKDOWN_G = 1e-3

# index of each stored field in the [7, nxi, ny, nx] output
PSI, DXPSI, DYPSI, EZ, BX, BY, BZ = range(7)
FIELD_NAMES = ("psi", "dxpsi", "dypsi", "Ez", "Bx", "By", "Bz")


class QSABreakdown(RuntimeError):
    """1 + psi fell to the breakdown threshold: the quasistatic push is invalid."""


@dataclass
class Grid:
    nx: int
    ny: int
    nxi: int
    dx: float
    dy: float
    dxi: float

    @property
    def lx(self) -> float:
        return self.nx * self.dx

    @property
    def ly(self) -> float:
        return self.ny * self.dy

    @property
    def nperp(self) -> int:
        return self.nx * self.ny

    @staticmethod
    def of(wl) -> "Grid":
        return Grid(wl.nx, wl.ny, wl.nxi, wl.dx, wl.dy, wl.dxi)


# ---------------------------------------------------------------------------
# spectral operators
# ---------------------------------------------------------------------------

def _axis_k(n: int, d: float):
    """Wavenumbers 2 pi m/(n d), m in [-n/2, n/2), in FFT order, and the
    derivative multipliers (same, but 0 on the Nyquist index m = -n/2)."""
    m = torch.fft.fftfreq(n, d=1.0 / n, dtype=F64)   # integers in FFT order
    k = 2.0 * math.pi * m / (n * d)
    kd = k.clone()
    if n % 2 == 0 and n > 1:
        kd[n // 2] = 0.0
    return k, kd


class Spectral:
    """k-space multipliers on the [ny, nx] grid."""

    def __init__(self, g: Grid):
        kx, kdx = _axis_k(g.nx, g.dx)
        ky, kdy = _axis_k(g.ny, g.dy)
        self.kdx = kdx[None, :].expand(g.ny, g.nx)
        self.kdy = kdy[:, None].expand(g.ny, g.nx)
        self.ksq = kx[None, :] ** 2 + ky[:, None] ** 2
        self.zero = self.ksq == 0.0
        inv = torch.where(self.zero, torch.zeros_like(self.ksq), 1.0 / torch.where(self.zero, torch.ones_like(self.ksq), self.ksq))
        self.inv_ksq = inv          # 1/|k|^2, 0 at k = 0
        self.n = g.nperp


def fft2(a: torch.Tensor) -> torch.Tensor:
    return torch.fft.fft2(a)


def ifft2r(a: torch.Tensor) -> torch.Tensor:
    return torch.fft.ifft2(a).real


def solve_psi(sp: Spectral, S: torch.Tensor, psi0):
    """-lap psi = S for k != 0; the mean of psi is psi0 (a number or a 0-d
    tensor).  Returns psi, d_x psi, d_y psi."""
    Sh = fft2(S)
    ph = Sh * sp.inv_ksq
    ph = torch.where(sp.zero, (psi0 * sp.n) * torch.ones_like(ph), ph)
    return ifft2r(ph), ifft2r(1j * sp.kdx * ph), ifft2r(1j * sp.kdy * ph)


def solve_bz_ez(sp: Spectral, Jxh: torch.Tensor, Jyh: torch.Tensor, ez0):
    """lap B_z = d_y J_x - d_x J_y and lap E_z = div J_perp for k != 0;
    B_z has zero mean, the mean of E_z is ez0."""
    bzh = -(1j * sp.kdy * Jxh - 1j * sp.kdx * Jyh) * sp.inv_ksq
    ezh = -(1j * sp.kdx * Jxh + 1j * sp.kdy * Jyh) * sp.inv_ksq
    ezh = torch.where(sp.zero, (ez0 * sp.n) * torch.ones_like(ezh), ezh)
    return ifft2r(bzh), ifft2r(ezh)


def helmholtz_bperp(sp: Spectral, Jzh, Dxh, Dyh, Bxh_old, Byh_old, kappa2: float):
    """One fixed-point step for B_perp:
    (-|k|^2 - kappa^2) B_x' = -d_y J_z - D_y - kappa^2 B_x,
    (-|k|^2 - kappa^2) B_y' =  d_x J_z + D_x - kappa^2 B_y  (all in k space)."""
    den = -sp.ksq - kappa2
    bxh = (-1j * sp.kdy * Jzh - Dyh - kappa2 * Bxh_old) / den
    byh = (1j * sp.kdx * Jzh + Dxh - kappa2 * Byh_old) / den
    return bxh, byh


# ---------------------------------------------------------------------------
# particle <-> grid (linear shape, periodic transverse)
# ---------------------------------------------------------------------------

class Stencil2:
    """Four nodes and weights of the linear shape at positions (x, y)."""

    def __init__(self, g: Grid, x: torch.Tensor, y: torch.Tensor):
        gx = x / g.dx
        gy = y / g.dy
        fx0 = torch.floor(gx)
        fy0 = torch.floor(gy)
        fx = gx - fx0
        fy = gy - fy0
        i0 = torch.remainder(fx0.to(torch.int64), g.nx)
        l0 = torch.remainder(fy0.to(torch.int64), g.ny)
        i1 = torch.remainder(i0 + 1, g.nx)
        l1 = torch.remainder(l0 + 1, g.ny)
        self.idx = [l0 * g.nx + i0, l0 * g.nx + i1, l1 * g.nx + i0, l1 * g.nx + i1]
        self.wt = [(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy]
        self.g = g

    def deposit(self, q: torch.Tensor) -> torch.Tensor:
        """Sum_p q_p W(x_node - x_p) / (dx dy) on the [ny, nx] grid."""
        g = self.g
        out = torch.zeros(g.nperp, dtype=F64)
        for idx, wt in zip(self.idx, self.wt):
            out = out.index_add(0, idx, q * wt)
        return out.reshape(g.ny, g.nx) / (g.dx * g.dy)

    def gather(self, F: torch.Tensor) -> torch.Tensor:
        """Sum_nodes F_node W(x_node - x_p)."""
        f = F.reshape(-1)
        acc = None
        for idx, wt in zip(self.idx, self.wt):
            t = f[idx] * wt
            acc = t if acc is None else acc + t
        return acc


def wrap(x: torch.Tensor, L: float) -> torch.Tensor:
    """Periodic wrap into [0, L); a value that rounds to L maps to 0."""
    r = x - L * torch.floor(x / L)
    return torch.where(r >= L, torch.zeros_like(r), r)


# ---------------------------------------------------------------------------
# plasma push in xi
# ---------------------------------------------------------------------------

def _check_g(G: torch.Tensor):
    if bool((G <= BREAKDOWN_G).any()) or not bool(torch.isfinite(G).all()):
        raise QSABreakdown("1 + psi <= %g or non-finite at a plasma particle" % BREAKDOWN_G)


def plasma_rhs(g: Grid, F: Sequence[torch.Tensor], x, y, ux, uy, b0z: float = 0.0, s=1.0):
    """d/dxi of (x, y, u_x, u_y) with the six fields F = (psi, dxpsi, dypsi,
    Bx, By, Bz) gathered at the particle; b0z is a uniform external magnetic
    field along the propagation axis, added to the wake's B_z.  s = -Z/M per
    particle (1 for an electron; a mobile ion of charge Z and mass M has
    G = 1 - (Z/M) psi and its accelerations scaled by -Z/M)."""
    st = Stencil2(g, x, y)
    psi, dxp, dyp, bx, by, bz = (st.gather(f) for f in F)
    bz = bz + b0z
    G = 1.0 + s * psi
    _check_g(G)
    gam = (1.0 + ux * ux + uy * uy + G * G) / (2.0 * G)
    return (ux / G, uy / G,
            s * (gam * dxp / G - by - uy * bz / G),
            s * (gam * dyp / G + bx + ux * bz / G))


def rk2(g: Grid, h: float, Fa, Fb, Y, b0z: float = 0.0, s=1.0):
    """Midpoint rule: Y* = Y + (h/2) f(Y; Fa), Y' = Y + h f(Y*; Fb)."""
    k1 = plasma_rhs(g, Fa, *Y, b0z=b0z, s=s)
    Ys = tuple(a + 0.5 * h * b for a, b in zip(Y, k1))
    k2 = plasma_rhs(g, Fb, *Ys, b0z=b0z, s=s)
    return tuple(a + h * b for a, b in zip(Y, k2))


# ---------------------------------------------------------------------------
# the slice sweep
# ---------------------------------------------------------------------------

def slice_sweep(g: Grid, plasma: Dict, sources: torch.Tensor, n_corr: int = 3,
                kappa2: float = 0.75, stats: Optional[Dict] = None, b0z: float = 0.0,
                ion_z: int = 1, ion_m: float = 0.0) -> torch.Tensor:
    """Quasistatic plasma response to the given beam sources.

    plasma: template dict with x, y, ux, uy (tensors) and w (a scalar or one
    weight per particle); optional "ion": the immobile ions' density at the
    nodes, [ny, nx] (uniform 1 when absent); optional "kind": 1 marks a
    mobile ion of charge ion_z and mass ion_m (in m_e), 0 an electron.
    sources: [4, nxi, ny, nx] beam (rho - J_z, J_x, J_y, J_z).
    b0z: uniform external magnetic field along the propagation axis (it
    enters the plasma push only; the stored B_z is the wake's).
    Returns fields [7, nxi, ny, nx] = psi, d_x psi, d_y psi, E_z, B_x, B_y, B_z.
    """
    sp = Spectral(g)
    h = g.dxi
    shape = (g.ny, g.nx)
    zeros = torch.zeros(shape, dtype=F64)
    out = torch.zeros((7, g.nxi) + shape, dtype=F64)
    x, y = plasma["x"].clone(), plasma["y"].clone()
    ux, uy = plasma["ux"].clone(), plasma["uy"].clone()
    w = plasma["w"]
    kind = plasma.get("kind")
    if kind is not None and ion_m > 0.0:
        mobile = kind > 0
        charge = torch.where(mobile, torch.full_like(x, float(ion_z)), torch.full_like(x, -1.0))
        s = torch.where(mobile, torch.full_like(x, -float(ion_z) / ion_m), torch.ones_like(x))
    else:
        charge = -torch.ones_like(x)
        s = 1.0
    nw = charge * w            # rho - J_z carried by each macro-particle
    ions = plasma.get("ion", 1.0)
    Sb, Jxb, Jyb, Jzb = sources[0], sources[1], sources[2], sources[3]

    e_half = 0.0      # <E_z> at j - 1/2
    psi0 = 0.0        # <psi> at j
    # previous slices (zero ahead of the beam)
    Fm1 = [zeros] * 6       # psi, dxpsi, dypsi, Bx, By, Bz at j-1
    psim2 = zeros           # psi at j-2
    bxm2, bym2 = zeros, zeros
    jxh_m1 = torch.zeros(shape, dtype=torch.complex128)
    jyh_m1 = torch.zeros(shape, dtype=torch.complex128)
    for j in range(g.nxi):
        # -- psi stage ------------------------------------------------------
        st = Stencil2(g, x, y)
        S = st.deposit(nw) + ions + Sb[j]
        psi, dxpsi, dypsi = solve_psi(sp, S, psi0)
        # -- J stage ----------------------------------------------------------
        G = 1.0 + s * st.gather(psi)
        _check_g(G)
        gam = (1.0 + ux * ux + uy * uy + G * G) / (2.0 * G)
        uz = gam - G
        Jx = st.deposit(nw * ux / G) + Jxb[j]
        Jy = st.deposit(nw * uy / G) + Jyb[j]
        Jz = st.deposit(nw * uz / G) + Jzb[j]
        Jxh, Jyh, Jzh = fft2(Jx), fft2(Jy), fft2(Jz)
        # transverse-mean (k = 0) equations, leapfrog in xi
        e_next = e_half - h * Jz.mean()
        ez0 = 0.5 * (e_half + e_next)
        psi0_next = psi0 + h * e_next
        Bz, Ez = solve_bz_ez(sp, Jxh, Jyh, ez0)
        # -- B_perp predictor-corrector --------------------------------------
        Bx = 2.0 * Fm1[3] - bxm2
        By = 2.0 * Fm1[4] - bym2
        bxh, byh = fft2(Bx), fft2(By)
        psi_p1 = 3.0 * psi - 3.0 * Fm1[0] + psim2      # psi extrapolated to j+1
        if j + 1 < g.nxi:
            jxb1, jyb1 = Jxb[j + 1], Jyb[j + 1]
        else:
            jxb1, jyb1 = zeros, zeros
        Y = (x, y, ux, uy)
        for _ in range(n_corr):
            Fj = [psi, dxpsi, dypsi, Bx, By, Bz]
            Fh = [0.5 * (3.0 * a - b) for a, b in zip(Fj, Fm1)]
            xt, yt, uxt, uyt = rk2(g, h, Fj, Fh, Y, b0z, s)
            stt = Stencil2(g, xt, yt)
            Gt = 1.0 + s * stt.gather(psi_p1)
            _check_g(Gt)
            Jxt = stt.deposit(nw * uxt / Gt) + jxb1
            Jyt = stt.deposit(nw * uyt / Gt) + jyb1
            Dxh = (fft2(Jxt) - jxh_m1) / (2.0 * h)
            Dyh = (fft2(Jyt) - jyh_m1) / (2.0 * h)
            bxh, byh = helmholtz_bperp(sp, Jzh, Dxh, Dyh, bxh, byh, kappa2)
            Bx, By = ifft2r(bxh), ifft2r(byh)
        # -- final advance to j+1 ---------------------------------------------
        Fj = [psi, dxpsi, dypsi, Bx, By, Bz]
        Fh = [0.5 * (3.0 * a - b) for a, b in zip(Fj, Fm1)]
        x, y, ux, uy = rk2(g, h, Fj, Fh, Y, b0z, s)
        x = wrap(x, g.lx)
        y = wrap(y, g.ly)
        for f, v in zip((PSI, DXPSI, DYPSI, EZ, BX, BY, BZ),
                        (psi, dxpsi, dypsi, Ez, Bx, By, Bz)):
            out[f, j] = v
        # -- shift history ----------------------------------------------------
        psim2, bxm2, bym2 = Fm1[0], Fm1[3], Fm1[4]
        Fm1 = Fj
        jxh_m1, jyh_m1 = Jxh, Jyh
        e_half, psi0 = e_next, psi0_next
    if stats is not None:
        stats["plasma"] = (x, y, ux, uy)
    return out


# ---------------------------------------------------------------------------
# beam: sources and push
# ---------------------------------------------------------------------------

class Stencil3:
    """Eight nodes and weights of the linear shape in (x, y, xi); xi nodes
    outside [0, nxi-1] are dropped (index -1, weight 0)."""

    def __init__(self, g: Grid, x, y, xi):
        st = Stencil2(g, x, y)
        gz = xi / g.dxi
        fz0 = torch.floor(gz)
        fz = gz - fz0
        j0 = fz0.to(torch.int64)
        j1 = j0 + 1
        self.idx, self.wt = [], []
        for jj, wz in ((j0, 1 - fz), (j1, fz)):
            ok = (jj >= 0) & (jj < g.nxi)
            jc = torch.where(ok, jj, torch.zeros_like(jj))
            for idx2, w2 in zip(st.idx, st.wt):
                self.idx.append(jc * g.nperp + idx2)
                self.wt.append(torch.where(ok, w2 * wz, torch.zeros_like(wz)))
        self.g = g

    def deposit(self, q):
        g = self.g
        out = torch.zeros(g.nxi * g.nperp, dtype=F64)
        for idx, wt in zip(self.idx, self.wt):
            out = out.index_add(0, idx, q * wt)
        return out.reshape(g.nxi, g.ny, g.nx) / (g.dx * g.dy * g.dxi)

    def gather(self, F):
        f = F.reshape(-1)
        acc = None
        for idx, wt in zip(self.idx, self.wt):
            t = f[idx] * wt
            acc = t if acc is None else acc + t
        return acc


def beam_sources(g: Grid, species: Sequence[Dict], Zs: Sequence[int]) -> torch.Tensor:
    """Beam rho - J_z, J_x, J_y, J_z on the [nxi, ny, nx] grid.

    Each particle carries charge Z w; rho - J_z uses 1 - v_z written without
    cancellation as (1 + |u_perp|^2)/(gamma (gamma + u_z))."""
    out = torch.zeros((4, g.nxi, g.ny, g.nx), dtype=F64)
    for b, Z in zip(species, Zs):
        ux, uy, uz = b["ux"], b["uy"], b["uz"]
        gam = torch.sqrt(1.0 + ux * ux + uy * uy + uz * uz)
        one_m_vz = (1.0 + ux * ux + uy * uy) / (gam * (gam + uz))
        q = Z * b["w"]
        st = Stencil3(g, b["x"], b["y"], b["xi"])
        out[0] += st.deposit(q * one_m_vz)
        out[1] += st.deposit(q * ux / gam)
        out[2] += st.deposit(q * uy / gam)
        out[3] += st.deposit(q * uz / gam)
    return out


def boris_push(g: Grid, b: Dict, Z: int, M: float, fields: torch.Tensor, dt: float,
               b0z: float = 0.0) -> Dict:
    """Advance one beam species by dt in the stored 3D fields (Boris 1970).

    E = (-d_x psi + B_y, -d_y psi - B_x, E_z), B = (B_x, B_y, B_z + b0z) from
    the 3D linear shape (zero outside the xi grid) plus the uniform external
    field b0z along the propagation axis.  Positions use the new momentum;
    dxi/dtau = 1 - v_z.  A particle reaching xi >= (nxi-1) dxi leaves the box:
    its weight becomes 0.
    """
    x, y, xi = b["x"], b["y"], b["xi"]
    ux, uy, uz = b["ux"], b["uy"], b["uz"]
    st = Stencil3(g, x, y, xi)
    dxp = st.gather(fields[DXPSI])
    dyp = st.gather(fields[DYPSI])
    ez = st.gather(fields[EZ])
    bx = st.gather(fields[BX])
    by = st.gather(fields[BY])
    bz = st.gather(fields[BZ]) + b0z
    ex = -dxp + by
    ey = -dyp - bx
    qh = (Z / M) * 0.5 * dt
    # half electric kick
    umx, umy, umz = ux + qh * ex, uy + qh * ey, uz + qh * ez
    gm = torch.sqrt(1.0 + umx * umx + umy * umy + umz * umz)
    tx, ty, tz = qh * bx / gm, qh * by / gm, qh * bz / gm
    s = 2.0 / (1.0 + tx * tx + ty * ty + tz * tz)
    sx, sy, sz = s * tx, s * ty, s * tz
    # rotation
    upx = umx + (umy * tz - umz * ty)
    upy = umy + (umz * tx - umx * tz)
    upz = umz + (umx * ty - umy * tx)
    uqx = umx + (upy * sz - upz * sy)
    uqy = umy + (upz * sx - upx * sz)
    uqz = umz + (upx * sy - upy * sx)
    # second half kick
    nux, nuy, nuz = uqx + qh * ex, uqy + qh * ey, uqz + qh * ez
    gam = torch.sqrt(1.0 + nux * nux + nuy * nuy + nuz * nuz)
    nx_ = wrap(x + dt * nux / gam, g.lx)
    ny_ = wrap(y + dt * nuy / gam, g.ly)
    nxi = xi + dt * (1.0 + nux * nux + nuy * nuy) / (gam * (gam + nuz))
    lost = nxi >= (g.nxi - 1) * g.dxi
    w = torch.where(lost, torch.zeros_like(b["w"]), b["w"])
    out = dict(b)
    out.update(x=nx_, y=ny_, xi=nxi, ux=nux, uy=nuy, uz=nuz, w=w)
    return out


# ---------------------------------------------------------------------------
# drivers
# ---------------------------------------------------------------------------

def to_torch(d: Dict) -> Dict:
    out = {}
    for k, v in d.items():
        if isinstance(v, float):
            out[k] = v
        elif k == "bin":
            out[k] = torch.as_tensor(v, dtype=torch.int64)
        else:
            out[k] = torch.as_tensor(v, dtype=F64)
    return out


class Sim:
    """A whole run: plasma template + beam species + the scheme's constants."""

    def __init__(self, wl, plasma: Dict, beams: List[Dict]):
        self.wl = wl
        self.g = Grid.of(wl)
        self.plasma = to_torch(plasma)
        self.beams = [to_torch(b) for b in beams]
        self.Z = [s.Z for s in wl.species]
        self.M = [s.M for s in wl.species]
        self.b0z = float(getattr(wl, "b0z", 0.0))
        self.fields = None

    def sweep(self) -> torch.Tensor:
        src = beam_sources(self.g, self.beams, self.Z)
        self.fields = slice_sweep(self.g, self.plasma, src, self.wl.n_corr, self.wl.kappa2, b0z=self.b0z,
                                  ion_z=int(getattr(self.wl, "ion_z", 1)),
                                  ion_m=float(getattr(self.wl, "ion_m", 0.0)))
        return self.fields

    def push(self):
        self.beams = [boris_push(self.g, b, Z, M, self.fields, self.wl.dt, self.b0z)
                      for b, Z, M in zip(self.beams, self.Z, self.M)]

    def beam_step(self, n: int = 1):
        """n x (sweep at tau_n; push to tau_{n+1})."""
        for _ in range(n):
            self.sweep()
            self.push()


def ex_ey(fields: torch.Tensor):
    """E_x = -d_x psi + B_y and E_y = -d_y psi - B_x from stored fields."""
    return -fields[DXPSI] + fields[BY], -fields[DYPSI] - fields[BX]


def output_fields(fields: torch.Tensor) -> Dict[str, torch.Tensor]:
    """The seven output fields psi, E_x, E_y, E_z, B_x, B_y, B_z."""
    ex, ey = ex_ey(fields)
    return {"psi": fields[PSI], "Ex": ex, "Ey": ey, "Ez": fields[EZ],
            "Bx": fields[BX], "By": fields[BY], "Bz": fields[BZ]}

"""Workload descriptions for the QSA particle-in-cell slice sweep.

Pure data: grid sizes, spacings, beam species and loading recipes, in the
paper's normalized units (lengths in c/omega_p, times in 1/omega_p, densities
in n_p, momenta u = p/(M m_e c)).  The problem statement (cold or warm plasma
electrons over immobile ions, beam species of charge Z e, mass M m_e and
density ratio alpha = n_b/n_p with a common Lorentz factor gamma_b) follows the
"Quasistatic model" section of the paper; the beams are flat-top in xi from the
leading edge xi = 0, transversely periodic, open in xi, as in its
"PIC simulations" section.

Nothing here computes any part of the method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Tuple


@dataclass(frozen=True)
class Species:
    """One beam species.

    Z: charge number (electron -1, positron +1); M: mass in m_e;
    alpha: n_b/n_p; ppc: macro-particles per 3D cell (per (x, xi) cell in a slab);
    sigma_par / sigma_perp: Gaussian momentum spread relative to gamma_b*beta_b;
    mod_eps, mod_m: optional weight modulation (1 + mod_eps*cos(2 pi mod_m x / Lx))
    used to seed a single transverse mode;
    w_spread: random macro-particle weights, each weight times
    (1 + w_spread (2U - 1)) with U uniform in [0, 1) (mean unchanged);
    ramp_head, ramp_tail: a longitudinal density profile instead of the flat
    top: the density rises linearly from 0 at the head (xi = 0) to its
    plateau over ramp_head, and falls linearly to 0 over the last ramp_tail
    of the beam (lengths in c/omega_p; 0 = a sharp edge).
    """
    Z: int = -1
    M: float = 1.0
    alpha: float = 0.1
    ppc: int = 8
    sigma_par: float = 0.0
    sigma_perp: float = 0.0
    mod_eps: float = 0.0
    mod_m: int = 0
    w_spread: float = 0.0
    ramp_head: float = 0.0
    ramp_tail: float = 0.0


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int                  # 1 = slab (x, xi)
    nxi: int
    dx: float
    dy: float
    dxi: float
    gamma_b: float
    species: Tuple[Species, ...]
    plasma_mx: int = 2       # plasma lattice per cell along x
    plasma_my: int = 2       # ... along y (1 in a slab)
    plasma_uth: float = 0.0  # thermal spread of u_x, u_y (0 = cold)
    plasma_w_spread: float = 0.0  # random plasma weights: w0 (1 + spread (2U - 1)), 0 = all w0
    plasma_n0: float = 1.0   # plasma density profile n0 (1 + mod cos(2 pi (mod_mx x/Lx + mod_my y/Ly)))
    plasma_mod: float = 0.0
    plasma_mod_mx: int = 0
    plasma_mod_my: int = 0
    dt: float = 5.0          # beam time step
    steps: int = 1
    seed: int = 0
    beam_loading: str = "random"   # "random" (uniform in each cell) or "lattice"
    n_corr: int = 3          # predictor-corrector iterations for B_perp
    kappa2: float = 0.75     # Helmholtz shift of the B_perp iteration (3/4: see oracle)
    precision: str = "f64"
    n_bins: int = 0          # piecewise-constant xi amplitude bins (adjoint workload)
    ckpt_every: int = 16
    b0z: float = 0.0         # uniform external magnetic field along the propagation axis (guide field)
    ion_m: float = 0.0       # mass of mobile plasma ions in m_e (0: immobile ion background)
    ion_z: int = 1           # their charge number

    # derived sizes -------------------------------------------------------
    @property
    def beta_b(self) -> float:
        return math.sqrt(1.0 - 1.0 / (self.gamma_b * self.gamma_b))

    @property
    def n_perp(self) -> int:
        return self.nx * self.ny

    @property
    def plasma_ppc(self) -> int:
        return self.plasma_mx * self.plasma_my

    @property
    def n_plasma(self) -> int:
        """Plasma macro-particles per slice (electrons, and as many mobile
        ions when ion_m > 0)."""
        return self.n_perp * self.plasma_ppc * (2 if self.ion_m > 0.0 else 1)

    @property
    def beam_slices(self) -> int:
        """Beam cells along xi: the flat top covers [0, (nxi-1)*dxi)."""
        return self.nxi - 1

    def n_beam(self, s: int) -> int:
        return self.n_perp * self.beam_slices * self.species[s].ppc

    @property
    def n_beam_total(self) -> int:
        return sum(self.n_beam(s) for s in range(len(self.species)))

    @property
    def updates_per_sweep(self) -> int:
        """Plasma particle-slice updates in one sweep."""
        return self.n_plasma * self.nxi

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# ---------------------------------------------------------------------------
# The five workloads the build is measured on (synthetic stand-ins for the
# paper's runs; see the design notes for the recipe and the readings).
# ---------------------------------------------------------------------------

def slab_electron() -> Workload:
    """2D slab (x, xi): 64 x 128, dx = dxi = 0.1; e- beam alpha 0.1, gamma 100."""
    return Workload(
        name="slab64x128_e", nx=64, ny=1, nxi=128, dx=0.1, dy=0.1, dxi=0.1,
        gamma_b=100.0,
        species=(Species(Z=-1, M=1.0, alpha=0.1, ppc=8, sigma_par=1e-3),),
        plasma_mx=4, plasma_my=1, plasma_uth=0.0, dt=5.0, steps=50, seed=1001,
        precision="f64")


def slab_pair(seeded_mode: bool = False, m: int = 5, eps: float = 1e-3) -> Workload:
    """Pair-beam variant of the slab workload (e- and e+ at alpha = 0.05 each).

    With seeded_mode the beam is lattice-loaded and the two species' weights
    are counter-modulated at transverse mode m, so that the only seed is a
    single current-filamentation mode.
    """
    if seeded_mode:
        sp = (Species(Z=-1, M=1.0, alpha=0.05, ppc=8, mod_eps=eps, mod_m=m),
              Species(Z=+1, M=1.0, alpha=0.05, ppc=8, mod_eps=-eps, mod_m=m))
        loading = "lattice"
    else:
        sp = (Species(Z=-1, M=1.0, alpha=0.05, ppc=8, sigma_par=1e-3),
              Species(Z=+1, M=1.0, alpha=0.05, ppc=8, sigma_par=1e-3))
        loading = "random"
    return Workload(
        name="slab64x128_pair" + ("_mode" if seeded_mode else ""), nx=64, ny=1,
        nxi=128, dx=0.1, dy=0.1, dxi=0.1, gamma_b=100.0, species=sp,
        plasma_mx=4, plasma_my=1, dt=5.0, steps=50, seed=1101,
        beam_loading=loading, precision="f64")


def cube256() -> Workload:
    """3D 256 x 256 x 512, dx = dy = dxi = 0.05; warm plasma; e- beam alpha 1e-2, gamma 1e3."""
    return Workload(
        name="3d256x256x512_e", nx=256, ny=256, nxi=512, dx=0.05, dy=0.05,
        dxi=0.05, gamma_b=1e3,
        species=(Species(Z=-1, M=1.0, alpha=1e-2, ppc=8),),
        plasma_mx=2, plasma_my=2, plasma_uth=0.01, dt=20.0, steps=200, seed=2002,
        precision="f64")


def pair512() -> Workload:
    """3D dilute pair beam 512 x 512 x 2048, dx = 0.1; alpha 1e-4 each, gamma 1e4."""
    return Workload(
        name="3d512x512x2048_pair", nx=512, ny=512, nxi=2048, dx=0.1, dy=0.1,
        dxi=0.1, gamma_b=1e4,
        species=(Species(Z=-1, M=1.0, alpha=1e-4, ppc=4, sigma_perp=1e-4),
                 Species(Z=+1, M=1.0, alpha=1e-4, ppc=4, sigma_perp=1e-4)),
        plasma_mx=2, plasma_my=2, plasma_uth=1e-3, dt=100.0, steps=500, seed=3003,
        precision="f32")


def adjoint128() -> Workload:
    """3D 128 x 128 x 256, dx = dy = dxi = 0.1, loading of the slab workload; 64 xi bins."""
    return Workload(
        name="3d128x128x256_e_adjoint", nx=128, ny=128, nxi=256, dx=0.1, dy=0.1,
        dxi=0.1, gamma_b=100.0,
        species=(Species(Z=-1, M=1.0, alpha=0.1, ppc=8, sigma_par=1e-3),),
        plasma_mx=2, plasma_my=2, dt=5.0, steps=20, seed=5005, precision="f32",
        n_bins=64, ckpt_every=16)


def scan_instances(n_inst: int = 64, seed: int = 4004):
    """Batched parameter scan: n_inst independent 3D instances.

    Nx, Ny iid uniform on {64, 128, 256}; Nxi uniform on {128, 256, 512, 1024};
    alpha = 10**U(-4, -1); gamma_b = 10**U(1, 4); dx = dy = dxi = 0.1, 2x2 cold
    plasma lattice, 8-ppc e- beam with sigma_par = 1e-3; dt = 0.16/omega_b.
    """
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_inst):
        nx = int(rng.choice([64, 128, 256]))
        ny = int(rng.choice([64, 128, 256]))
        nxi = int(rng.choice([128, 256, 512, 1024]))
        alpha = float(10.0 ** rng.uniform(-4.0, -1.0))
        gamma = float(10.0 ** rng.uniform(1.0, 4.0))
        omega_b = math.sqrt(alpha / gamma)
        out.append(Workload(
            name=f"scan{i:02d}", nx=nx, ny=ny, nxi=nxi, dx=0.1, dy=0.1, dxi=0.1,
            gamma_b=gamma,
            species=(Species(Z=-1, M=1.0, alpha=alpha, ppc=8, sigma_par=1e-3),),
            plasma_mx=2, plasma_my=2, dt=0.16 / omega_b, steps=100,
            seed=40000 + i, precision="f32"))
    return out


def small_3d(nx: int = 32, ny: int = 32, nxi: int = 24, **kw) -> Workload:
    """A small 3D case of the cube workload's loading, for quick checks."""
    base = dict(
        name=f"3d{nx}x{ny}x{nxi}_e", nx=nx, ny=ny, nxi=nxi, dx=0.1, dy=0.1,
        dxi=0.1, gamma_b=100.0,
        species=(Species(Z=-1, M=1.0, alpha=0.05, ppc=2, sigma_par=1e-3,
                         sigma_perp=1e-3),),
        plasma_mx=2, plasma_my=2, plasma_uth=0.01, dt=5.0, steps=1, seed=7)
    base.update(kw)
    return Workload(**base)


CONFIGS = {
    "slab": slab_electron,
    "slab_pair": slab_pair,
    "cube256": cube256,
    "pair512": pair512,
    "adjoint128": adjoint128,
}

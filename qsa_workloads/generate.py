"""Seeded synthetic inputs: the plasma template and the beam particles.

Every random number of a run is drawn here, with NumPy's PCG64, and handed to
both implementations as plain float64 arrays; neither implementation draws
random numbers of its own.  This module holds no arithmetic of the method:
it only places particles in cells and draws momenta.

Streams are split so that any range of xi slices can be generated alone and
bit-identically: the beam particles of slice j of species s come from
PCG64(SeedSequence([seed, 1 + s, j])); the plasma thermal draws from
PCG64(SeedSequence([seed, 0])).
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np

from .configs import Workload


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def plasma_template(wl: Workload) -> Dict[str, np.ndarray]:
    """Plasma macro-particles entering the box at xi = 0.

    A plasma_mx x plasma_my lattice per transverse cell at
    x = (i + (a + 1/2)/mx) dx, y = (l + (b + 1/2)/my) dy, ordered by cell
    (row l, column i) then lattice site; all weights dx*dy/ppc (unit density),
    or, with plasma_w_spread > 0, an array of random macro-particle weights
    dx*dy/ppc (1 + spread (2U - 1)), U uniform on [0, 1) from a stream of its
    own.  With a density profile (plasma_n0 != 1 or plasma_mod != 0) every
    weight is also multiplied by n(x_p, y_p) and "ion" holds the immobile
    ions' density at the nodes, [ny, nx].  With mobile ions (ion_m > 0) the
    template holds the electrons, then as many ions on the same sites ("kind"
    1, weights divided by the charge number ion_z), and "ion" is zero.  Cold
    (u = 0) or u_x, u_y ~ N(0, u_th^2).
    """
    mx, my = wl.plasma_mx, wl.plasma_my
    ii = np.arange(wl.nx)
    ll = np.arange(wl.ny)
    aa = (np.arange(mx) + 0.5) / mx
    bb = (np.arange(my) + 0.5) / my
    # order: l, i, b, a
    L, I, B, A = np.meshgrid(ll, ii, bb, aa, indexing="ij")
    x = ((I + A) * wl.dx).reshape(-1)
    y = ((L + B) * wl.dy).reshape(-1)
    n = x.size
    if wl.plasma_uth > 0.0:
        g = _rng(wl.seed, 0)
        u = wl.plasma_uth * g.standard_normal((2, n))
        ux, uy = u[0].copy(), u[1].copy()
    else:
        ux = np.zeros(n)
        uy = np.zeros(n)
    w = wl.dx * wl.dy / (mx * my)
    profiled = wl.plasma_n0 != 1.0 or wl.plasma_mod != 0.0
    mobile = wl.ion_m > 0.0
    if wl.plasma_w_spread > 0.0:
        gw = _rng(wl.seed, 0, 1)
        wa = w * (1.0 + wl.plasma_w_spread * (2.0 * gw.random(n) - 1.0))
    elif profiled or mobile:
        wa = np.full(n, w)
    else:
        return {"x": x, "y": y, "ux": ux, "uy": uy, "w": float(w)}
    out = {"x": x, "y": y, "ux": ux, "uy": uy, "w": wa}
    xn, yn = np.meshgrid(ii * wl.dx, ll * wl.dy)   # [ny, nx] nodes
    if profiled:
        out["w"] = wa * plasma_density(wl, x, y)
        out["ion"] = plasma_density(wl, xn, yn)
    if mobile:
        # mobile ions on the electrons' lattice sites, 1/Z of their number
        # (neutral), thermal momenta at the electrons' temperature
        # (u = p/(M c): spread u_th/sqrt(M)); no immobile background
        if wl.plasma_uth > 0.0:
            ui = (wl.plasma_uth / np.sqrt(wl.ion_m)) * _rng(wl.seed, 0, 2).standard_normal((2, n))
        else:
            ui = np.zeros((2, n))
        out = {"x": np.concatenate([x, x]), "y": np.concatenate([y, y]),
               "ux": np.concatenate([ux, ui[0]]), "uy": np.concatenate([uy, ui[1]]),
               "w": np.concatenate([out["w"], out["w"] / wl.ion_z]),
               "kind": np.concatenate([np.zeros(n, np.int32), np.ones(n, np.int32)]),
               "ion": np.zeros(xn.shape)}
    return out


def plasma_density(wl: Workload, x, y):
    """The plasma's density profile n(x, y) = n0 (1 + a cos(2 pi (mx x/Lx +
    my y/Ly))) in units of the reference density (the paper's outlook item
    of plasma inhomogeneity; uniform n = 1 by default).  The electrons carry
    it in their weights and the immobile ions match it at the nodes, so the
    plasma enters the box neutral."""
    lx, ly = wl.nx * wl.dx, wl.ny * wl.dy
    ph = 2.0 * np.pi * (wl.plasma_mod_mx * np.asarray(x) / lx + wl.plasma_mod_my * np.asarray(y) / ly)
    return wl.plasma_n0 * (1.0 + wl.plasma_mod * np.cos(ph))


def beam_species(wl: Workload, s: int, j0: int = 0, j1: Optional[int] = None,
                 ) -> Dict[str, np.ndarray]:
    """Particles of beam species s in xi-cells [j0, j1) (default: the whole beam).

    Flat-top beam over xi in [0, (nxi-1) dxi), uniform transversely.  Per cell,
    ppc particles either uniformly random in the cell ("random") or on a
    regular sub-lattice ("lattice", ppc = mx*my*mxi chosen as the most even
    split).  Order: slice j, row l, column i, then particle.  Momenta
    u_z = gamma_b beta_b (1 + sigma_par N), u_perp = gamma_b beta_b sigma_perp N.
    Weight alpha dx dy dxi / ppc, times (1 + eps cos(2 pi m x / Lx)) when a
    mode is seeded, and times (1 + w_spread (2U - 1)) for random weights
    (U from a stream of its own per species and slice).  Also returns the cell-independent 'bin' index (-1 if no
    bins) that the adjoint workload uses.
    """
    sp = wl.species[s]
    if j1 is None:
        j1 = wl.beam_slices
    j1 = min(j1, wl.beam_slices)
    ppc = sp.ppc
    ncell = wl.nx * wl.ny
    n_slice = ncell * ppc
    nsl = max(j1 - j0, 0)
    n = n_slice * nsl
    out = {k: np.empty(n) for k in ("x", "y", "xi", "ux", "uy", "uz", "w")}
    gb = wl.gamma_b * wl.beta_b
    w0 = sp.alpha * wl.dx * wl.dy * wl.dxi / ppc
    cell = np.repeat(np.arange(ncell), ppc)
    ci = (cell % wl.nx).astype(np.float64)
    cl = (cell // wl.nx).astype(np.float64)
    if wl.beam_loading == "lattice":
        sub = _lattice_offsets(ppc, wl.ny > 1)
        sub = np.tile(sub, (ncell, 1))
    for jj in range(nsl):
        j = j0 + jj
        sl = slice(jj * n_slice, (jj + 1) * n_slice)
        if wl.beam_loading == "lattice":
            U = sub.T
            g = None
        else:
            g = _rng(wl.seed, 1 + s, j)
            U = g.random((3, n_slice))
        x = (ci + U[0]) * wl.dx
        out["x"][sl] = x
        out["y"][sl] = (cl + U[1]) * wl.dy
        out["xi"][sl] = (j + U[2]) * wl.dxi
        if sp.sigma_par > 0.0 and g is not None:
            out["uz"][sl] = gb * (1.0 + sp.sigma_par * g.standard_normal(n_slice))
        else:
            out["uz"][sl] = gb
        if sp.sigma_perp > 0.0 and g is not None:
            up = gb * sp.sigma_perp * g.standard_normal((2, n_slice))
            out["ux"][sl] = up[0]
            out["uy"][sl] = up[1] if wl.ny > 1 else 0.0
        else:
            out["ux"][sl] = 0.0
            out["uy"][sl] = 0.0
        if sp.mod_eps != 0.0:
            lx = wl.nx * wl.dx
            out["w"][sl] = w0 * (1.0 + sp.mod_eps * np.cos(2.0 * math.pi * sp.mod_m * x / lx))
        else:
            out["w"][sl] = w0
        if sp.w_spread > 0.0:
            gw = _rng(wl.seed, 100 + s, j)
            out["w"][sl] *= 1.0 + sp.w_spread * (2.0 * gw.random(n_slice) - 1.0)
        if sp.ramp_head > 0.0 or sp.ramp_tail > 0.0:
            out["w"][sl] *= longitudinal_profile(wl, s, out["xi"][sl])
    if wl.n_bins > 0:
        extent = wl.beam_slices * wl.dxi
        b = np.floor(out["xi"] / (extent / wl.n_bins)).astype(np.int32)
        out["bin"] = np.clip(b, 0, wl.n_bins - 1)
    return out


def longitudinal_profile(wl: Workload, s: int, xi) -> np.ndarray:
    """Beam density of species s at xi relative to its plateau: linear from
    0 at xi = 0 to 1 at ramp_head, 1 on the plateau, linear from 1 to 0 over
    the last ramp_tail before the beam's end (beam_slices * dxi)."""
    sp = wl.species[s]
    xi = np.asarray(xi, dtype=np.float64)
    end = wl.beam_slices * wl.dxi
    f = np.ones_like(xi)
    if sp.ramp_head > 0.0:
        f = np.minimum(f, xi / sp.ramp_head)
    if sp.ramp_tail > 0.0:
        f = np.minimum(f, (end - xi) / sp.ramp_tail)
    return np.clip(f, 0.0, 1.0)


def _lattice_offsets(ppc: int, three_d: bool) -> np.ndarray:
    """Regular sub-cell offsets in [0,1)^3 for ppc particles (x, y, xi)."""
    if three_d:
        # split ppc into mx*my*mxi with mx >= my >= mxi as even as possible
        best = None
        for mx in range(1, ppc + 1):
            if ppc % mx:
                continue
            for my in range(1, ppc // mx + 1):
                if (ppc // mx) % my:
                    continue
                mxi = ppc // mx // my
                key = max(mx, my, mxi)
                if best is None or key < best[0]:
                    best = (key, mx, my, mxi)
        _, mx, my, mxi = best
    else:
        # slab: particles spread along x and xi only
        mxi = 1
        for d in range(int(math.isqrt(ppc)), 0, -1):
            if ppc % d == 0:
                mxi = d
                break
        mx, my = ppc // mxi, 1
    a = (np.arange(mx) + 0.5) / mx
    b = (np.arange(my) + 0.5) / my
    c = (np.arange(mxi) + 0.5) / mxi
    C, B, A = np.meshgrid(c, b, a, indexing="ij")
    return np.stack([A.reshape(-1), B.reshape(-1), C.reshape(-1)], axis=1)


def beam(wl: Workload, j0: int = 0, j1: Optional[int] = None):
    """All species: a list of dicts (see beam_species)."""
    return [beam_species(wl, s, j0, j1) for s in range(len(wl.species))]

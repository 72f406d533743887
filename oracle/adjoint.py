"""Reference gradient of the transverse magnetic field energy with respect to
piecewise-constant beam-amplitude bins, in float64 on the CPU.

TEST INFRASTRUCTURE ONLY (see oracle/qsa_pic.py).

The objective is the total transverse magnetic energy of the sweep after
n beam steps, L = 1/2 sum (B_x^2 + B_y^2) dx dy dxi over every node of every
slice.  Beam particle p of bin b carries weight w_p a_b (w_p as loaded, bin
membership fixed by the particle's xi at loading).  The gradient is the exact
derivative of the discrete scheme of qsa_pic (every sweep, every deposit and
every Boris push), obtained by reverse-mode automatic differentiation of that
very code: it is the adjoint of the discretization, not of the continuous
equations.  Floors of cell indices and the loss flag are piecewise constant
and contribute nothing.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

from . import qsa_pic as O


def field_energy(g: O.Grid, fields: torch.Tensor) -> torch.Tensor:
    """1/2 sum (B_x^2 + B_y^2) dV over the [7, nxi, ny, nx] fields."""
    return 0.5 * (fields[O.BX].pow(2).sum() + fields[O.BY].pow(2).sum()) * (g.dx * g.dy * g.dxi)


def run_energy(wl, plasma: Dict, beams: List[Dict], n_steps: int, amps: torch.Tensor) -> torch.Tensor:
    """The objective as a function of the bin amplitudes (differentiable)."""
    g = O.Grid.of(wl)
    pl = O.to_torch(plasma)
    bs = []
    for b in beams:
        t = O.to_torch(b)
        t["w"] = t["w"] * amps[t["bin"].long()]
        bs.append(t)
    Z = [s.Z for s in wl.species]
    M = [s.M for s in wl.species]
    fields = None
    for n in range(n_steps + 1):
        src = O.beam_sources(g, bs, Z)
        fields = O.slice_sweep(g, pl, src, wl.n_corr, wl.kappa2)
        if n < n_steps:
            bs = [O.boris_push(g, b, z, m, fields, wl.dt) for b, z, m in zip(bs, Z, M)]
    return field_energy(g, fields)


def energy_and_gradient(wl, plasma: Dict, beams: List[Dict], n_steps: int,
                        amps: Sequence[float]) -> Tuple[float, np.ndarray]:
    """L(a) and dL/da_b by reverse-mode differentiation of the scheme."""
    a = torch.tensor(np.asarray(amps, dtype=np.float64), requires_grad=True)
    L = run_energy(wl, plasma, beams, n_steps, a)
    L.backward()
    return float(L.detach()), a.grad.detach().numpy().copy()


def energy(wl, plasma: Dict, beams: List[Dict], n_steps: int, amps: Sequence[float]) -> float:
    with torch.no_grad():
        return float(run_energy(wl, plasma, beams, n_steps,
                                torch.tensor(np.asarray(amps, dtype=np.float64))))

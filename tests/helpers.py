"""Shared test helpers: run a workload through the oracle and through the
HIP library on the same seeded inputs, and compare slice by slice."""
from __future__ import annotations

import numpy as np

import qsa_workloads as W

OUT_FIELDS = ("psi", "Ex", "Ey", "Ez", "Bx", "By", "Bz")


def oracle_fields(sim_o):
    from oracle import qsa_pic as O
    of = O.output_fields(sim_o.fields)
    return {k: v.numpy() for k, v in of.items()}


def run_oracle(wl, steps: int = 0, beams=None, plasma=None):
    from oracle import qsa_pic as O
    plasma = plasma if plasma is not None else W.plasma_template(wl)
    beams = beams if beams is not None else W.beam(wl)
    s = O.Sim(wl, plasma, beams)
    if steps:
        s.beam_step(steps)
    s.sweep()
    return s, oracle_fields(s)


def run_gpu(wl, steps: int = 0, precision=None, beams=None, plasma=None):
    import paper_2607_24214_amd as Q
    plasma = plasma if plasma is not None else W.plasma_template(wl)
    beams = beams if beams is not None else W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    sim = Q.Sim(Q.params_from_workload(wl, precision=precision, beam_capacity=caps))
    sim.load_plasma(plasma)
    for s, b in enumerate(beams):
        sim.load_beam(s, b)
    if steps:
        sim.beam_step(steps)
    sim.slice_sweep()
    out = {k: sim.fields(k) for k in OUT_FIELDS}
    return sim, out


def slice_errors(got: dict, ref: dict, j0: int = 0, j1=None, floor: float = 0.0):
    """Per slice and field: ||got - ref||_2 / max_f ||ref_f||_2 over the slice
    (the scale is the largest field of that slice, so that fields that are
    identically zero in a geometry are judged on an absolute scale; it is
    raised to `floor` where a slice's fields are weaker, so that a slice
    whose fields sit at rounding level is judged on the box's scale).
    Returns (max error, worst (field, slice))."""
    names = list(ref.keys())
    nxi = ref[names[0]].shape[0]
    j1 = nxi if j1 is None else j1
    worst, where = 0.0, None
    for j in range(j0, j1):
        scale = max(max(float(np.linalg.norm(ref[f][j])) for f in names), floor)
        if scale == 0.0:
            scale = 1.0
        for f in names:
            e = float(np.linalg.norm(got[f][j] - ref[f][j])) / scale
            if e > worst:
                worst, where = e, (f, j)
    return worst, where


def psi_floor(wl, precision):
    """Rounding floor of the L2 norm of psi on one slice.  A CIC weight is
    known to eps_w: float64 weights come from absolute positions, so
    eps_w = eps_64 n_x (positions up to n_x cells, resolved to eps_64 of
    their value); float32 weights are rounded to eps_32.  Independent
    errors of that size in the deposited source, carried through the
    inverse Laplacian, give ||d psi||_2 ~ eps_w (L/2 pi)^2 (sum over
    m != 0 of |m|^-4)^(1/2), the sum about 6."""
    L = max(wl.nx * wl.dx, wl.ny * wl.dy)
    eps_w = np.finfo(np.float64).eps * max(wl.nx, wl.ny) if precision == "f64" else np.finfo(np.float32).eps
    return eps_w * (L / (2.0 * np.pi)) ** 2 * np.sqrt(6.0)


def scale_floor(*refs, frac: float = 1e-3):
    """frac times the largest per-slice field scale (max_f ||F_f||_2 over a
    slice) found in the given field dicts: the smallest scale a slice is
    judged on when the one-ulp rule compares two runs."""
    s = 0.0
    for ref in refs:
        names = list(ref.keys())
        for j in range(ref[names[0]].shape[0]):
            s = max(s, max(float(np.linalg.norm(ref[f][j])) for f in names))
    return frac * s


def matched_kappa2(wl) -> float:
    """Helmholtz shift of the B_perp iteration matched to the plasma: the
    predicted current responds to B_perp with (3/4) n_eff, n_eff = sum over
    the plasma species of Z^2 n/M (electrons at the mean density, plus
    mobile ions of charge Z and mass M at 1/Z of it), so kappa^2 = 3 n_eff/4
    zeroes the iteration's gain at k = 0 (3/4 for the unit-density plasma
    of the benchmark workloads)."""
    n0 = getattr(wl, "plasma_n0", 1.0)
    n_eff = n0
    if getattr(wl, "ion_m", 0.0) > 0.0:
        n_eff += wl.ion_z * n0 / wl.ion_m
    return 0.75 * n_eff

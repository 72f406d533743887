"""A beam loaded in parts (qsa_load_beam_range, the way the benchmark loads
the 4.3e9-particle pair beam) equals the same beam loaded at once: the same
particles read back in load order and the same fields and beam after steps,
one at a time and with steps in flight; host and device parts; the order
rules (a part starts the beam or appends to it) and the capacity bound."""
import numpy as np
import pytest
import torch

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, slice_errors

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "xi", "ux", "uy", "uz", "w")


def _sim(wl, pipeline=1, caps=None):
    import paper_2607_24214_amd as Q
    caps = caps or [wl.n_beam(s) for s in range(len(wl.species))]
    s = Q.Sim(Q.params_from_workload(wl, beam_capacity=caps, pipeline=pipeline))
    s.load_plasma(W.plasma_template(wl))
    return s


def _parts(wl, s, sizes, device):
    """The beam of species s as consecutive slice ranges of the given sizes."""
    out, j = [], 0
    for m in sizes:
        b = W.beam_species(wl, s, j, j + m)
        if device:
            b = {k: torch.from_numpy(np.ascontiguousarray(b[k])).to("cuda") for k in KEYS}
        out.append(b)
        j += m
    return out


@pytest.mark.parametrize("pipeline,device", [(1, False), (1, True), (3, True)])
def test_parts_equal_whole(pipeline, device):
    wl = W.small_3d(32, 16, 21).with_(
        dt=20.0, species=(W.Species(Z=-1, alpha=0.03, ppc=2, sigma_perp=1e-2),
                          W.Species(Z=1, alpha=0.03, ppc=2, sigma_perp=1e-2)))
    whole, parts = _sim(wl, pipeline), _sim(wl, pipeline)
    for s, b in enumerate(W.beam(wl)):
        whole.load_beam(s, b)
        first = 0
        for part in _parts(wl, s, [3, 8, 1, wl.beam_slices - 12], device):
            parts.load_beam_range(s, first, part)
            first += int(part["x"].shape[0])
        assert first == len(b["x"])
        got = parts.read_beam(s)
        for k in KEYS:
            assert np.array_equal(got[k], b[k]), (s, k)
    whole.beam_step(3)
    parts.beam_step(3)
    whole.slice_sweep()
    parts.slice_sweep()
    fw = {k: whole.fields(k) for k in OUT_FIELDS}
    fp = {k: parts.fields(k) for k in OUT_FIELDS}
    err, where = slice_errors(fp, fw)
    assert err <= 1e-12, (err, where)
    for s in range(2):
        a, b = parts.read_beam(s), whole.read_beam(s)
        for k in KEYS:
            assert np.abs(a[k] - b[k]).max() <= 1e-12 * max(1.0, np.abs(b[k]).max()), (s, k)


def test_range_rules():
    import paper_2607_24214_amd as Q
    wl = W.small_3d(16, 16, 9)
    n_slice = wl.n_perp * wl.species[0].ppc
    sim = _sim(wl, caps=[3 * n_slice])
    p0, p1, p2, p3 = _parts(wl, 0, [1, 1, 1, 1], False)
    sim.load_beam_range(0, 0, p0)
    with pytest.raises(Q.QSAError):          # a gap
        sim.load_beam_range(0, 2 * n_slice, p1)
    sim.load_beam_range(0, n_slice, p1)
    with pytest.raises(Q.QSAError):          # overlapping the loaded part
        sim.load_beam_range(0, n_slice // 2, p2)
    sim.load_beam_range(0, 2 * n_slice, p2)
    with pytest.raises(Q.QSAError):          # past the capacity
        sim.load_beam_range(0, 3 * n_slice, p3)
    assert len(sim.read_beam(0)["x"]) == 3 * n_slice
    sim.load_beam_range(0, 0, p3)            # first = 0 starts a new beam
    got = sim.read_beam(0)
    assert np.array_equal(got["xi"], p3["xi"])
    bad = {k: v.copy() for k, v in p0.items()}
    bad["ux"][5] = np.nan
    with pytest.raises(Q.QSAError):
        sim.load_beam_range(0, len(got["x"]), bad)

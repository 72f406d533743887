"""Resuming a run from a saved beam: 10 beam steps in one context equal 5
steps, the beam read back to the host, and 5 more steps in a new context
loaded with that beam and the same plasma template (the template re-enters
unperturbed at every sweep, so the beam is the whole state of a run between
beam steps; *Quasistatic model*: the plasma is a function of xi only through
the sweep, the beam evolves in tau).  Both ways also match the oracle run
straight through."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, run_oracle, slice_errors

pytestmark = pytest.mark.gpu

BEAM_KEYS = ("x", "y", "xi", "ux", "uy", "uz", "w")


def _sim(wl, caps, precision, pipeline=1):
    import paper_2607_24214_amd as Q
    sim = Q.Sim(Q.params_from_workload(wl, precision=precision, beam_capacity=caps, pipeline=pipeline))
    sim.load_plasma(W.plasma_template(wl))
    return sim


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_ten_steps_equal_five_saved_and_five_resumed(precision, tol):
    wl = W.small_3d(32, 16, 24, species=(W.Species(Z=-1, alpha=0.05, ppc=2, sigma_par=1e-3, sigma_perp=1e-3),
                                         W.Species(Z=1, alpha=0.05, ppc=2, sigma_par=1e-3, sigma_perp=1e-3)),
                    seed=71)
    beams = W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    # straight through
    a = _sim(wl, caps, precision)
    for s, b in enumerate(beams):
        a.load_beam(s, b)
    a.beam_step(10)
    a.slice_sweep()
    fa = {k: a.fields(k) for k in OUT_FIELDS}
    ba = [a.read_beam(s) for s in range(len(beams))]
    a.close()
    # five steps, save, drop the context
    b5 = _sim(wl, caps, precision)
    for s, b in enumerate(beams):
        b5.load_beam(s, b)
    b5.beam_step(5)
    saved = [{k: v.copy() for k, v in b5.read_beam(s).items()} for s in range(len(beams))]
    b5.close()
    for s, sv in enumerate(saved):
        assert len(sv["x"]) == caps[s]
        assert all(np.isfinite(sv[k]).all() for k in BEAM_KEYS)
    # resume in a fresh context
    c = _sim(wl, caps, precision)
    for s, sv in enumerate(saved):
        c.load_beam(s, sv)
    c.beam_step(5)
    c.slice_sweep()
    fc = {k: c.fields(k) for k in OUT_FIELDS}
    bc = [c.read_beam(s) for s in range(len(beams))]
    c.close()
    err, where = slice_errors(fc, fa)
    print(f"[resume {precision}] fields of the resumed run vs straight through: {err:.2e} at {where}")
    assert err <= tol, (err, where)
    for s in range(len(beams)):
        for k in BEAM_KEYS:
            scale = max(float(np.abs(ba[s][k]).max()), 1e-300)
            d = float(np.abs(bc[s][k] - ba[s][k]).max()) / scale
            assert d <= tol, (s, k, d)
    if precision == "f64":
        # and the oracle's ten steps straight through
        _, ref = run_oracle(wl, steps=10)
        err, where = slice_errors(fc, ref)
        print(f"[resume f64] resumed run vs the oracle's ten steps: {err:.2e} at {where}")
        assert err <= 1e-9, (err, where)


def test_resume_with_steps_in_flight_matches_one_at_a_time():
    """Steps in flight (8 per group, a copy of the beam kept) before and after
    the save: the resumed beam gives the same fields as one step at a time."""
    wl = W.small_3d(32, 16, 24, seed=72)
    beams = W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    ref = _sim(wl, caps, "f64")
    for s, b in enumerate(beams):
        ref.load_beam(s, b)
    ref.beam_step(16)
    ref.slice_sweep()
    fr = {k: ref.fields(k) for k in OUT_FIELDS}
    ref.close()
    p = _sim(wl, caps, "f64", pipeline=8)
    for s, b in enumerate(beams):
        p.load_beam(s, b)
    p.beam_step(8)
    saved = [{k: v.copy() for k, v in p.read_beam(s).items()} for s in range(len(beams))]
    p.close()
    q = _sim(wl, caps, "f64", pipeline=8)
    for s, sv in enumerate(saved):
        q.load_beam(s, sv)
    q.beam_step(8)
    q.slice_sweep()
    fq = {k: q.fields(k) for k in OUT_FIELDS}
    q.close()
    err, where = slice_errors(fq, fr)
    print(f"[resume pipelined] vs one step at a time: {err:.2e} at {where}")
    assert err <= 1e-10, (err, where)

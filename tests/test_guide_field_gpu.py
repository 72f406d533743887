"""The external guide field (uniform B_0 along the propagation axis, an
outlook item of the paper's conclusion) on the GPU against the oracle: a
beam-driven warm plasma in B_0 through beam steps, one step at a time and
with steps in flight."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, run_gpu, run_oracle, slice_errors

pytestmark = pytest.mark.gpu


def _wl(b0z, **kw):
    base = dict(dt=20.0, b0z=b0z, plasma_uth=0.01,
                species=(W.Species(Z=-1, alpha=0.05, ppc=2, sigma_perp=1e-2),
                         W.Species(Z=1, M=2.0, alpha=0.03, ppc=2, sigma_perp=1e-2)))
    base.update(kw)
    return W.small_3d(32, 16, 24).with_(**base)


@pytest.mark.parametrize("steps,prec,tol", [(0, "f64", 1e-10), (2, "f64", 1e-10), (2, "f32", 1e-4)])
def test_guide_field_matches_the_oracle(steps, prec, tol):
    wl = _wl(0.7)
    print(f"[guide] {wl.name} b0z={wl.b0z} steps={steps} prec={prec}", flush=True)
    so, ref = run_oracle(wl, steps)
    sg, got = run_gpu(wl, steps, precision=prec)
    err, where = slice_errors(got, ref)
    print(f"[guide]   max slice error {err:.3e} at {where}", flush=True)
    assert err <= tol, (err, where)
    if steps:
        for s in range(len(wl.species)):
            bg, bo = sg.read_beam(s), so.beams[s]
            for k in ("x", "y", "ux", "uy", "uz"):
                d = float(np.abs(bg[k] - bo[k].numpy()).max())
                scale = max(1.0, float(np.abs(bo[k].numpy()).max()))
                assert d <= (1e-11 if prec == "f64" else 1e-4) * scale, (s, k, d)
    sg.close()
    # the field changes the answer (the test would pass vacuously otherwise)
    _, ref0 = run_oracle(wl.with_(b0z=0.0), steps)
    d0, _ = slice_errors(ref0, ref)
    assert d0 > 100 * tol, d0


def test_guide_field_steps_in_flight_match_one_at_a_time():
    import paper_2607_24214_amd as Q
    wl = _wl(-0.5)
    beams = W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    sims = []
    for pipe in (1, 4):
        s = Q.Sim(Q.params_from_workload(wl, precision="f64", beam_capacity=caps, pipeline=pipe))
        s.load_plasma(W.plasma_template(wl))
        for k, b in enumerate(beams):
            s.load_beam(k, b)
        s.beam_step(4)
        s.slice_sweep()
        sims.append(s)
    assert sims[1].pipeline == 4
    a = {k: sims[0].fields(k) for k in OUT_FIELDS}
    b = {k: sims[1].fields(k) for k in OUT_FIELDS}
    err, where = slice_errors(b, a)
    print(f"[guide] 4 steps in flight vs one at a time: {err:.3e} at {where}", flush=True)
    assert err <= 1e-10, (err, where)
    for s in sims:
        s.close()

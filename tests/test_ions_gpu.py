"""Mobile plasma ions on the GPU against the oracle (ion motion is in the
outlook of the paper's conclusion): electrons and ions of charge Z and mass
M in one template, the ions marked by negative weights at the boundary;
light and heavy ions, one step at a time and in flight."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, matched_kappa2, run_gpu, run_oracle, slice_errors

pytestmark = pytest.mark.gpu


def _wl(**kw):
    base = dict(dt=20.0, plasma_uth=0.01, ion_m=4.0, ion_z=1,
                species=(W.Species(Z=-1, alpha=0.05, ppc=2, sigma_perp=1e-2),))
    base.update(kw)
    wl = W.small_3d(32, 16, 24).with_(**base)
    # the B_perp iteration's shift matched to electrons plus mobile ions
    return wl.with_(kappa2=matched_kappa2(wl))


@pytest.mark.parametrize("kw,steps,prec,tol", [
    (dict(), 0, "f64", 1e-10),
    (dict(), 2, "f64", 1e-10),
    (dict(ion_z=2, ion_m=8.0), 2, "f64", 1e-10),
    (dict(ion_m=1836.0, b0z=0.3), 1, "f64", 1e-10),
    (dict(), 2, "f32", 1e-4),
])
def test_mobile_ions_match_the_oracle(kw, steps, prec, tol):
    wl = _wl(**kw)
    print(f"[ions] {wl.name} Z={wl.ion_z} M={wl.ion_m} b0z={wl.b0z} steps={steps} prec={prec}", flush=True)
    so, ref = run_oracle(wl, steps)
    sg, got = run_gpu(wl, steps, precision=prec)
    err, where = slice_errors(got, ref)
    print(f"[ions]   max slice error {err:.3e} at {where}", flush=True)
    assert err <= tol, (err, where)
    sg.close()
    if steps and wl.ion_m < 100:
        # the ions' motion changes the answer
        _, ref0 = run_oracle(wl.with_(ion_m=0.0), steps)
        d0, _ = slice_errors(ref0, ref)
        assert d0 > 100 * tol, d0


def test_mobile_ions_steps_in_flight_match_one_at_a_time():
    import paper_2607_24214_amd as Q
    wl = _wl(ion_m=2.0)
    beams = W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    out = []
    for pipe in (1, 4):
        s = Q.Sim(Q.params_from_workload(wl, precision="f64", beam_capacity=caps, pipeline=pipe))
        s.load_plasma(W.plasma_template(wl))
        for k, b in enumerate(beams):
            s.load_beam(k, b)
        s.beam_step(4)
        s.slice_sweep()
        assert s.pipeline == pipe
        out.append({k: s.fields(k) for k in OUT_FIELDS})
        s.close()
    err, where = slice_errors(out[1], out[0])
    print(f"[ions] 4 steps in flight vs one at a time: {err:.3e} at {where}", flush=True)
    assert err <= 1e-10, (err, where)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_slab_with_mobile_ions_guide_field_and_density(prec, tol):
    """The slab geometry (ny = 1) with every plasma option at once: mobile
    ions of charge 2, a guide field and a modulated density."""
    wl = W.slab_electron().with_(nxi=64, ion_m=6.0, ion_z=2, b0z=0.4, plasma_uth=0.01,
                                  plasma_n0=1.1, plasma_mod=0.25, plasma_mod_mx=2)
    wl = wl.with_(kappa2=matched_kappa2(wl))
    so, ref = run_oracle(wl, 1)
    sg, got = run_gpu(wl, 1, precision=prec)
    err, where = slice_errors(got, ref)
    print(f"[ions] slab, all plasma options, {prec}: {err:.3e} at {where}", flush=True)
    assert err <= tol, (err, where)
    sg.close()

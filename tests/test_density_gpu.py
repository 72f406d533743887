"""An inhomogeneous plasma on the GPU against the oracle (plasma
inhomogeneity is in the outlook of the paper's conclusion): the electrons
carry a density profile in their weights, the immobile ions match it at the
nodes (qsa_load_ions).  A transverse profile through beam steps, and a
density that changes along the propagation distance (new weights and ions
loaded between beam steps)."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, matched_kappa2, run_gpu, run_oracle, slice_errors

pytestmark = pytest.mark.gpu


def _wl(**kw):
    base = dict(dt=20.0, plasma_uth=0.01, plasma_n0=1.2, plasma_mod=0.3, plasma_mod_mx=1, plasma_mod_my=2,
                species=(W.Species(Z=-1, alpha=0.05, ppc=2, sigma_perp=1e-2),))
    base.update(kw)
    wl = W.small_3d(32, 16, 24).with_(**base)
    # the B_perp iteration's shift matched to the denser plasma
    return wl.with_(kappa2=matched_kappa2(wl))


@pytest.mark.parametrize("steps,prec,tol", [(0, "f64", 1e-10), (2, "f64", 1e-10), (2, "f32", 1e-4)])
def test_transverse_profile_matches_the_oracle(steps, prec, tol):
    wl = _wl()
    print(f"[density] {wl.name} n0={wl.plasma_n0} mod={wl.plasma_mod} steps={steps} prec={prec}", flush=True)
    so, ref = run_oracle(wl, steps)
    sg, got = run_gpu(wl, steps, precision=prec)
    err, where = slice_errors(got, ref)
    print(f"[density]   max slice error {err:.3e} at {where}", flush=True)
    assert err <= tol, (err, where)
    sg.close()
    # the profile changes the answer
    _, ref0 = run_oracle(wl.with_(plasma_n0=1.0, plasma_mod=0.0), steps)
    d0, _ = slice_errors(ref0, ref)
    assert d0 > 100 * tol, d0


def test_profile_with_random_weights_matches_the_oracle():
    wl = _wl(plasma_w_spread=0.4)
    _, ref = run_oracle(wl, 1)
    sg, got = run_gpu(wl, 1, precision="f64")
    err, where = slice_errors(got, ref)
    print(f"[density] with random weights: {err:.3e} at {where}", flush=True)
    assert err <= 1e-10, (err, where)
    sg.close()


def test_density_along_the_propagation_distance():
    """Three beam steps in plasmas of densities 1.0, 1.3, 1.6 (a density
    ramp along z): the template's weights and the ions are reloaded before
    each step."""
    import paper_2607_24214_amd as Q
    from oracle import qsa_pic as O
    wl = _wl(plasma_mod=0.2)
    ramp = (1.0, 1.3, 1.6)
    beams = W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    sim = Q.Sim(Q.params_from_workload(wl, precision="f64", beam_capacity=caps))
    so = O.Sim(wl, W.plasma_template(wl), beams)
    for s, b in enumerate(beams):
        sim.load_beam(s, b)
    for n0 in ramp:
        wn = wl.with_(plasma_n0=n0)
        tmpl = W.plasma_template(wn)
        sim.load_plasma(tmpl)
        so.plasma = O.to_torch(tmpl)
        sim.beam_step(1)
        so.beam_step(1)
    sim.slice_sweep()
    so.sweep()
    got = {k: sim.fields(k) for k in OUT_FIELDS}
    ref = {k: v.numpy() for k, v in O.output_fields(so.fields).items()}
    err, where = slice_errors(got, ref)
    print(f"[density] ramp along z, 3 steps: {err:.3e} at {where}", flush=True)
    assert err <= 1e-10, (err, where)
    sim.close()


def test_ions_need_a_weighted_context():
    import paper_2607_24214_amd as Q
    from paper_2607_24214_amd import _lib as L
    wl = W.small_3d(16, 8, 8)
    sim = Q.Sim(Q.params_from_workload(wl, precision="f64"))
    sim.load_plasma(W.plasma_template(wl))
    ion = np.ones(wl.nx * wl.ny)
    st = sim.lib.qsa_load_ions(sim.ctx, ion.ctypes.data, ion.size, 0)
    assert st == -6        # QSA_E_STATE
    wl2 = _wl()
    s2 = Q.Sim(Q.params_from_workload(wl2, precision="f64"))
    s2.load_plasma(W.plasma_template(wl2))
    bad = np.ones(wl2.nx * wl2.ny - 1)
    assert s2.lib.qsa_load_ions(s2.ctx, bad.ctypes.data, bad.size, 0) == -1
    nan = np.full(wl2.nx * wl2.ny, np.nan)
    assert s2.lib.qsa_load_ions(s2.ctx, nan.ctypes.data, nan.size, 0) == -5
    sim.close()
    s2.close()

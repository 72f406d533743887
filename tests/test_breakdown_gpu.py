"""Quasistatic breakdown: a dense positron beam (alpha = 5, gamma_b = 2) in
the slab drives 1 + psi below the threshold at plasma particles within the
first slices.  The oracle raises on it (a CPU test pins that); on the GPU the
kernels only set the context's device flag and run to their end: the next
synchronizing call reports QSA_E_BREAKDOWN, every later call does too, and
the device stays usable (a fresh context afterwards matches the oracle)."""
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, run_oracle, slice_errors

pytestmark = pytest.mark.gpu

QSA_E_BREAKDOWN = -4


def dense_positron_slab():
    return W.slab_electron().with_(
        nx=16, nxi=32, gamma_b=2.0, species=(W.Species(Z=+1, M=1.0, alpha=5.0, ppc=2),), steps=1)


def _sim(wl, precision):
    import paper_2607_24214_amd as Q
    beams = W.beam(wl)
    s = Q.Sim(Q.params_from_workload(wl, precision=precision, beam_capacity=[len(b["x"]) for b in beams]))
    s.load_plasma(W.plasma_template(wl))
    for k, b in enumerate(beams):
        s.load_beam(k, b)
    return s


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("call", ["sweep", "step"])
def test_breakdown_is_flagged_and_sticky(precision, call):
    import paper_2607_24214_amd as Q
    s = _sim(dense_positron_slab(), precision)
    print(f"[breakdown] {precision} {call}", flush=True)
    if call == "sweep":
        s.slice_sweep()
    else:
        s.beam_step(1)
    with pytest.raises(Q.QSAError) as e:
        s.sync()
    assert e.value.status == QSA_E_BREAKDOWN, e.value
    with pytest.raises(Q.QSAError) as e2:   # sticky
        s.fields("psi")
    assert e2.value.status == QSA_E_BREAKDOWN, e2.value
    with pytest.raises(Q.QSAError) as e3:
        s.beam_step(1)
    assert e3.value.status == QSA_E_BREAKDOWN, e3.value
    s.close()
    # the device is still usable
    wl = W.small_3d(16, 16, 12)
    t = _sim(wl, "f64")
    t.slice_sweep()
    t.sync()
    got = {k: t.fields(k) for k in OUT_FIELDS}
    _, ref = run_oracle(wl)
    err, where = slice_errors(got, ref)
    assert err <= 1e-10, (err, where)

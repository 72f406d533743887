"""Beam steps in flight without a second copy of the beam (lean_pipeline):
each group's sort by cell row gathers the beam in place, so the fields,
sources and particles after pipelined groups must equal the same steps taken
one at a time (particles matched by their weights, which the push leaves
unchanged and the test makes distinct, since the storage order is no longer
the load order); a group that breaks the drift schedule cannot be repeated
and must fail, and the parameters refuse a capacity the in-place sort cannot
hold."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, slice_errors

pytestmark = pytest.mark.gpu

SRC_FIELDS = ("src_S", "src_Jx", "src_Jy", "src_Jz")
KEYS = ("x", "y", "xi", "ux", "uy", "uz", "w")


def _tagged(wl, s, seed):
    """The species' beam shuffled, its weights scaled by distinct factors
    1 + k 2^-20 (distinct in float32 too) so that each names its particle,
    none within three cells of the back of the box (where the push retires
    particles to weight 0)."""
    b = W.beam(wl)[s]
    rng = np.random.default_rng(seed)
    n = len(b["x"])
    order = rng.permutation(n)
    out = {k: np.ascontiguousarray(v[order]) for k, v in b.items()}
    out["xi"] = np.minimum(out["xi"], (wl.nxi - 4) * wl.dxi)
    out["w"] = out["w"] * (1.0 + rng.permutation(n).astype(np.float64) * 2.0 ** -20)
    return out


def _sim(wl, pipeline, lean, beams, precision="f64"):
    import paper_2607_24214_amd as Q
    caps = [len(b["x"]) for b in beams]
    s = Q.Sim(Q.params_from_workload(wl, precision=precision, beam_capacity=caps, pipeline=pipeline,
                                     lean_pipeline=lean))
    s.load_plasma(W.plasma_template(wl))
    for k, b in enumerate(beams):
        s.load_beam(k, b)
    return s


def _match(a, b):
    """b's particles in a's order, matched by weight."""
    ia, ib = np.argsort(a["w"], kind="stable"), np.argsort(b["w"], kind="stable")
    assert np.allclose(a["w"][ia], b["w"][ib], rtol=1e-6, atol=0.0)
    inv = np.empty_like(ia)
    inv[ia] = np.arange(len(ia))
    return {k: v[ib][inv] for k, v in b.items()}


def _compare(tag, a, b, tol_f, tol_b, n_species):
    fa = {k: a.fields(k) for k in OUT_FIELDS + SRC_FIELDS}
    fb = {k: b.fields(k) for k in OUT_FIELDS + SRC_FIELDS}
    err, where = slice_errors(fa, fb)
    print(f"[lean] {tag}: fields and sources {err:.3e} at {where}", flush=True)
    assert err <= tol_f, (tag, err, where)
    for s in range(n_species):
        ba = a.read_beam(s)
        bb = _match(ba, b.read_beam(s))
        for k in KEYS:
            scale = max(1.0, float(np.abs(bb[k]).max()))
            d = float(np.abs(ba[k] - bb[k]).max())
            assert d <= tol_b * scale, (tag, s, k, d)


def test_lean_groups_match_one_at_a_time_fp64():
    wl = W.small_3d(32, 32, 40).with_(dt=20.0)
    beams = [_tagged(wl, 0, 1)]
    seq, lean = _sim(wl, 1, False, beams), _sim(wl, 4, True, beams)
    assert lean.pipeline == 4
    for n in (4, 5, 1):   # one full group; a group and a lone step; a lone step
        seq.beam_step(n)
        lean.beam_step(n)
        _compare(f"after +{n} steps", lean, seq, 1e-10, 1e-11, 1)
    assert lean.pipeline == 4


def test_lean_pair_rectangular_fp64():
    wl = W.small_3d(64, 16, 27).with_(
        species=(W.Species(Z=-1, alpha=0.03, ppc=2, sigma_perp=1e-2),
                 W.Species(Z=1, alpha=0.03, ppc=2, sigma_perp=1e-2)), dt=10.0)
    beams = [_tagged(wl, 0, 2), _tagged(wl, 1, 3)]
    seq, lean = _sim(wl, 1, False, beams), _sim(wl, 3, True, beams)
    seq.beam_step(6)
    lean.beam_step(6)
    _compare("pair, two groups of 3", lean, seq, 1e-10, 1e-11, 2)


def test_lean_fp32():
    wl = W.small_3d(32, 32, 29).with_(dt=20.0)
    beams = [_tagged(wl, 0, 4)]
    seq, lean = _sim(wl, 1, False, beams, "f32"), _sim(wl, 4, True, beams, "f32")
    seq.beam_step(4)
    lean.beam_step(4)
    _compare("fp32", lean, seq, 1e-4, 1e-5, 1)


def test_lean_equals_full_pipeline_fp64():
    """The same groups with and without the beam copy."""
    wl = W.small_3d(32, 16, 33).with_(dt=20.0)
    beams = [_tagged(wl, 0, 5)]
    full, lean = _sim(wl, 4, False, beams), _sim(wl, 4, True, beams)
    full.beam_step(8)
    lean.beam_step(8)
    assert full.pipeline == 4 and lean.pipeline == 4
    _compare("lean against full", lean, full, 1e-10, 1e-11, 1)


def test_lean_drift_violation_fails():
    """A slow beam (gamma 2) slips several cells per step: a lean group
    cannot be repeated one step at a time, so the step fails and the context
    keeps the error."""
    import paper_2607_24214_amd as Q
    wl = W.small_3d(32, 16, 24).with_(gamma_b=2.0, dt=2.0)
    lean = _sim(wl, 3, True, W.beam(wl))
    with pytest.raises(Q.QSAError):
        lean.beam_step(3)
    with pytest.raises(Q.QSAError):
        lean.beam_step(1)


def test_lean_parameter_rules():
    import paper_2607_24214_amd as Q
    wl = W.small_3d(16, 16, 9)
    n_fit = (4 + 7) * wl.nxi * wl.nx * wl.ny   # float64 values of one set's sources and fields
    with pytest.raises(Q.QSAError):
        Q.Sim(Q.params_from_workload(wl, beam_capacity=[n_fit + 1], pipeline=2, lean_pipeline=True))
    Q.Sim(Q.params_from_workload(wl, beam_capacity=[n_fit], pipeline=2, lean_pipeline=True))
    # one step at a time: the flag is ignored, so any capacity goes
    Q.Sim(Q.params_from_workload(wl, beam_capacity=[n_fit + 1], pipeline=1, lean_pipeline=True))
    with pytest.raises(Q.QSAError):
        Q.Sim(Q.params_from_workload(wl, pipeline=2, lean_pipeline=True, adjoint_steps=2))

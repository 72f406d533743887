"""Beam steps in flight (pipeline > 1): each group of pipelined steps must give
the fields, sources and beam of the same steps taken one at a time (only the
order of floating-point additions in the beam deposit differs), and the
oracle's after several steps.  A beam that breaks the pipeline's drift bound
(one slipping several cells per step) must be detected, rolled back and
repeated one step at a time."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, run_oracle, slice_errors

pytestmark = pytest.mark.gpu

SRC_FIELDS = ("src_S", "src_Jx", "src_Jy", "src_Jz")
BEAM_KEYS = ("x", "y", "xi", "ux", "uy", "uz", "w")


def _sim(wl, pipeline, precision="f64", beams=None):
    import paper_2607_24214_amd as Q
    beams = beams if beams is not None else W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    s = Q.Sim(Q.params_from_workload(wl, precision=precision, beam_capacity=caps, pipeline=pipeline))
    s.load_plasma(W.plasma_template(wl))
    for k, b in enumerate(beams):
        s.load_beam(k, b)
    return s


def _fields(sim):
    return {k: sim.fields(k) for k in OUT_FIELDS + SRC_FIELDS}


def _compare(tag, a, b, tol_f, tol_b, n_species=1):
    err, where = slice_errors(_fields(a), _fields(b))
    print(f"[pipe] {tag}: fields and sources {err:.3e} at {where}", flush=True)
    assert err <= tol_f, (tag, err, where)
    for s in range(n_species):
        ba, bb = a.read_beam(s), b.read_beam(s)
        for k in BEAM_KEYS:
            d = float(np.abs(ba[k] - bb[k]).max()) if len(bb[k]) else 0.0
            scale = max(1.0, float(np.abs(bb[k]).max()) if len(bb[k]) else 1.0)
            assert d <= tol_b * scale, (tag, s, k, d)


def test_pipelined_steps_match_one_at_a_time_fp64():
    wl = W.small_3d(32, 32, 40).with_(dt=20.0)
    seq, pip = _sim(wl, 1), _sim(wl, 4)
    assert pip.pipeline == 4
    for n in (4, 5, 1):   # one full group; a group and a lone step; a lone step
        seq.beam_step(n)
        pip.beam_step(n)
        _compare(f"after +{n} steps", pip, seq, 1e-10, 1e-11)
    assert pip.pipeline == 4
    pip.slice_sweep()
    got = {k: pip.fields(k) for k in OUT_FIELDS}
    _, ref = run_oracle(wl, 10)
    err, where = slice_errors(got, ref)
    print(f"[pipe] 10 pipelined steps vs oracle {err:.3e} at {where}", flush=True)
    assert err <= 1e-9, (err, where)


def test_pipeline_deeper_than_box_fp64():
    """Eight steps in flight on a box of 12 slices (lags beyond the box)."""
    wl = W.small_3d(16, 16, 12).with_(dt=10.0)
    seq, pip = _sim(wl, 1), _sim(wl, 8)
    seq.beam_step(8)
    pip.beam_step(8)
    _compare("8 in flight, nxi 12", pip, seq, 1e-10, 1e-11)


def test_pipeline_sixteen_deep_fp64():
    """The deepest pipeline: sixteen steps in flight (lags up to 120 slices,
    beyond a 24-slice box), as one group and then as a group of 5."""
    wl = W.small_3d(16, 16, 24).with_(dt=10.0)
    seq, pip = _sim(wl, 1), _sim(wl, 16)
    for n in (16, 5):
        seq.beam_step(n)
        pip.beam_step(n)
        _compare(f"16 in flight, +{n} steps", pip, seq, 1e-10, 1e-11)
    assert pip.pipeline == 16


def test_pipelined_slab_fp64():
    wl = W.slab_electron()
    seq, pip = _sim(wl, 1), _sim(wl, 4)
    seq.beam_step(4)
    pip.beam_step(4)
    _compare("slab", pip, seq, 1e-10, 1e-11)


def test_pipelined_pair_rectangular_fp64():
    wl = W.small_3d(64, 16, 20).with_(
        species=(W.Species(Z=-1, alpha=0.03, ppc=2, sigma_perp=1e-2),
                 W.Species(Z=1, alpha=0.03, ppc=2, sigma_perp=1e-2)), dt=10.0)
    seq, pip = _sim(wl, 1), _sim(wl, 3)
    seq.beam_step(3)
    pip.beam_step(3)
    _compare("pair", pip, seq, 1e-10, 1e-11, n_species=2)


def test_pipelined_warm_beam_fp64():
    """A warm beam moves about two cells per step transversely: many
    particles leave the row window the deposit gathers and take the atomic
    path; the results must not change."""
    wl = W.small_3d(32, 32, 24).with_(
        dt=20.0, species=(W.Species(Z=-1, alpha=0.05, ppc=2, sigma_par=1e-3, sigma_perp=1e-2),))
    seq, pip = _sim(wl, 1), _sim(wl, 4)
    seq.beam_step(4)
    pip.beam_step(4)
    assert pip.pipeline == 4
    _compare("warm beam", pip, seq, 1e-10, 1e-11)


def test_pipelined_random_plasma_weights_fp64():
    wl = W.small_3d(32, 16, 24).with_(dt=20.0, plasma_uth=0.01, plasma_w_spread=0.6)
    seq, pip = _sim(wl, 1), _sim(wl, 3)
    seq.beam_step(3)
    pip.beam_step(3)
    assert pip.pipeline == 3
    _compare("plasma weights", pip, seq, 1e-10, 1e-11)


def test_pipelined_fp32():
    wl = W.small_3d(32, 32, 24).with_(dt=20.0)
    seq, pip = _sim(wl, 1, "f32"), _sim(wl, 4, "f32")
    seq.beam_step(4)
    pip.beam_step(4)
    _compare("fp32", pip, seq, 1e-4, 1e-5)


def test_pipeline_graphs_match_direct_launches_fp64():
    wl = W.small_3d(32, 16, 16).with_(dt=20.0)
    a, b = _sim(wl, 3), _sim(wl, 3)
    b.set_graphs(False)
    for _ in range(3):
        a.beam_step(3)
        b.beam_step(3)
        _compare("graph vs direct", a, b, 1e-12, 1e-13)


def test_shuffled_beam_pipelines_fp64():
    """Particles loaded in random order: the library sorts them by cell row
    (reading them back gives load order), and the pipeline stays on."""
    wl = W.small_3d(32, 16, 16).with_(dt=20.0)
    beams = W.beam(wl)
    perm = np.random.default_rng(11).permutation(len(beams[0]["x"]))
    shuffled = [{k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in beams[0].items()}]
    seq, pip = _sim(wl, 1, beams=shuffled), _sim(wl, 3, beams=shuffled)
    b0 = pip.read_beam(0)
    for k in BEAM_KEYS:
        assert np.array_equal(b0[k], shuffled[0][k]), k
    seq.beam_step(3)
    pip.beam_step(3)
    assert pip.pipeline == 3
    _compare("shuffled", pip, seq, 1e-10, 1e-11)


def test_drift_violation_rolls_back_fp64():
    """A slow beam (gamma 2) slips several cells per step behind its slab:
    the group must be undone and taken one step at a time, with pipelining
    then off until the caller turns it on again."""
    wl = W.small_3d(32, 16, 24).with_(gamma_b=2.0, dt=2.0)
    seq, pip = _sim(wl, 1), _sim(wl, 3)
    seq.beam_step(3)
    pip.beam_step(3)
    assert pip.pipeline == 1
    _compare("rolled back", pip, seq, 1e-10, 1e-11)
    pip.set_pipeline(3)
    assert pip.pipeline == 3
    seq.beam_step(3)
    pip.beam_step(3)
    assert pip.pipeline == 1
    _compare("rolled back twice", pip, seq, 1e-10, 1e-11)

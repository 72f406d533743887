"""Launch shapes and the autotuner: every plasma-row and row-transform block
width and column-transform thread count gives the same sweep (up to the
order of additions), and autotuning leaves the beam untouched and later
steps unchanged."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, slice_errors

pytestmark = pytest.mark.gpu


def _sim(wl, pipeline=1):
    import paper_2607_24214_amd as Q
    s = Q.Sim(Q.params_from_workload(wl, precision="f64", pipeline=pipeline))
    s.load_plasma(W.plasma_template(wl))
    for k, b in enumerate(W.beam(wl)):
        s.load_beam(k, b)
    return s


@pytest.mark.parametrize("nt,rt", [(64, 64), (128, 128), (256, 256), (128, 64)])
def test_launch_shapes_agree_fp64(nt, rt):
    wl = W.small_3d(64, 32, 16)
    ref, sim = _sim(wl), _sim(wl)
    sim.set_shapes(nt, rt)
    assert sim.shapes()[:2] == (nt, rt)
    ref.slice_sweep()
    sim.slice_sweep()
    err, where = slice_errors({k: sim.fields(k) for k in OUT_FIELDS}, {k: ref.fields(k) for k in OUT_FIELDS})
    print(f"[shapes] nt={nt} rt={rt}: {err:.3e} at {where}", flush=True)
    assert err <= 1e-12, (err, where)


@pytest.mark.parametrize("ct", [16, 32, 64])
def test_column_threads_agree_fp64(ct):
    """ny = 256: 16, 32 or 64 threads per column transform (4, 2 or 1
    columns per wavefront)."""
    wl = W.small_3d(32, 256, 6)
    ref, sim = _sim(wl), _sim(wl)
    sim.set_shapes(0, 0, ct)
    assert sim.shapes()[2] == ct
    ref.slice_sweep()
    sim.slice_sweep()
    err, where = slice_errors({k: sim.fields(k) for k in OUT_FIELDS}, {k: ref.fields(k) for k in OUT_FIELDS})
    print(f"[shapes] column threads {ct}: {err:.3e} at {where}", flush=True)
    assert err <= 1e-12, (err, where)


def test_invalid_shapes_rejected():
    import paper_2607_24214_amd as Q
    sim = _sim(W.small_3d(32, 16, 8))
    for nt, rt, ct in ((96, 0, 0), (0, 32, 0), (512, 0, 0), (0, 0, 8), (0, 0, 128)):
        with pytest.raises(Q.QSAError):
            sim.set_shapes(nt, rt, ct)


def test_autotune_keeps_the_beam_and_the_physics_fp64():
    import paper_2607_24214_amd as Q
    wl = W.small_3d(32, 32, 24).with_(dt=20.0)
    ref, sim = _sim(wl, 4), _sim(wl, 4)
    before = sim.read_beam(0)
    ms = sim.autotune()
    print(f"[autotune] best {ms:.3f} ms/step, shapes {sim.shapes()}, steps in flight {sim.pipeline}",
          flush=True)
    assert ms > 0.0
    after = sim.read_beam(0)
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    nt, rt, ct = sim.shapes()
    assert nt in (64, 128, 256) and rt in (64, 128, 256) and ct in (8, 16, 32, 64)
    assert sim.pipeline in (2, 4)
    with pytest.raises(Q.QSAError):
        sim.fields("psi")
    ref.beam_step(4)
    sim.beam_step(4)
    err, where = slice_errors({k: sim.fields(k) for k in OUT_FIELDS}, {k: ref.fields(k) for k in OUT_FIELDS})
    print(f"[autotune] 4 steps after tuning vs untuned: {err:.3e} at {where}", flush=True)
    assert err <= 1e-10, (err, where)

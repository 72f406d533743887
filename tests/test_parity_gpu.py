"""GPU parity: the HIP library against the float64 oracle on identical seeded
inputs, slice by slice and field by field, after 0 and 1 beam steps.

Tolerances: float64 path 1e-10 (only the order of atomic additions, FMA
contraction and the transform's rounding differ); float32 path 1e-4.  The
error of a field on a slice is ||GPU - oracle||_2 divided by the largest
oracle field norm on that slice.
"""
import math

import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, run_gpu, run_oracle, slice_errors

pytestmark = pytest.mark.gpu


def _case(wl, steps, prec, tol):
    print(f"[parity] {wl.name} nx={wl.nx} ny={wl.ny} nxi={wl.nxi} steps={steps} prec={prec}", flush=True)
    so, ref = run_oracle(wl, steps)
    sg, got = run_gpu(wl, steps, precision=prec)
    err, where = slice_errors(got, ref)
    print(f"[parity]   max slice error {err:.3e} at {where}", flush=True)
    assert err <= tol, (err, where)
    return so, sg


@pytest.mark.parametrize("steps", [0, 1])
def test_slab_fp64(steps):
    _case(W.slab_electron(), steps, "f64", 1e-10)


@pytest.mark.parametrize("steps", [0, 1])
def test_3d_warm_fp64(steps):
    _case(W.small_3d(32, 32, 24), steps, "f64", 1e-10)


def test_3d_rectangular_pair_fp64():
    wl = W.small_3d(64, 16, 20).with_(
        species=(W.Species(Z=-1, alpha=0.03, ppc=2, sigma_perp=1e-2),
                 W.Species(Z=1, alpha=0.03, ppc=2, sigma_perp=1e-2)))
    _case(wl, 1, "f64", 1e-10)


def test_random_beam_weights_fp64():
    """Random macro-particle weights (each weight times 1 + 0.9 (2U - 1)), the
    paper's noise-control loading, through a beam step."""
    wl = W.small_3d(32, 16, 20).with_(
        species=(W.Species(Z=-1, alpha=0.05, ppc=4, sigma_perp=1e-3, w_spread=0.9),))
    _case(wl, 1, "f64", 1e-10)


def test_ramped_beam_fp64():
    """A longitudinal profile instead of the flat top (linear head and tail
    ramps, with random weights on top), through two beam steps."""
    wl = W.small_3d(32, 16, 30).with_(
        dt=20.0, species=(W.Species(Z=-1, alpha=0.05, ppc=4, sigma_perp=1e-3, w_spread=0.3,
                                    ramp_head=0.9, ramp_tail=0.6),))
    _case(wl, 2, "f64", 1e-10)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_random_plasma_weights(prec, tol):
    """Random plasma macro-particle weights (each w0 (1 + 0.6 (2U - 1))),
    a warm plasma, through two beam steps: the weights follow the particles
    through the sorts."""
    wl = W.small_3d(32, 16, 20).with_(plasma_uth=0.01, plasma_w_spread=0.6, dt=20.0)
    _case(wl, 2, prec, tol)


def test_plasma_weights_need_the_parameter():
    import paper_2607_24214_amd as Q
    wl = W.small_3d(16, 16, 8).with_(plasma_w_spread=0.5)
    pl = W.plasma_template(wl)
    p = Q.params_from_workload(wl)
    assert p.plasma_weights == 1
    p0 = Q.params_from_workload(wl.with_(plasma_w_spread=0.0))
    s = Q.Sim(p0)
    with pytest.raises(ValueError):
        s.load_plasma(pl)
    s.load_plasma(W.plasma_template(wl.with_(plasma_w_spread=0.0)))
    import ctypes as C
    w = np.ascontiguousarray(pl["w"])
    assert s.lib.qsa_load_plasma_weights(s.ctx, C.c_void_p(w.ctypes.data), w.size, 0) == -6   # QSA_E_STATE
    t = Q.Sim(p)
    t.load_plasma(pl)
    bad = w.copy()
    bad[3] = -1.0
    assert t.lib.qsa_load_plasma_weights(t.ctx, C.c_void_p(bad.ctypes.data), bad.size, 0) == -5   # NONFINITE
    assert t.lib.qsa_load_plasma_weights(t.ctx, C.c_void_p(w.ctypes.data), w.size - 1, 0) == -1   # count


def test_3d_fp32():
    _case(W.small_3d(32, 32, 24), 1, "f32", 1e-4)


def test_slab_fp32():
    _case(W.slab_electron(), 1, "f32", 1e-4)


def test_beam_sources_and_push_fp64():
    wl = W.small_3d(16, 16, 12)
    from oracle import qsa_pic as O
    so, _ = run_oracle(wl, 0)
    sg, _ = run_gpu(wl, 0)
    src = O.beam_sources(so.g, so.beams, so.Z).numpy()
    for c, name in enumerate(("src_S", "src_Jx", "src_Jy", "src_Jz")):
        g = sg.fields(name)
        scale = max(np.abs(src[c]).max(), 1e-300)
        assert np.abs(g - src[c]).max() <= 1e-12 * np.abs(src).max(), name
    # one push in the fields of that sweep
    so.push()
    sg.beam_step(1)
    b = sg.read_beam(0)
    ob = so.beams[0]
    for k in ("x", "y", "xi", "ux", "uy", "uz", "w"):
        ref = ob[k].numpy()
        assert np.abs(b[k] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), k


def test_unsorted_beam_input_fp64():
    """Beam particles loaded in random order: every particle is outside the
    cell row its block expects, so the whole deposit takes the out-of-row
    path; the fields must not change."""
    wl = W.small_3d(32, 16, 16)
    beams = W.beam(wl)
    rng = np.random.default_rng(5)
    perm = rng.permutation(len(beams[0]["x"]))
    shuffled = [{k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in beams[0].items()}]
    so, ref = run_oracle(wl, 1, beams=beams)
    sg, got = run_gpu(wl, 1, precision="f64", beams=shuffled)
    err, where = slice_errors(got, ref)
    print(f"[parity] shuffled beam: max slice error {err:.3e} at {where}", flush=True)
    assert err <= 1e-10, (err, where)


def test_three_steps_fp64():
    """Several beam steps: particles drift across cell rows between steps."""
    wl = W.small_3d(32, 32, 16).with_(dt=20.0)
    _case(wl, 3, "f64", 1e-9)


def test_graph_replays_match_eager_fp64():
    """The captured sweep and step graphs, replayed several times with eager
    work (field reads) in between, give the eager launch sequence's fields."""
    import paper_2607_24214_amd as Q
    wl = W.small_3d(32, 16, 16).with_(dt=20.0)
    plasma = W.plasma_template(wl)
    beams = W.beam(wl)
    sims = []
    for graphs in (True, False):
        s = Q.Sim(Q.params_from_workload(wl, precision="f64"))
        s.set_graphs(graphs)
        s.load_plasma(plasma)
        s.load_beam(0, beams[0])
        sims.append(s)
    for step in range(3):
        for s in sims:
            s.beam_step(1)
            s.slice_sweep()
        a = {k: sims[0].fields(k) for k in OUT_FIELDS}
        b = {k: sims[1].fields(k) for k in OUT_FIELDS}
        err, where = slice_errors(a, b)
        print(f"[graph] replay {step}: max slice difference {err:.3e} at {where}", flush=True)
        assert err <= 1e-12, (step, err, where)


def _scan_like(i, nx, ny, nxi, alpha, gamma, dt):
    return W.Workload(
        name=f"batch{i}", nx=nx, ny=ny, nxi=nxi, dx=0.1, dy=0.1, dxi=0.1, gamma_b=gamma,
        species=(W.Species(Z=-1, alpha=alpha, ppc=2, sigma_par=1e-3, sigma_perp=1e-3),),
        plasma_mx=2, plasma_my=2, plasma_uth=0.005, dt=dt, seed=900 + i)


def test_batch_of_uneven_instances_fp64():
    """Uneven boxes (different nx, ny, nxi, alpha, gamma_b, dt) advanced as one
    batch: each member matches the same box run alone (1e-12) and the oracle."""
    import paper_2607_24214_amd as Q
    wls = [_scan_like(0, 32, 16, 20, 0.02, 50.0, 10.0),
           _scan_like(1, 16, 32, 12, 0.05, 200.0, 5.0),
           _scan_like(2, 64, 8, 28, 0.01, 30.0, 20.0)]
    sims, alone = [], []
    for wl in wls:
        plasma, beams = W.plasma_template(wl), W.beam(wl)
        for lst in (sims, alone):
            s = Q.Sim(Q.params_from_workload(wl, precision="f64"))
            s.load_plasma(plasma)
            s.load_beam(0, beams[0])
            lst.append(s)
    batch = Q.Batch(sims)
    batch.step(1)
    batch.sweep()
    batch.sync()
    for wl, sb, sa in zip(wls, sims, alone):
        sa.beam_step(1)
        sa.slice_sweep()
        got = {k: sb.fields(k) for k in OUT_FIELDS}
        ref1 = {k: sa.fields(k) for k in OUT_FIELDS}
        err, where = slice_errors(got, ref1)
        print(f"[batch] {wl.name}: member vs alone {err:.3e} at {where}", flush=True)
        assert err <= 1e-12, (wl.name, err, where)
        so, ref = run_oracle(wl, 1)
        err, where = slice_errors(got, ref)
        print(f"[batch] {wl.name}: member vs oracle {err:.3e} at {where}", flush=True)
        assert err <= 1e-10, (wl.name, err, where)

"""One beam step at a time with the beam work beside the slice loop
(QSA_OPT_BEAM_BESIDE): the source deposit runs a few slabs ahead of the slice loop and the
push a few slabs behind it, on a second stream.  It must give the fields,
sources and beam of deposit, sweep and push taken one after the other (only
the order of the deposit's additions differs), over slab counts that leave a
ragged last chunk, with several species, a beam in random order, particles
ahead of and behind the box, and in float32; and the oracle's after several
steps."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, run_oracle, slice_errors

pytestmark = pytest.mark.gpu

SRC_FIELDS = ("src_S", "src_Jx", "src_Jy", "src_Jz")
BEAM_KEYS = ("x", "y", "xi", "ux", "uy", "uz", "w")


def _sim(wl, beside, precision="f64", beams=None):
    import paper_2607_24214_amd as Q
    beams = beams if beams is not None else W.beam(wl)
    caps = [len(b["x"]) for b in beams]
    s = Q.Sim(Q.params_from_workload(wl, precision=precision, beam_capacity=caps))
    s.set_beam_beside(beside)
    s.load_plasma(W.plasma_template(wl))
    for k, b in enumerate(beams):
        s.load_beam(k, b)
    return s


def _fields(sim):
    return {k: sim.fields(k) for k in OUT_FIELDS + SRC_FIELDS}


def _compare(tag, a, b, tol_f, tol_b, n_species=1):
    err, where = slice_errors(_fields(a), _fields(b))
    print(f"[beside] {tag}: fields and sources {err:.3e} at {where}", flush=True)
    assert err <= tol_f, (tag, err, where)
    for s in range(n_species):
        ba, bb = a.read_beam(s), b.read_beam(s)
        for k in BEAM_KEYS:
            assert len(ba[k]) == len(bb[k]), (tag, s, k)
            d = float(np.abs(ba[k] - bb[k]).max()) if len(bb[k]) else 0.0
            scale = max(1.0, float(np.abs(bb[k]).max()) if len(bb[k]) else 1.0)
            assert d <= tol_b * scale, (tag, s, k, d)


@pytest.mark.parametrize("nxi", [8, 9, 16, 37])
def test_beside_matches_sequential_fp64(nxi):
    # 8 and 16 slabs: whole chunks (one chunk; the push of chunk 0 after
    # the loop); 9: a one-slab last chunk; 37: five chunks, the last ragged
    wl = W.small_3d(32, 32, nxi).with_(dt=20.0)
    a, b = _sim(wl, True), _sim(wl, False)
    for n in (1, 2):
        a.beam_step(n)
        b.beam_step(n)
        _compare(f"nxi={nxi} +{n} steps", a, b, 1e-10, 1e-11)


def test_beside_pair_rectangular_fp64():
    wl = W.small_3d(64, 16, 27).with_(
        species=(W.Species(Z=-1, alpha=0.03, ppc=2, sigma_perp=1e-2),
                 W.Species(Z=1, alpha=0.03, ppc=2, sigma_perp=1e-2)), dt=10.0)
    a, b = _sim(wl, True), _sim(wl, False)
    a.beam_step(3)
    b.beam_step(3)
    _compare("pair", a, b, 1e-10, 1e-11, n_species=2)


def test_beside_shuffled_and_outside_fp64():
    """Particles in random order (the key-range pushes gather through the
    permutation), a few ahead of the box (xi < 0: those within a cell of it
    go with slab 0, the others after the slice loop with the particles that
    left), in a warm beam."""
    wl = W.small_3d(32, 16, 21).with_(
        dt=20.0, species=(W.Species(Z=-1, alpha=0.05, ppc=2, sigma_par=1e-3, sigma_perp=1e-2),))
    beams = W.beam(wl)
    b0 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in beams[0].items()}
    n = len(b0["x"])
    rng = np.random.default_rng(17)
    ahead = rng.choice(n, size=64, replace=False)
    b0["xi"][ahead] = -rng.uniform(0.0, 3.0 * wl.dxi, size=64)   # some in (-dxi, 0), some further
    perm = rng.permutation(n)
    shuffled = [{k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in b0.items()}]
    a, b = _sim(wl, True, beams=shuffled), _sim(wl, False, beams=shuffled)
    for _ in range(3):
        a.beam_step(1)
        b.beam_step(1)
    _compare("shuffled, some ahead of the box", a, b, 1e-10, 1e-11)


def test_beside_fp32():
    wl = W.small_3d(32, 32, 29).with_(dt=20.0)
    a, b = _sim(wl, True, "f32"), _sim(wl, False, "f32")
    a.beam_step(3)
    b.beam_step(3)
    _compare("fp32", a, b, 1e-4, 1e-5)


def test_beside_matches_oracle_fp64():
    wl = W.small_3d(32, 32, 26).with_(dt=20.0)
    a = _sim(wl, True)
    a.beam_step(6)
    a.slice_sweep()
    got = {k: a.fields(k) for k in OUT_FIELDS}
    _, ref = run_oracle(wl, 6)
    err, where = slice_errors(got, ref)
    print(f"[beside] 6 steps vs oracle {err:.3e} at {where}", flush=True)
    assert err <= 1e-9, (err, where)


def test_beside_option_round_trip():
    import ctypes as C

    import paper_2607_24214_amd as Q
    wl = W.small_3d(16, 16, 8)
    s = Q.Sim(Q.params_from_workload(wl, beam_capacity=[len(b["x"]) for b in W.beam(wl)]))

    def get():
        v = C.c_int64(-1)
        assert s.lib.qsa_get_option(s.ctx, 5, C.byref(v)) == 0
        return int(v.value)

    default = get()
    assert default in (0, 1)
    s.set_beam_beside(True)
    assert get() == 1
    s.set_beam_beside(False)
    assert get() == 0
    assert s.lib.qsa_set_option(s.ctx, 5, 2) != 0   # only 0 or 1
    assert get() == 0


def test_beside_key_counts_survive_mixed_calls_fp64():
    """The pushes beside the slice loop count the next deposit's keys; any
    other path that moves the beam must drop those counts: beside steps
    mixed with steps taken one after the other (graph replay), a sweep on
    its own and a reload give what steps one after the other give."""
    wl = W.small_3d(32, 16, 21).with_(
        dt=20.0, species=(W.Species(Z=-1, alpha=0.05, ppc=2, sigma_par=1e-3, sigma_perp=1e-2),))
    a, b = _sim(wl, True), _sim(wl, False)
    plan = [("beside", 2), ("seq", 1), ("beside", 1), ("sweep", 0), ("beside", 1), ("seq", 2), ("beside", 1)]
    for what, n in plan:
        if what == "sweep":
            a.slice_sweep()
            b.slice_sweep()
            continue
        a.set_beam_beside(what == "beside")
        a.beam_step(n)
        b.beam_step(n)
    _compare("mixed calls", a, b, 1e-10, 1e-11)
    # a reload in between: the counts of the old beam must not be used
    beams = W.beam(wl.with_(seed=wl.seed + 1))
    a.set_beam_beside(True)
    a.beam_step(1)
    for k, bb in enumerate(beams):
        a.load_beam(k, bb)
        b.load_beam(k, bb)
    a.beam_step(2)
    b.beam_step(2)
    _compare("after a reload", a, b, 1e-10, 1e-11)


@pytest.mark.parametrize("blocks", [1, 7, 64])
def test_beside_capped_grids_fp64(blocks):
    """QSA_OPT_BESIDE_BLOCKS caps the deposit and push launches beside the
    slice loop: each workgroup loops over several rows or particle ranges."""
    wl = W.small_3d(32, 32, 19).with_(dt=20.0)
    a, b = _sim(wl, True), _sim(wl, False)
    a.set_beside_blocks(blocks)
    a.beam_step(2)
    b.beam_step(2)
    _compare(f"beside blocks {blocks}", a, b, 1e-10, 1e-11)

"""Storage re-sort of the beam by deposit key (QSA_OPT_RESORT_EVERY, one step
at a time): the step after a re-sort finds the particles stored in key order
(cell row, slab-major: the order the deposit gathers them in), the fields and
particles match a context that never re-sorts (particles matched by their
weights, which the push leaves unchanged and the test makes distinct), with
the beam work after the sweep and beside it, in float64 and float32; the
setting is refused where it cannot apply."""
import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, slice_errors

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "xi", "ux", "uy", "uz", "w")


def _workload():
    return W.small_3d(32, 16, 21).with_(
        dt=20.0, species=(W.Species(Z=-1, alpha=0.03, ppc=2, sigma_perp=1e-2),
                          W.Species(Z=1, alpha=0.03, ppc=2, sigma_perp=1e-2)))


def _shuffled_tagged(wl, s, seed):
    """The species' beam in a random order, 48 particles moved ahead of the
    box (some within a cell of it, which deposit into slab 0, the others
    outside) and none within three cells of its back, each weight scaled by a distinct factor 1 + k 2^-20 (distinct
    in float32 too) so that it names its particle."""
    b = W.beam(wl)[s]
    rng = np.random.default_rng(seed)
    n = len(b["x"])
    order = rng.permutation(n)
    out = {k: np.ascontiguousarray(v[order]) for k, v in b.items()}
    ahead = rng.choice(n, size=48, replace=False)
    out["xi"][ahead] = -rng.uniform(0.0, 3.0 * wl.dxi, size=48)
    # three cells clear of the back edge, where the push retires particles
    # (weight 0, which would no longer name them)
    out["xi"] = np.minimum(out["xi"], (wl.nxi - 4) * wl.dxi)
    out["w"] = out["w"] * (1.0 + rng.permutation(n).astype(np.float64) * 2.0 ** -20)
    return out


def _sim(wl, precision, resort, beside=False):
    import paper_2607_24214_amd as Q
    s = Q.Sim(Q.params_from_workload(wl, precision=precision, pipeline=1))
    s.load_plasma(W.plasma_template(wl))
    if resort:
        s.set_resort_every(resort)
    if beside:
        s.set_beam_beside(True)
    return s


def _host_keys(wl, b, precision):
    """Deposit key of each particle, in the library's arithmetic: slab
    floor(xi/dxi) (xi in float64; slab 0 also for xi in (-dxi, 0)), cell row
    and group of eight cells along x from x, y in the working precision,
    slab-major; past every cell's key for a particle outside the box."""
    ft = np.float32 if precision == "f32" else np.float64
    nxc = wl.nx // 8 if wl.nx >= 8 else 1
    gz = b["xi"] * (1.0 / wl.dxi)
    out = ~((gz > -1.0) & (gz < wl.nxi))
    j = np.maximum(np.floor(gz), 0).astype(np.int64)
    i = np.mod(np.floor(b["x"].astype(ft) * ft(1.0 / wl.dx)).astype(np.int64), wl.nx)
    l = np.mod(np.floor(b["y"].astype(ft) * ft(1.0 / wl.dy)).astype(np.int64), wl.ny)
    k = (j * wl.ny + l) * nxc + i // 8
    k[out] = wl.nxi * wl.ny * nxc
    return k


def _match(a, b):
    """b's particles in a's order, matched by weight (a may hold b's weights
    rounded to float32, which keeps their order)."""
    ia, ib = np.argsort(a["w"], kind="stable"), np.argsort(b["w"], kind="stable")
    assert np.allclose(a["w"][ia], b["w"][ib], rtol=1e-6, atol=0.0)
    inv = np.empty_like(ia)
    inv[ia] = np.arange(len(ia))
    return {k: v[ib][inv] for k, v in b.items()}


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_step_after_resort_sees_key_order(precision):
    wl = _workload()
    sim = _sim(wl, precision, resort=1)
    beams = [_shuffled_tagged(wl, s, 10 + s) for s in range(2)]
    for s, b in enumerate(beams):
        sim.load_beam(s, b)
    sim.beam_step(1)   # the first step after a load re-sorts before it runs
    for s, b in enumerate(beams):
        got = sim.read_beam(s)
        before = _match(got, b)   # each stored particle as it was loaded
        assert np.abs(got["xi"] - before["xi"]).max() <= 0.5 * wl.dxi   # one step moved them little
        k = _host_keys(wl, before, precision)
        bad = int(np.sum(np.diff(k) < 0))
        print(f"[resort] {precision} species {s}: {len(k)} particles, {bad} out of key order", flush=True)
        assert bad == 0
        assert k[-1] == wl.nxi * wl.ny * (wl.nx // 8)   # the particles outside the box last


@pytest.mark.parametrize("precision,tol_f,tol_b", [("f64", 1e-10, 1e-11), ("f32", 1e-4, 1e-5)])
@pytest.mark.parametrize("every,beside", [(1, False), (2, False), (1, True)])
def test_resorted_run_matches_plain(precision, tol_f, tol_b, every, beside):
    wl = _workload()
    plain = _sim(wl, precision, resort=0, beside=beside)
    sorted_ = _sim(wl, precision, resort=every, beside=beside)
    for s in range(2):
        b = _shuffled_tagged(wl, s, 20 + s)
        plain.load_beam(s, b)
        sorted_.load_beam(s, b)
    plain.beam_step(3)
    sorted_.beam_step(3)
    plain.slice_sweep()
    sorted_.slice_sweep()
    err, where = slice_errors({k: sorted_.fields(k) for k in OUT_FIELDS},
                              {k: plain.fields(k) for k in OUT_FIELDS})
    print(f"[resort] {precision} every {every} beside {beside}: field error {err:.3e} at {where}", flush=True)
    assert err <= tol_f, (err, where)
    for s in range(2):
        a = sorted_.read_beam(s)
        b = _match(a, plain.read_beam(s))
        for k in KEYS:
            scale = max(1.0, np.abs(b[k]).max())
            assert np.abs(a[k] - b[k]).max() <= tol_b * scale, (s, k)


def test_resort_setting_rules():
    import paper_2607_24214_amd as Q
    wl = _workload()
    sim = _sim(wl, "f64", resort=0)
    with pytest.raises(Q.QSAError):
        sim.set_resort_every(-1)
    sim.set_resort_every(4)
    sim.set_resort_every(0)
    # steps in flight: the beam is sorted by cell row already
    piped = Q.Sim(Q.params_from_workload(wl, pipeline=3))
    with pytest.raises(Q.QSAError):
        piped.set_resort_every(1)
    # a capacity whose float64 copy exceeds the sources and fields it would use
    n_fit = (4 + 7) * wl.nxi * wl.nx * wl.ny
    big = Q.Sim(Q.params_from_workload(wl, beam_capacity=[n_fit + 1, 16], pipeline=1))
    with pytest.raises(Q.QSAError):
        big.set_resort_every(1)
    ok = Q.Sim(Q.params_from_workload(wl, beam_capacity=[n_fit, 16], pipeline=1))
    ok.set_resort_every(1)

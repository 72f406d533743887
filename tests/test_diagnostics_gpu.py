"""Device diagnostics (qsa_field_moments, qsa_beam_moments) against the
oracle's definitions: on the library's own fields and beam (the reductions
alone, float64 summation order only), and on the oracle's run (through the
field parity of the sweep)."""
import numpy as np
import pytest

import qsa_workloads as W
from oracle import diagnostics as D
from tests.helpers import run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _rel(a, b):
    scale = max(float(np.abs(b).max()), 1e-300)
    return float(np.abs(a - b).max()) / scale


def _gpu_out(sim):
    return {k: sim.fields(k) for k in D.FIELDS}


@pytest.mark.parametrize("window", [1, 3, 64])
def test_field_moments_match_definition_fp64(window):
    """40 slices with 2 beam steps; windows of 1, 3 (the last one of one
    slice) and 64 slices (one window, wider than the box)."""
    wl = W.small_3d(32, 32, 40).with_(dt=20.0)
    sim, _ = run_gpu(wl, steps=2, precision="f64")
    got = sim.field_moments(window)
    per = D.field_slice_means(_gpu_out(sim))
    ref = D.windows(per, 1.0, float(window)) / D.window_counts(per.shape[0], 1.0, float(window))[:, None]
    assert got.shape == ref.shape
    err = _rel(got, ref)
    print(f"[diag] field moments, window {window}: {err:.2e}", flush=True)
    assert err <= 1e-12, err
    assert np.all(got[:, 5] > 0)   # B_z is driven by the beam current


def test_beam_moments_match_definition_fp64():
    wl = W.small_3d(32, 32, 40).with_(dt=20.0)
    sim, _ = run_gpu(wl, steps=2, precision="f64")
    for window in (1, 5):
        got = sim.beam_moments(0, window)
        per = D.beam_slice_sums(sim.read_beam(0), wl.dxi, wl.nxi)
        ref = D.windows(per, wl.dxi, window * wl.dxi)
        for k in range(7):
            err = _rel(got[:, k], ref[:, k])
            assert err <= 1e-12, (window, D.BEAM_SUMS[k], err)
    sp = D.momentum_spread(sim.beam_moments(0, 8), wl.dxi, 8 * wl.dxi)
    assert np.all(np.isfinite(sp[:, :2]))


def test_pair_beam_moments_per_species_fp64():
    wl = W.small_3d(64, 16, 20).with_(
        species=(W.Species(Z=-1, alpha=0.03, ppc=2, sigma_perp=1e-2),
                 W.Species(Z=1, alpha=0.03, ppc=2, sigma_perp=1e-2)), dt=10.0)
    sim, _ = run_gpu(wl, steps=1, precision="f64")
    for s in range(2):
        got = sim.beam_moments(s, 2)
        ref = D.windows(D.beam_slice_sums(sim.read_beam(s), wl.dxi, wl.nxi), wl.dxi, 2 * wl.dxi)
        assert _rel(got, ref) <= 1e-12, s


def test_field_moments_against_oracle_run_fp64():
    """Through the sweep: the oracle's fields give the same moments to the
    field parity of the sweep."""
    wl = W.small_3d(32, 16, 24)
    sim, _ = run_gpu(wl, steps=1, precision="f64")
    _, ref_f = run_oracle(wl, steps=1)
    ref = D.field_slice_means(ref_f)
    got = sim.field_moments(1)
    err = _rel(got, ref)
    print(f"[diag] field moments vs oracle run: {err:.2e}", flush=True)
    assert err <= 1e-9, err


def test_moments_fp32_and_on_device():
    import torch
    wl = W.small_3d(32, 32, 24).with_(dt=20.0)
    sim, _ = run_gpu(wl, steps=1, precision="f32")
    per = D.field_slice_means(_gpu_out(sim))
    got = sim.field_moments(1)
    assert _rel(got, per) <= 1e-6
    dev = sim.field_moments(1, on_device=True)
    assert isinstance(dev, torch.Tensor) and dev.is_cuda
    assert _rel(dev.cpu().numpy(), got) <= 1e-12
    bm = sim.beam_moments(0, 4)
    ref = D.windows(D.beam_slice_sums(sim.read_beam(0), wl.dxi, wl.nxi), wl.dxi, 4 * wl.dxi)
    assert _rel(bm, ref) <= 1e-6


def test_moment_errors():
    import paper_2607_24214_amd as Q
    wl = W.small_3d(16, 16, 8)
    sim = Q.Sim(Q.params_from_workload(wl, precision="f64", beam_capacity=[len(W.beam(wl)[0]["x"])]))
    sim.load_plasma(W.plasma_template(wl))
    sim.load_beam(0, W.beam(wl)[0])
    with pytest.raises(Q.QSAError, match="STATE"):
        sim.field_moments(1)            # no sweep yet
    sim.slice_sweep()
    with pytest.raises(Q.QSAError, match="INVALID"):
        sim.field_moments(0)
    with pytest.raises(Q.QSAError, match="INVALID"):
        sim.beam_moments(0, -2)
    with pytest.raises(Q.QSAError, match="INVALID"):
        sim.beam_moments(3, 1)          # one species only
    assert sim.field_moments(8).shape == (1, 6)

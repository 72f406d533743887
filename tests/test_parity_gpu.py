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

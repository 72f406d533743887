"""The C ABI: libqsa.so loads and exports every entry point include/qsa.h
declares; host-side validation answers without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsa.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(qsa_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("qsa_create", "qsa_slice_sweep", "qsa_beam_step", "qsa_fields",
                 "qsa_workspace_bytes", "qsa_load_plasma", "qsa_load_beam", "qsa_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def _params(**kw):
    from paper_2607_24214_amd import make_params
    base = dict(nx=64, ny=1, nxi=128, dx=0.1, dy=0.1, dxi=0.1, dt=5.0,
                species=[(-1, 1.0)], n_plasma=256, plasma_w=0.0025, beam_capacity=[65024])
    base.update(kw)
    return make_params(**base)


def test_workspace_bytes_validates_parameters():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    ok = lib.qsa_workspace_bytes(C.byref(_params()))
    assert ok > 0
    # fields (7) + sources (4) per slice, float64, plus the beam: a lower bound
    assert ok >= (7 + 4) * 128 * 64 * 8 + 65024 * 7 * 8
    for bad in (dict(nx=48), dict(nx=4), dict(ny=2), dict(nxi=1), dict(dt=0.0),
                dict(dx=-1.0), dict(n_plasma=0), dict(plasma_w=0.0), dict(species=[]),
                dict(n_corr=-1), dict(kappa2=0.0), dict(nx=1024)):
        kw = dict(bad)
        if "species" in kw:
            kw["beam_capacity"] = []
        assert lib.qsa_workspace_bytes(C.byref(_params(**kw))) == 0, bad
    f32 = lib.qsa_workspace_bytes(C.byref(_params(precision="f32")))
    assert f32 < ok


def test_create_rejects_without_touching_the_device():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    p = _params()
    ctx = C.c_void_p()
    assert lib.qsa_create(C.byref(_params(nx=3)), C.c_void_p(256), 1 << 30, None, C.byref(ctx)) == -1
    assert lib.qsa_create(C.byref(p), None, 1 << 30, None, C.byref(ctx)) == -1
    assert lib.qsa_create(C.byref(p), C.c_void_p(257), 1 << 30, None, C.byref(ctx)) == -1
    need = lib.qsa_workspace_bytes(C.byref(p))
    assert lib.qsa_create(C.byref(p), C.c_void_p(256), need - 1, None, C.byref(ctx)) == -2
    assert lib.qsa_status_string(-4).decode().startswith("quasistatic breakdown")


def test_pipeline_workspace_and_validation():
    """Steps in flight hold one working set each (sources, fields, plasma
    state) and a copy of the beam; depth 0 and 1 mean the same."""
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    one = lib.qsa_workspace_bytes(C.byref(_params()))
    assert lib.qsa_workspace_bytes(C.byref(_params(pipeline=0))) == one
    four = lib.qsa_workspace_bytes(C.byref(_params(pipeline=4)))
    # three more sets of fields (7) and sources (4), and the beam copy
    assert four >= one + 3 * (7 + 4) * 128 * 64 * 8 + 65024 * 7 * 8
    assert lib.qsa_workspace_bytes(C.byref(_params(pipeline=16))) > four
    assert lib.qsa_workspace_bytes(C.byref(_params(pipeline=17))) == 0
    assert lib.qsa_workspace_bytes(C.byref(_params(pipeline=-1))) == 0
    p = _params()
    p.adjoint_steps = -1
    assert lib.qsa_workspace_bytes(C.byref(p)) == 0
    p.adjoint_steps = 2
    # the beam (7 arrays) and the fields (7 planes) of 3 steps, at least
    assert lib.qsa_workspace_bytes(C.byref(p)) >= one + 3 * (7 * 128 * 64 * 8 + 65024 * 7 * 8)
    v = C.c_int64()
    assert lib.qsa_get_option(None, 1, C.byref(v)) == -1


def test_autotune_rejects_null_context():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    ms = C.c_double()
    assert lib.qsa_autotune(None, C.byref(ms)) == -1


def test_linear_model_rejects_bad_arguments_without_a_launch():
    """qsa_linear_model checks its arguments on the host before any launch."""
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    taus = (C.c_double * 2)(0.0, 1.0)
    null = C.c_void_p(0)
    dummy = C.c_void_p(16)
    assert lib.qsa_linear_model(0, 10, 0.1, 0.1, dummy, 0, dummy, 2, taus, dummy, dummy, null) == -1
    assert lib.qsa_linear_model(1, 4097, 0.1, 0.1, dummy, 0, dummy, 2, taus, dummy, dummy, null) == -1
    assert lib.qsa_linear_model(1, 10, 0.0, 0.1, dummy, 0, dummy, 2, taus, dummy, dummy, null) == -1
    assert lib.qsa_linear_model(1, 10, 0.1, -1.0, dummy, 0, dummy, 2, taus, dummy, dummy, null) == -1
    assert lib.qsa_linear_model(1, 10, 0.1, 0.1, null, 0, dummy, 2, taus, dummy, dummy, null) == -1
    assert lib.qsa_linear_model(1, 10, 0.1, 0.1, dummy, 0, dummy, 257, taus, dummy, dummy, null) == -1
    back = (C.c_double * 2)(1.0, 0.5)
    assert lib.qsa_linear_model(1, 10, 0.1, 0.1, dummy, 0, dummy, 2, back, dummy, dummy, null) == -1
    assert lib.qsa_linear_model(1, 10, 0.1, 0.1, dummy, 2, dummy, 2, taus, dummy, dummy, null) == -1


def test_static_batch_sweep_rejects_null_and_empty():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    assert lib.qsa_batch_sweep_static(None, 1, None) == -1
    arr = (C.c_void_p * 1)(None)
    assert lib.qsa_batch_sweep_static(arr, 0, None) == -1
    assert lib.qsa_batch_sweep_static(arr, 1, None) == -1


def test_checkpoint_stride_validated():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    ok = _params(adjoint_steps=2, ckpt_every=8)
    assert lib.qsa_workspace_bytes(C.byref(ok)) > 0
    small = lib.qsa_workspace_bytes(C.byref(_params(adjoint_steps=2, ckpt_every=64)))
    big = lib.qsa_workspace_bytes(C.byref(_params(adjoint_steps=2, ckpt_every=4)))
    assert big != small       # checkpoint and segment storage follow the stride
    assert lib.qsa_workspace_bytes(C.byref(_params(adjoint_steps=2, ckpt_every=-1))) == 0
    assert lib.qsa_workspace_bytes(C.byref(_params(adjoint_steps=2, ckpt_every=129))) == 0


def test_guide_field_validated():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    assert lib.qsa_workspace_bytes(C.byref(_params(b0z=0.5))) == lib.qsa_workspace_bytes(C.byref(_params()))
    assert lib.qsa_workspace_bytes(C.byref(_params(b0z=float("inf")))) == 0
    assert lib.qsa_workspace_bytes(C.byref(_params(b0z=float("nan")))) == 0
    # the adjoint takes no external field
    assert lib.qsa_workspace_bytes(C.byref(_params(adjoint_steps=2, b0z=0.5))) == 0
    assert lib.qsa_workspace_bytes(C.byref(_params(adjoint_steps=2))) > 0


def test_mobile_ions_validated():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    assert lib.qsa_workspace_bytes(C.byref(_params(ion_m=4.0, plasma_weights=True))) > 0
    assert lib.qsa_workspace_bytes(C.byref(_params(ion_m=4.0))) == 0             # needs plasma_weights
    assert lib.qsa_workspace_bytes(C.byref(_params(ion_m=-1.0, plasma_weights=True))) == 0
    assert lib.qsa_workspace_bytes(C.byref(_params(ion_m=float("inf"), plasma_weights=True))) == 0
    assert lib.qsa_workspace_bytes(C.byref(_params(ion_m=4.0, ion_z=0, plasma_weights=True))) == 0
    assert lib.qsa_workspace_bytes(C.byref(_params(ion_m=4.0, ion_z=65, plasma_weights=True))) == 0

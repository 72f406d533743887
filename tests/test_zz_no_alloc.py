"""qsa_batch_sweep_static, the entry point for callers that cannot allocate
device memory: the lane table of its batched sweep lives in the library's
static device array instead of a batch workspace.  Its fields equal those of
qsa_batch_sweep on the same members, on two calls in a row, the second with
fewer and smaller boxes (the array keeps the first call's descriptors)."""
import ctypes as C

import numpy as np
import pytest

import qsa_workloads as W
from tests.helpers import OUT_FIELDS, slice_errors

pytestmark = pytest.mark.gpu


def _members(wls, precision):
    import paper_2607_24214_amd as Q
    sims = []
    for wl in wls:
        beams = W.beam(wl)
        s = Q.Sim(Q.params_from_workload(wl, precision=precision, beam_capacity=[len(b["x"]) for b in beams]))
        s.load_plasma(W.plasma_template(wl))
        for k, b in enumerate(beams):
            s.load_beam(k, b)
        sims.append(s)
    return sims


def _static(sims):
    """The C ABI call itself (ctypes), on the members' stream."""
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    arr = (C.c_void_p * len(sims))(*[s.ctx.value for s in sims])
    st = lib.qsa_batch_sweep_static(arr, len(sims), C.c_void_p(sims[0].stream.cuda_stream))
    assert st == 0, lib.qsa_last_error(sims[0].ctx).decode()


def _fields(sims):
    return [{k: s.fields(k) for k in OUT_FIELDS} for s in sims]


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_static_sweep_equals_batch_sweep_on_two_calls(precision, tol):
    import paper_2607_24214_amd as Q
    calls = [
        [W.small_3d(32, 16, 24), W.small_3d(16, 32, 12, seed=9), W.small_3d(64, 64, 20, seed=11)],
        [W.small_3d(16, 16, 10, seed=13), W.small_3d(32, 8, 16, seed=15)],
    ]
    for n, wls in enumerate(calls):
        print(f"[no-alloc] {precision} call {n}: {[w.name for w in wls]}", flush=True)
        ref_sims = _members(wls, precision)
        batch = Q.Batch(ref_sims)
        batch.sweep()
        batch.sync()
        ref = _fields(ref_sims)
        batch.close()
        sims = _members(wls, precision)
        _static(sims)
        for s in sims:
            s.sync()
        got = _fields(sims)
        for wl, a, b in zip(wls, got, ref):
            err, where = slice_errors(a, b)
            print(f"[no-alloc] {precision} call {n} {wl.name}: static vs batch {err:.3e} at {where}", flush=True)
            assert err <= tol, (wl.name, err, where)
            assert all(np.isfinite(v).all() for v in a.values())
        del sims, ref_sims


def test_static_sweep_rejects_too_many_or_repeated_contexts():
    from paper_2607_24214_amd import _lib as L
    lib = L.lib()
    (s,) = _members([W.small_3d(16, 16, 8)], "f64")
    too_many = (C.c_void_p * (L.QSA_STATIC_MAX_CTX + 1))(*([s.ctx.value] * (L.QSA_STATIC_MAX_CTX + 1)))
    assert lib.qsa_batch_sweep_static(too_many, L.QSA_STATIC_MAX_CTX + 1, None) == -1
    assert str(L.QSA_STATIC_MAX_CTX) in lib.qsa_last_error(s.ctx).decode()
    twice = (C.c_void_p * 2)(s.ctx.value, s.ctx.value)
    assert lib.qsa_batch_sweep_static(twice, 2, None) == -1
    assert lib.qsa_batch_sweep_static(None, 1, None) == -1

"""The seeded input generators (shared by the oracle and the GPU tests):
random macro-particle weights keep everything else of the loading and the
mean weight."""
import numpy as np

import qsa_workloads as W


def test_random_weights_only_change_weights():
    base = W.small_3d(16, 16, 10).with_(species=(W.Species(Z=-1, alpha=0.05, ppc=4, sigma_perp=1e-3),))
    rnd = base.with_(species=(W.Species(Z=-1, alpha=0.05, ppc=4, sigma_perp=1e-3, w_spread=0.5),))
    a, b = W.beam(base)[0], W.beam(rnd)[0]
    for k in ("x", "y", "xi", "ux", "uy", "uz"):
        assert np.array_equal(a[k], b[k]), k
    w0 = a["w"][0]
    assert np.all(a["w"] == w0)
    r = b["w"] / w0
    assert r.min() >= 0.5 and r.max() < 1.5
    assert abs(r.mean() - 1.0) < 4 * 0.5 / np.sqrt(3 * r.size)    # 4 sigma of the mean of U(0.5, 1.5)
    # the first K slices of the full beam are the beam of the first K slices
    c = W.beam(rnd, 0, 3)[0]
    assert np.array_equal(c["w"], b["w"][:c["w"].size])

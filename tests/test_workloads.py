"""The seeded input generators (shared by the oracle and the GPU tests):
random macro-particle weights keep everything else of the loading and the
mean weight; longitudinal ramps scale the weights by the density profile."""
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


def test_longitudinal_ramps_scale_weights_by_the_profile():
    """Head and tail ramps: weights are the flat-top weights times the
    profile (0 at the head, 1 on the plateau, 0 at the beam's end), and the
    particles themselves are unchanged; the charge per slice follows the
    profile's slice averages."""
    sp = dict(Z=-1, alpha=0.05, ppc=4, sigma_perp=1e-3)
    base = W.small_3d(8, 8, 41).with_(species=(W.Species(**sp),))
    ramp = base.with_(species=(W.Species(**sp, ramp_head=1.0, ramp_tail=0.5),))
    a, b = W.beam(base)[0], W.beam(ramp)[0]
    for k in ("x", "y", "xi", "ux", "uy", "uz"):
        assert np.array_equal(a[k], b[k]), k
    f = b["w"] / a["w"]
    xi = a["xi"]
    end = ramp.beam_slices * ramp.dxi
    assert np.allclose(f, np.clip(np.minimum(np.minimum(xi / 1.0, (end - xi) / 0.5), 1.0), 0.0, 1.0), rtol=0, atol=1e-15)
    assert np.all(f[(xi > 1.0) & (xi < end - 0.5)] == 1.0)
    # per slice: mean relative weight ~ the profile at the slice centre (linear inside a slice)
    j = np.floor(xi / ramp.dxi).astype(int)
    for jj in (0, 3, 9, 20, 37, 39):
        m = f[j == jj].mean()
        c = min(1.0, (jj + 0.5) * ramp.dxi / 1.0, (end - (jj + 0.5) * ramp.dxi) / 0.5)
        assert abs(m - c) < 0.05, (jj, m, c)
    # a range of slices is the same as the full beam's slices
    c3 = W.beam(ramp, 2, 5)[0]
    n_slice = ramp.n_perp * 4
    assert np.array_equal(c3["w"], b["w"][2 * n_slice:5 * n_slice])

"""The seeded workload generators: resolution independence, windows and the
stated statistics (they carry no part of the kinetic method)."""
import numpy as np

from paper_2603_13618_amd import inputs


def test_spectral_noise_unit_variance_zero_mean():
    rho, ux, uy = inputs.smooth_random(64, seed=0, cutoff=16)
    for f, scale, off in ((rho, 0.01, 1.0), (ux, 0.03, 0.0), (uy, 0.03, 0.0)):
        n = (f - off) / scale
        assert abs(n.mean()) < 1e-12
        assert abs(n.var() - 1.0) < 1e-12


def test_spectral_noise_same_field_at_every_resolution_and_window():
    a = inputs.smooth_random(64, seed=3, cutoff=8)
    b = inputs.smooth_random(128, seed=3, cutoff=8)
    for fa, fb in zip(a, b):
        np.testing.assert_allclose(fb[::2, ::2], fa, rtol=0, atol=1e-14)
    w = inputs.smooth_random(128, seed=3, cutoff=8, window=(120, 5, 20, 7))
    for fw, fb in zip(w, b):
        ref = np.roll(np.roll(fb, -5, 0), -120, 1)[:7, :20]
        np.testing.assert_allclose(fw, ref, rtol=0, atol=1e-14)


def test_double_shear_layer_formula():
    rho, ux, uy = inputs.double_shear_layer(8)
    y = np.arange(8) / 8
    assert (rho == 1).all()
    np.testing.assert_allclose(ux[:, 0], np.where(y < 0.5, 0.05 * np.tanh(80 * (y - 0.25)),
                                                  0.05 * np.tanh(80 * (0.75 - y))))
    np.testing.assert_allclose(uy[0], 0.0025 * np.sin(2 * np.pi * (np.arange(8) / 8 + 0.25)))


def test_riemann_quadrants_ranges_and_window():
    rho, ux, uy, T, states = inputs.riemann_quadrants(16, seed=0)
    assert len(states) == 4
    for r, a, b, t in states:
        assert 0.5 <= r <= 1.5 and np.hypot(a, b) <= 0.1 and 0.9 <= t <= 1.1
    assert rho[15, 15] == states[0][0] and rho[15, 0] == states[1][0]
    assert rho[0, 0] == states[2][0] and rho[0, 15] == states[3][0]
    w = inputs.riemann_quadrants(16, seed=0, window=(6, 3, 5, 9))
    np.testing.assert_array_equal(w[0], rho[3:12, 6:11])
    dt = inputs.riemann_dt(states, 1 / 2048)
    assert 2e-6 < dt < 5e-6

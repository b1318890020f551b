"""Pins of the exact 1D Riemann solver (the inviscid reference of the shock
tube): the jump conditions every wave must satisfy, not stored values.
Shocks satisfy Rankine-Hugoniot (mass, momentum and energy fluxes equal in
the shock frame); rarefactions keep the entropy p/rho^gamma and the Riemann
invariant u +- 2c/(gamma - 1); pressure and velocity are continuous across
the contact; uniform data stay uniform; mirrored data give the mirrored
solution."""
import math

import numpy as np
import pytest

from oracle import riemann_exact as rx

G = 1.4
SOD = ((1.0, 1.0, 0.0), (0.125, 0.1, 0.0))


def _state(left, right, xi):
    r, u, p = rx.sample(left, right, np.array([xi]), G)
    return r[0], u[0], p[0]


def _fluxes(r, u, p, s):
    """Mass, momentum and energy fluxes in the frame moving at s."""
    E = p / (G - 1.0) + 0.5 * r * u * u
    return np.array([r * (u - s), r * u * (u - s) + p, E * (u - s) + p * u])


def _rh_residual(left, right, s, eps=1e-9):
    a = _state(left, right, s - eps)
    b = _state(left, right, s + eps)
    fa, fb = _fluxes(*a, s), _fluxes(*b, s)
    return np.abs(fa - fb).max() / np.abs(fa).max(), a, b


def test_sod_wave_structure_and_jump_conditions():
    w = rx.wave_speeds(*SOD, G)
    ps, us = rx.star_state(*SOD, G)
    assert w["left"][0] < w["left"][1] < w["contact"] < w["right"][0] == w["right"][1]
    assert SOD[1][1] < ps < SOD[0][1] and us > 0          # rarefaction left, shock right
    res, a, b = _rh_residual(*SOD, w["right"][0])
    assert res < 1e-12 and b[0] == SOD[1][0] and a[0] > b[0]   # compressive shock
    # the fan: entropy and the left Riemann invariant are those of the left state
    xs = np.linspace(w["left"][0] + 1e-9, w["left"][1] - 1e-9, 17)
    r, u, p = rx.sample(*SOD, xs, G)
    rl, pl, ul = SOD[0]
    c = np.sqrt(G * p / r)
    assert np.abs(p / r ** G - pl / rl ** G).max() < 1e-13
    assert np.abs(u + 2 * c / (G - 1) - (ul + 2 * math.sqrt(G * pl / rl) / (G - 1))).max() < 1e-13
    # the star region behind the fan keeps the left entropy
    rs, _, _ = _state(*SOD, 0.5 * (w["left"][1] + w["contact"]))
    assert abs(ps / rs ** G - pl / rl ** G) < 1e-13
    # contact: p and u continuous, rho jumps
    a = _state(*SOD, us - 1e-9)
    b = _state(*SOD, us + 1e-9)
    assert a[1] == pytest.approx(b[1], abs=1e-14) and a[2] == pytest.approx(b[2], abs=1e-14)
    assert a[0] > b[0]


def test_uniform_data_stay_uniform():
    s = (0.7, 0.4, 0.3)
    r, u, p = rx.sample(s, s, np.linspace(-3, 3, 41), G)
    assert np.allclose(r, 0.7, rtol=1e-13) and np.allclose(u, 0.3, atol=1e-13)
    assert np.allclose(p, 0.4, rtol=1e-13)


def test_mirror_symmetry():
    left, right = (1.0, 1.0, 0.2), (0.3, 0.2, -0.1)
    ml, mr = (right[0], right[1], -right[2]), (left[0], left[1], -left[2])
    xi = np.linspace(-2.5, 2.5, 101)
    r1, u1, p1 = rx.sample(left, right, xi, G)
    r2, u2, p2 = rx.sample(ml, mr, -xi, G)
    # away from the waves themselves (the side a sample point at a
    # discontinuity falls on is a convention)
    w = rx.wave_speeds(left, right, G)
    edges = [w["left"][0], w["left"][1], w["contact"], w["right"][0], w["right"][1]]
    ok = np.min(np.abs(xi[:, None] - np.array(edges)[None, :]), axis=1) > 1e-6
    assert np.allclose(r1[ok], r2[ok], rtol=1e-12) and np.allclose(p1[ok], p2[ok], rtol=1e-12)
    assert np.allclose(u1[ok], -u2[ok], atol=1e-12)


def test_colliding_streams_make_two_shocks():
    left, right = (1.0, 1.0, 1.0), (1.0, 1.0, -1.0)
    ps, us = rx.star_state(left, right, G)
    assert abs(us) < 1e-14 and ps > 1.0
    w = rx.wave_speeds(left, right, G)
    assert w["left"][0] == pytest.approx(-w["right"][0], rel=1e-13)
    for s in (w["left"][0], w["right"][0]):
        assert _rh_residual(left, right, s)[0] < 1e-12


def test_receding_streams_make_two_rarefactions():
    left, right = (1.0, 1.0, -0.5), (1.0, 1.0, 0.5)
    ps, us = rx.star_state(left, right, G)
    assert abs(us) < 1e-14 and ps < 1.0
    # isentropic throughout
    r, u, p = rx.sample(left, right, np.linspace(-2, 2, 81), G)
    assert np.abs(p / r ** G - 1.0).max() < 1e-12


def test_vacuum_is_reported():
    with pytest.raises(ValueError):
        rx.star_state((1.0, 1.0, -10.0), (1.0, 1.0, 10.0), G)

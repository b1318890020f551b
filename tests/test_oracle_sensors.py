"""Pins of the oracle's sensors and flags against closed forms.

Sensors (Sec. III): S_KL (eq. HKL-sensor, f term), S_NEQ (eq. sensor-neq-kin,
f term), S_PI (eq. sensor-TauNS-kin, Frobenius norm), S_Q (eq.
sensor-qNSF-kin-ryk with g = 0); positivity caveat (Sec. III.C).
"""
import numpy as np
import pytest

from paper_2603_13618_amd import inputs


def _invariant_free(orc, q, seed, energy):
    """Random population perturbation with zero mass and momentum (and energy),
    i.e. orthogonal to the collision invariants in the plain dot product."""
    vx, vy, _ = orc.lattice(q)
    cols = [np.ones(q), vx, vy] + ([0.5 * (vx ** 2 + vy ** 2)] if energy else [])
    A = np.stack(cols, 1)
    r = inputs.perturbation(q, seed, 1.0)
    h = r - A @ np.linalg.lstsq(A, r, rcond=None)[0]
    assert np.abs(A.T @ h).max() < 1e-13
    return h


@pytest.mark.parametrize("q", [9, 25])
def test_sensors_vanish_at_equilibrium(orc, q):
    args = inputs.random_state((6, 5), 4, (0.7, 1.3), 0.1, (0.9, 1.1) if q == 25 else None)
    f = orc.equilibrium(q, *args)
    s, nf = orc.sensors(q, f)
    assert nf == 0
    assert np.abs(s[0]).max() < 1e-28       # second order in the round-off of the moments
    assert np.abs(s[1]).max() < 1e-14
    assert np.abs(s[2]).max() < 1e-14
    assert np.abs(s[3]).max() < 1e-14


@pytest.mark.parametrize("q", [9, 25])
def test_kl_small_perturbation_closed_form(orc, q):
    # f = feq + eps h with invariant-free h keeps the moments, so the equilibrium
    # is unchanged and S_KL = sum eps^2 h^2 / (2 feq) + O(eps^3); S_NEQ and S_PI
    # are exactly linear in eps.
    energy = q == 25
    args = (np.array([1.1]), np.array([0.03]), np.array([-0.02])) + \
        ((np.array([1.05]),) if q == 25 else ())
    feq = orc.equilibrium(q, *args)[:, 0]
    h = _invariant_free(orc, q, 7, energy) * feq.min()
    vx, vy, _ = orc.lattice(q)
    prev = None
    for eps in [1e-2, 1e-3]:
        f = feq + eps * h
        s, _ = orc.sensors(q, f[:, None])
        ref = np.sum((eps * h) ** 2 / (2 * feq))
        rel = abs(s[0, 0] / ref - 1)
        assert rel < 30 * eps
        if prev is not None:
            assert rel < prev / 5          # the error is O(eps)
        prev = rel
        np.testing.assert_allclose(s[1, 0], eps * np.abs(h).sum(), rtol=1e-10)
        P = np.array([[np.sum(vx * vx * h), np.sum(vx * vy * h)],
                      [np.sum(vx * vy * h), np.sum(vy * vy * h)]]) * eps
        np.testing.assert_allclose(s[2, 0], np.sqrt(np.sum(P ** 2)), rtol=1e-9)


def test_pi_pure_shear_d2q9(orc):
    # h_i = s w_i cx cy has only Pi_xy = s/9 (four corners of weight 1/36), so
    # ||Pi||_F = sqrt(2) s / 9.
    vx, vy, w = orc.lattice(9)
    feq = orc.equilibrium(9, np.array([1.0]), np.array([0.0]), np.array([0.0]))[:, 0]
    s = 1e-3
    f = feq + s * w * vx * vy
    sens, _ = orc.sensors(9, f[:, None])
    np.testing.assert_allclose(sens[2, 0], np.sqrt(2) * s / 9, rtol=1e-10)
    np.testing.assert_allclose(sens[1, 0], 4 * s / 36, rtol=1e-10)
    assert sens[3, 0] == 0.0


def test_q_energy_flux_mode_d2q25(orc):
    # h_i = s w_i vx (|v|^2 - 4): zero mass, momentum, energy and stress, and
    # q_x = s (E[X^2 (X^2+Y^2)^2]/2 - 2 E[X^2 (X^2+Y^2)]) = s (24/2 - 8) = 4 s.
    vx, vy, w = orc.lattice(25)
    feq = orc.equilibrium(25, np.array([1.0]), np.array([0.0]), np.array([0.0]),
                          np.array([1.0]))[:, 0]
    s = 1e-4
    f = feq + s * w * vx * (vx ** 2 + vy ** 2 - 4)
    sens, _ = orc.sensors(25, f[:, None])
    np.testing.assert_allclose(sens[3, 0], 4 * s, rtol=1e-10)
    assert sens[2, 0] < 1e-15
    m = orc.moments(25, f[:, None])
    np.testing.assert_allclose(m[:, 0], [1.0, 0.0, 0.0, 1.0], atol=1e-15)


@pytest.mark.parametrize("q", [9, 25])
def test_kl_nonnegative_and_equals_literal_form(orc, q):
    # Gibbs' inequality: S_KL >= 0 for any positive populations; it equals the
    # literal sum f ln(f/feq) since sum f = sum feq = rho.
    args = inputs.random_state((200,), 9, (0.8, 1.2), 0.1, (0.9, 1.1) if q == 25 else None)
    feq = orc.equilibrium(q, *args)
    f = feq * np.exp(inputs.perturbation(feq.shape, 10, 0.2))
    s, nf = orc.sensors(q, f)
    assert nf == 0 and (s[0] >= 0).all()
    m = orc.moments(q, f)
    fe = orc.equilibrium(q, m[0], m[1], m[2], m[3] if q == 25 else None)
    literal = np.sum(f * np.log(f / fe), 0)
    big = s[0] > 1e-10 * m[0]
    assert big.sum() > 150
    np.testing.assert_allclose(s[0][big], literal[big], rtol=1e-9)


def test_positivity_fault(orc):
    feq = orc.equilibrium(9, np.ones(3), np.zeros(3), np.zeros(3))
    f = feq.copy()
    f[2, 1] = -1e-3           # one negative population in cell 1
    f[4, 1] += 1e-3 + feq[2, 1]
    s, nf = orc.sensors(9, f)
    assert nf == 1
    assert np.isinf(s[0, 1]) and np.isfinite(s[0, [0, 2]]).all()
    assert np.isfinite(s[1:, 1]).all() and s[1, 1] > 0


def test_flag_rule_bruteforce(orc):
    # The C flag rule against an independent numpy re-evaluation, including
    # the fault bit, on a stepped field with thresholds inside its range.
    rho, ux, uy = inputs.double_shear_layer(32)
    f = orc.equilibrium(9, rho, ux, uy)
    out = orc.d2q9_step(f, 0.55)
    out = orc.d2q9_step(out["f"], 0.55)
    s = out["sens"]
    thr = np.array([[np.quantile(s[k], 0.5), np.quantile(s[k], 0.9)] for k in range(4)])
    for mask in [1, 2, 3, 4, 7]:
        o = orc.d2q9_step(out["f"], 0.55, thr=thr, mask=mask)
        ref = orc.flags_from_sensors(o["sens"], thr, mask)
        np.testing.assert_array_equal(o["flags"], ref)
        assert set(np.unique(o["flags"])) <= {0, 1, 2}
    # disabled sensors (+inf thresholds) never flag
    o = orc.d2q9_step(out["f"], 0.55, thr=np.full((4, 2), np.inf), mask=15)
    assert (o["flags"] == 0).all()

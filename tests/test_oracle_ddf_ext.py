"""Pins of the oracle's extension sensors on the double distribution (the rest
of Table I with the g terms superposed, the quasi-equilibrium collision as
Omega): zero at equilibrium; with g at its equilibrium and Pr = 1 (the QE
collision is then BGK) they equal the single-distribution sensors of f,
which have pins of their own; the Gibbs sign and the ln(h^eq/w) split of the
dissipations; the Fourier flux of a temperature wave against kappa |grad T|
with kappa = C_p mu / Pr; the model's bulk viscosity (2 - gamma) mu measured
on compression waves at three gamma, and the compression and strain sensors
against the velocity gradients of compression and shear waves; +inf on a
positivity fault."""
import numpy as np
import pytest

from oracle import macro
from paper_2603_13618_amd import inputs

GAMMA, PR = 1.4, 0.71
CV = 1.0 / (GAMMA - 1.0)
NAMES = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "qf")


def _idx(orc, name):
    return orc.EXT_NAMES.index(name)


def _moment_free(orc, shape, seed, scale):
    """A perturbation of f with zero mass, momentum and |v|^2 moment."""
    vx, vy, w = orc.lattice(25)
    M = np.stack([np.ones(25), vx, vy, vx * vx + vy * vy]) * w       # moments of w_i d_i
    P = np.eye(25) - M.T @ np.linalg.solve(M @ M.T, M)
    rng = np.random.default_rng(seed)
    d = P @ rng.standard_normal((25, int(np.prod(shape))))
    return (scale * w[:, None] * d).reshape((25,) + shape)


def test_zero_at_equilibrium(orc):
    rho, ux, uy = inputs.random_state((4, 5), seed=2, umax=0.1)
    T = 1.0 + 0.2 * (rho - 1.0)
    s = orc.ddf_ext_sensors(orc.ddf_equilibrium(rho, ux, uy, T, GAMMA), 1e-3, GAMMA, PR)
    for name in NAMES + ("comp", "strain"):   # round-off, amplified by the small corner weights
        assert np.abs(s[_idx(orc, name)]).max() < 1e-12, name


def test_reduces_to_the_single_distribution_sensors(orc):
    # f = f^eq + a moment-free perturbation keeps rho, u, T, hence g^eq: with
    # g = g^eq and Pr = 1 every sensor is the one of f alone
    shape = (3, 4)
    rho, ux, uy = inputs.random_state(shape, seed=5, umax=0.1)
    T = 1.0 + 0.1 * (rho - 1.0)
    fg = orc.ddf_equilibrium(rho, ux, uy, T, GAMMA)
    fg[:25] += _moment_free(orc, shape, seed=6, scale=2e-2)
    m = orc.ddf_moments(fg, GAMMA)
    assert np.abs(m[3] - T).max() < 1e-13
    mu = 2e-3
    dd = orc.ddf_ext_sensors(fg, mu, GAMMA, 1.0)
    single = orc.ext_sensors(25, fg[:25], mu)
    for name in NAMES:
        k = _idx(orc, name)
        assert np.allclose(dd[k], single[k], rtol=1e-11, atol=1e-15), name
    assert np.abs(dd[_idx(orc, "kn")]).min() > 0


def test_dissipations_sign_and_split(orc):
    shape = (4, 4)
    rng = np.random.default_rng(9)
    rho = 1.0 + 0.1 * rng.standard_normal(shape)
    T = 1.0 + 0.1 * rng.standard_normal(shape)
    z = np.zeros(shape)
    fg = orc.ddf_equilibrium(rho, z, z, T, GAMMA) * (1 + 2e-2 * rng.standard_normal((50,) + shape))
    mu = 1e-3
    s = orc.ddf_ext_sensors(fg, mu, GAMMA, 1.0)
    _, q = orc.ddf_moments(fg, GAMMA, qe=True)
    m = orc.ddf_moments(fg, GAMMA)
    _, _, w = orc.lattice(25)
    w = w[:, None, None]
    feq, geq = q[:25], q[25:50]
    inv_tau = m[0] * m[3] / mu
    # Gibbs: with a BGK collision every term (h - h^eq) ln(h/h^eq) >= 0
    assert (s[_idx(orc, "sigma_hkl")] > 0).all()
    split = inv_tau * (((fg[:25] - feq) * np.log(feq / w)).sum(0) + ((fg[25:] - geq) * np.log(geq / w)).sum(0))
    diff = s[_idx(orc, "sigma_h")] - s[_idx(orc, "sigma_hkl")]
    assert np.allclose(diff, split, rtol=1e-9, atol=1e-12)


def test_fourier_flux_of_a_temperature_wave(orc):
    # heat flux at rest: q = -kappa grad T, kappa = C_p mu / Pr, C_p = gamma / (gamma - 1)
    n, mu = 128, 0.01
    y = (np.arange(n) + 0.5) / n
    s = np.sin(2 * np.pi * y)[:, None] * np.ones((1, 2))
    one = np.ones((n, 2))
    rho0, T0 = 1.2, 1.5
    T = T0 * (1 + 1e-3 * s)
    f = orc.ddf_equilibrium(rho0 * T0 / T, 0 * one, 0 * one, T, GAMMA)
    dx = 1.0 / n
    dt = 0.05 * dx / 2.857
    o = orc.ddf_run(f, 400, mu, dt, dx, bc=(0, 0), gamma=GAMMA, prandtl=PR)
    qf = orc.ddf_ext_sensors(o["f"], mu, GAMMA, PR)[_idx(orc, "qf")]
    m = orc.ddf_moments(o["f"], GAMMA)
    kappa = GAMMA / (GAMMA - 1.0) * mu / PR
    want = macro.macro_sensors(m[0], m[1], m[2], m[3], 0.0, 0.0, kappa, dx=dx, bc=(0, 0), which=("qf",))["qf"]
    err = np.linalg.norm(qf - want) / np.linalg.norm(want)
    assert err < 0.03, err


def test_positivity_fault_gives_inf(orc):
    rho, ux, uy = inputs.random_state((2, 3), seed=1, umax=0.05)
    fg = orc.ddf_equilibrium(rho, ux, uy, 1.0 + 0 * rho, GAMMA)
    fg[25 + 3, 1, 2] = -1e-4
    s = orc.ddf_ext_sensors(fg, 1e-3, GAMMA, PR)
    for name in ("kn", "hr", "sigma_h", "sigma_hkl", "alpha"):
        assert np.isinf(s[_idx(orc, name)][1, 2]), name
        assert np.isfinite(s[_idx(orc, name)][0]).all(), name
    assert np.isfinite(s[_idx(orc, "qf")]).all()


def _wave(orc, gamma, mu, kind, n=128, steps=200):
    """A small compression (sound) or shear wave along x, run `steps` steps
    from its equilibrium; returns the state, its moments and its pressure
    tensor of f^neq."""
    x = (np.arange(n) + 0.5) / n
    X = np.tile(x, (4, 1))
    amp = 1e-3
    s = np.sin(2 * np.pi * X)
    if kind == "compression":
        rho, ux, uy, T = 1 + amp * s, amp * np.sqrt(gamma) * s, 0 * X, 1 + (gamma - 1) * amp * s
    else:
        rho, ux, uy, T = 1 + 0 * X, 0 * X, amp * s, 1 + 0 * X
    dx = 1.0 / n
    dt = 0.05 * dx / (np.sqrt(gamma) + amp)
    f = orc.ddf_run(orc.ddf_equilibrium(rho, ux, uy, T, gamma), steps, mu, dt, dx, bc=(0, 0),
                    gamma=gamma, prandtl=PR)["f"]
    m, q = orc.ddf_moments(f, gamma, qe=True)
    vx, vy, _ = orc.lattice(25)
    fneq = f[:25] - q[:25]
    P = [(a[:, None, None] * b[:, None, None] * fneq).sum(0) for a, b in ((vx, vx), (vx, vy), (vy, vy))]
    return f, m, P, dx


@pytest.mark.parametrize("gamma", [1.2, 1.4, 1.6])
def test_bulk_viscosity_of_a_compression_wave(orc, gamma):
    # Chapman-Enskog (Sec. II.A.2, eq. visc_bluk_1): P^neq = -mu (A + A^T) -
    # lambda (div u) I, so tr P = -D eta div u with eta = 2 mu / D + lambda =
    # (2/D - R/C_v) mu = (2 - gamma) mu in two dimensions: 0.8, 0.6, 0.4 mu
    # here; the deviatoric part keeps the shear viscosity mu.
    mu = 2e-3
    f, m, (pxx, pxy, pyy), dx = _wave(orc, gamma, mu, "compression")
    div = (np.roll(m[1], -1, axis=1) - np.roll(m[1], 1, axis=1)) / (2 * dx)
    sel = np.abs(div) > 0.5 * np.abs(div).max()
    eta = np.median((pxx + pyy)[sel] / (-2.0 * div[sel]))
    assert abs(eta / mu - (2.0 - gamma)) < 0.01 * (2.0 - gamma), eta / mu
    dev = np.median((0.5 * (pxx - pyy))[sel] / (-mu * div[sel]))
    assert abs(dev - 1.0) < 0.01, dev


@pytest.mark.parametrize("gamma", [1.2, 1.4, 1.6])
def test_compression_and_strain_against_velocity_gradients(orc, gamma):
    # Sec. III.A.2/4: with the model's lambda = -(gamma - 1) mu the kinetic
    # compression sensor is sqrt(D)|div u| and the strain sensor |E|_F, the
    # same kinematic rates the macroscopic sensors take from central
    # differences; a shear wave has no compression.  Relative L2 over the
    # wave: 0.8-1.1 % on the sound wave (the non-equilibrium stress lags the
    # travelling gradient by about tau: a phase of c_s tau k ~ 1.5e-2), 0.2 %
    # on the standing shear wave; bars 2 % and 0.5 %
    mu = 2e-3
    for kind, bar in (("compression", 0.02), ("shear", 0.005)):
        f, m, _, dx = _wave(orc, gamma, mu, kind)
        s = orc.ddf_ext_sensors(f, mu, gamma, PR)
        want = macro.macro_sensors(m[0], m[1], m[2], m[3], mu, -(gamma - 1.0) * mu, 0.0, dx=dx,
                                   bc=(0, 0), which=("c", "e"))
        e = np.linalg.norm(s[_idx(orc, "strain")] - want["e"]) / np.linalg.norm(want["e"])
        assert e < bar, (kind, e)
        if kind == "compression":
            c = np.linalg.norm(s[_idx(orc, "comp")] - want["c"]) / np.linalg.norm(want["c"])
            assert c < bar, c
        else:
            assert np.abs(s[_idx(orc, "comp")]).max() < 1e-3 * np.abs(s[_idx(orc, "strain")]).max()

"""Pins of the macroscopic class-1 sensors (central differences): exact on
linear fields away from the boundaries, the sin(k dx)/dx response on Fourier
modes, zero for rigid motions, and the closed-form invariants of the tensors
(C and S from the eigen-structure of the strain rate)."""
import numpy as np
import pytest

from oracle import macro

MU, LAM, KAP = 0.3, -0.2, 0.7


def _grid(n, m):
    y, x = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    return x.astype(float), y.astype(float)


def test_linear_field_is_exact_in_the_interior():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((2, 2))            # A_ab = d_a u_b
    g = rng.standard_normal(2)
    x, y = _grid(12, 9)
    dx = 0.25
    X, Y = x * dx, y * dx
    ux = 0.3 + A[0, 0] * X + A[1, 0] * Y
    uy = -0.1 + A[0, 1] * X + A[1, 1] * Y
    T = 1.0 + g[0] * X + g[1] * Y
    rho = np.ones_like(X)
    out = macro.macro_sensors(rho, ux, uy, T, MU, LAM, KAP, dx=dx, bc=(1, 1))
    sl = (slice(1, -1), slice(1, -1))
    Sym = A + A.T
    div = np.trace(A)
    tau = -MU * Sym - LAM * div * np.eye(2)
    want = {"tau": np.linalg.norm(tau), "c": np.sqrt(2) * abs(div),
            "s": np.linalg.norm(Sym - div * np.eye(2)), "e": 0.5 * np.linalg.norm(Sym)}
    for k, v in want.items():
        assert np.allclose(out[k][sl], v, rtol=1e-12, atol=1e-12), k
    u = np.stack([ux[sl], uy[sl]])
    qh = np.einsum("a...,ab->b...", u, tau)
    assert np.allclose(out["qh"][sl], np.hypot(*qh), rtol=1e-12)
    assert np.allclose(out["qf"][sl], KAP * np.hypot(*g), rtol=1e-12)
    assert np.allclose(out["qnsf"][sl], np.hypot(-KAP * g[0] + qh[0], -KAP * g[1] + qh[1]), rtol=1e-12)
    # zero-gradient edges see half the slope (one neighbour is the cell itself)
    c_edge = macro.macro_sensors(rho, ux, 0 * uy, T, MU, LAM, KAP, dx=dx, bc=(1, 1), which=("c",))["c"]
    assert np.allclose(c_edge[3, 0], np.sqrt(2) * abs(0.5 * A[0, 0]), rtol=1e-12)


def test_fourier_mode_response():
    n = 32
    x, y = _grid(n, n)
    kx = 3
    ux = 0 * x
    uy = np.sin(2 * np.pi * kx * x / n)                 # pure shear, periodic
    out = macro.macro_sensors(np.ones_like(x), ux, uy, None, MU, LAM, KAP, bc=(0, 0),
                              which=("s", "e", "c", "tau"))
    amp = np.sin(2 * np.pi * kx / n) * np.cos(2 * np.pi * kx * x / n)     # central difference
    assert np.allclose(out["s"], np.sqrt(2) * np.abs(amp), atol=1e-14)
    assert np.allclose(out["e"], np.abs(amp) / np.sqrt(2), atol=1e-14)
    assert np.abs(out["c"]).max() < 1e-14
    assert np.allclose(out["tau"], MU * np.sqrt(2) * np.abs(amp), atol=1e-14)


def test_rigid_motions_give_zero_rates():
    x, y = _grid(10, 10)
    w = 0.7
    ux, uy = -w * y + 0.2, w * x - 0.1                   # rotation + translation
    out = macro.macro_sensors(np.ones_like(x), ux, uy, np.ones_like(x), MU, LAM, KAP, bc=(1, 1))
    sl = (slice(1, -1), slice(1, -1))
    for k in ("tau", "c", "s", "e", "qh", "qf", "qnsf"):
        assert np.abs(out[k][sl]).max() < 1e-13, k


def test_per_rho_scales_the_transport_terms():
    rng = np.random.default_rng(3)
    f = [rng.standard_normal((8, 8)) for _ in range(4)]
    rho = 1.0 + 0.1 * rng.random((8, 8))
    a = macro.macro_sensors(rho, *f[:2], f[2], MU, LAM, KAP, per_rho=True)
    b = macro.macro_sensors(rho, *f[:2], f[2], MU, LAM, KAP, per_rho=False)
    for k in ("tau", "qh", "qf", "qnsf"):
        assert np.allclose(a[k], rho * b[k], rtol=1e-13), k
    for k in ("c", "s", "e"):
        assert np.array_equal(a[k], b[k]), k

"""Seeded synthetic initial fields (rho, ux, uy[, T]) for the workloads.

This module holds no part of the kinetic method: it only produces macroscopic
fields, in FP64 numpy arrays of shape [ny, nx] (y rows, x fastest).  Both the
HIP path and the FP64 reference read their initial conditions from here.

Workloads (x = i/N node-centred on periodic grids, (i+1/2)/N cell-centred on
bounded ones):

* double shear layer on [0,1)^2: rho = 1,
  ux = 0.05 tanh(80 (y - 1/4)) for y < 1/2 else 0.05 tanh(80 (3/4 - y)),
  uy = 0.0025 sin(2 pi (x + 1/4));
* smooth random field: rho = 1 + 0.01 n_rho, u = 0.03 (n_x, n_y) where each n
  is a seeded Gaussian random Fourier series band-limited to |k|_inf <= cutoff,
  normalised to unit variance on the grid;
* four-quadrant Riemann problem on [0,1]^2 split at x = y = 1/2: per quadrant
  (drawn in the order NE, NW, SW, SE) rho ~ U[0.5, 1.5], |u| ~ U[0, 0.1] at a
  uniform random angle, T ~ U[0.9, 1.1];
* shear wave: rho = 1, ux = U sin(2 pi y / N), uy = 0.

The spectral noise is evaluated as a separable sum over its modes, so a window
of a large grid can be generated without the whole grid and the field is the
same function of position at every resolution (the 8192^2 field sampled at
every other node is the 4096^2 field).
"""
import numpy as np


def _half_plane_modes(cutoff):
    """Half-plane wavevectors {ky > 0} U {ky = 0, kx > 0}, |k|_inf <= cutoff,
    in row-major order (ky, then kx ascending)."""
    ks = []
    for ky in range(0, cutoff + 1):
        for kx in range(-cutoff, cutoff + 1):
            if ky > 0 or kx > 0:
                ks.append((kx, ky))
    return ks


def spectral_coefficients(seed, cutoff, nfields=3):
    """Complex coefficients c_k = (a + i b)/sqrt(2), a, b ~ N(0,1) drawn in that
    order, for each of nfields fields in turn, from numpy's PCG64 stream."""
    rng = np.random.default_rng(seed)
    ks = _half_plane_modes(cutoff)
    out = []
    for _ in range(nfields):
        c = np.empty(len(ks), np.complex128)
        for m in range(len(ks)):
            a = rng.standard_normal()
            b = rng.standard_normal()
            c[m] = (a + 1j * b) / np.sqrt(2.0)
        out.append(c)
    return ks, out


def spectral_field(ks, c, n, x0=0, y0=0, wx=None, wy=None):
    """n(x) = sum_k c_k e^{2 pi i k.x} + c.c., x = (i/n, j/n), normalised to
    unit variance over the full n x n grid (sum over both half-planes of |c_k|^2
    = 1 by Parseval, since no mode reaches the Nyquist index).  Returns the
    window rows y0..y0+wy-1, columns x0..x0+wx-1 (indices taken mod n)."""
    wx = n if wx is None else wx
    wy = n if wy is None else wy
    cutoff = max(max(abs(kx), ky) for kx, ky in ks)
    if 2 * cutoff >= n:
        raise ValueError("cutoff must stay below the Nyquist index")
    xs = (np.arange(x0, x0 + wx) % n) / n
    ys = (np.arange(y0, y0 + wy) % n) / n
    kxs = np.arange(-cutoff, cutoff + 1)
    kys = np.arange(0, cutoff + 1)
    C = np.zeros((len(kys), len(kxs)), np.complex128)
    for (kx, ky), ck in zip(ks, c):
        C[ky, kx + cutoff] = ck
    Ex = np.exp(2j * np.pi * np.outer(kxs, xs))     # [Kx, wx]
    Ey = np.exp(2j * np.pi * np.outer(ys, kys))     # [wy, Ky]
    field = 2.0 * np.real(Ey @ C @ Ex)              # c_k e^{ikx} + conj
    norm = np.sqrt(2.0 * np.sum(np.abs(c) ** 2))
    return field / norm


def smooth_random(n, seed=0, cutoff=16, window=None):
    """Smooth random workload on an n x n periodic grid.  window = (x0, y0, wx, wy)
    selects a sub-block (indices mod n).  Returns rho, ux, uy."""
    ks, (cr, cx, cy) = spectral_coefficients(seed, cutoff, 3)
    x0, y0, wx, wy = (0, 0, n, n) if window is None else window
    nr = spectral_field(ks, cr, n, x0, y0, wx, wy)
    nxf = spectral_field(ks, cx, n, x0, y0, wx, wy)
    nyf = spectral_field(ks, cy, n, x0, y0, wx, wy)
    return 1.0 + 0.01 * nr, 0.03 * nxf, 0.03 * nyf


def double_shear_layer(n):
    """Double shear layer on an n x n periodic grid (node-centred)."""
    x = np.arange(n) / n
    y = np.arange(n) / n
    X, Y = np.meshgrid(x, y)
    ux = np.where(Y < 0.5, 0.05 * np.tanh(80.0 * (Y - 0.25)), 0.05 * np.tanh(80.0 * (0.75 - Y)))
    uy = 0.05 * 0.05 * np.sin(2.0 * np.pi * (X + 0.25))
    rho = np.ones((n, n))
    return rho, ux, uy


def riemann_quadrants(nx, ny=None, seed=0, window=None):
    """Four-quadrant Riemann problem on [0,1]^2 (cell-centred), split at 1/2.
    Returns rho, ux, uy, T and the per-quadrant states (NE, NW, SW, SE)."""
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(4):
        rho = rng.uniform(0.5, 1.5)
        speed = rng.uniform(0.0, 0.1)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        T = rng.uniform(0.9, 1.1)
        states.append((rho, speed * np.cos(ang), speed * np.sin(ang), T))
    x0, y0, wx, wy = (0, 0, nx, ny) if window is None else window
    x = (np.arange(x0, x0 + wx) + 0.5) / nx
    y = (np.arange(y0, y0 + wy) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    east, north = X >= 0.5, Y >= 0.5
    quad = np.where(north & east, 0, np.where(north, 1, np.where(~east, 2, 3)))
    fields = [np.choose(quad, [s[k] for s in states]).astype(np.float64) for k in range(4)]
    return fields[0], fields[1], fields[2], fields[3], states


def riemann_dt(states, dx, cfl=0.01, gamma=2.0):
    """Time step from the initial states: cfl * dx / max(|u| + sqrt(gamma T))."""
    smax = max(np.hypot(ux, uy) + np.sqrt(gamma * T) for (_, ux, uy, T) in states)
    return cfl * dx / smax


# The paper's own workloads (Sec. IV): analytic initial conditions, air
# (gamma = 1.4, R = 1, T = p / rho), equilibrium populations.

SOD_STATES = ((1.0, 1.0, 0.0), (0.125, 0.1, 0.0))      # (rho, p, u_x) left / right of x = 1/2


def sod_tube(nx, ny=2):
    """Sod shock tube on x in [0, 1] (cell-centred, split at 1/2), run as
    pseudo-1D on an nx x ny grid (periodic in y).  Returns rho, ux, uy, T."""
    x = (np.arange(nx) + 0.5) / nx
    left = x <= 0.5
    (rl, pl, ul), (rr, pr, ur) = SOD_STATES
    rho = np.where(left, rl, rr)
    p = np.where(left, pl, pr)
    u = np.where(left, ul, ur)
    one = np.ones((ny, 1))
    return rho * one, u * one, 0.0 * rho * one, (p / rho) * one


# modified configuration 3 of the 2D Riemann problems: quadrants split at
# x = y = 0.85; (rho, p, u_x, u_y) for NE, NW, SW, SE
CASE3_STATES = ((1.5, 1.5, 0.0, 0.0), (0.5323, 0.3, 1.206, 0.0), (0.138, 0.029, 1.206, 1.206),
                (0.5323, 0.3, 0.0, 1.206))


def riemann_case3(n, window=None):
    """The modified 2D Riemann problem No. 3 on [0, 1]^2 (cell-centred, split
    at 0.85).  window = (x0, y0, wx, wy) selects a sub-block.  Returns rho,
    ux, uy, T."""
    x0, y0, wx, wy = (0, 0, n, n) if window is None else window
    x = (np.arange(x0, x0 + wx) + 0.5) / n
    y = (np.arange(y0, y0 + wy) + 0.5) / n
    X, Y = np.meshgrid(x, y)
    east, north = X >= 0.85, Y >= 0.85
    quad = np.where(north & east, 0, np.where(north, 1, np.where(~east, 2, 3)))
    rho, p, ux, uy = (np.choose(quad, [s[k] for s in CASE3_STATES]).astype(np.float64) for k in range(4))
    return rho, ux, uy, p / rho


def cfl_dt(fields, dx, gamma=1.4, cfl=0.01):
    """The paper's time step rule dt = CFL min(dx, dy) / max(|u| + c_s), c_s =
    sqrt(gamma T), from the initial fields (rho, ux, uy, T)."""
    _, ux, uy, T = fields
    return cfl * dx / float(np.max(np.hypot(ux, uy) + np.sqrt(gamma * T)))


def shear_wave(n, amp=1e-4, ny=None):
    """rho = 1, ux = amp sin(2 pi y / ny), uy = 0 on an n x ny grid."""
    ny = n if ny is None else ny
    y = np.arange(ny)[:, None] * np.ones((1, n))
    return np.ones((ny, n)), amp * np.sin(2.0 * np.pi * y / ny), np.zeros((ny, n))


def random_state(shape, seed, rho_range=(0.9, 1.1), umax=0.1, T_range=None):
    """Independent uniform random fields per cell (tests of cell-local maths)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(*rho_range, size=shape)
    ux = rng.uniform(-umax, umax, size=shape)
    uy = rng.uniform(-umax, umax, size=shape)
    if T_range is None:
        return rho, ux, uy
    return rho, ux, uy, rng.uniform(*T_range, size=shape)


def perturbation(shape, seed, scale):
    """Seeded Gaussian perturbation array of the given shape and scale."""
    return scale * np.random.default_rng(seed).standard_normal(shape)

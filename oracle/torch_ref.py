"""Differentiable FP64 D2Q9 reference in plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY.  It is the autograd reference for the hand-written
adjoint: the loss is the smooth KL sensor summed over cells at the last step,

    L(u0) = sum_x sum_i [g_i ln(g_i / f^eq_i) - g_i + f^eq_i](g_N(x)),

with g_N the pre-collision (post-stream) populations of step N and the initial
populations at the equilibrium of (rho0, u0) (Sec. IV setup: equilibrium
initial conditions).  The D2Q9 equilibrium is the order-2 Grad-Hermite form on
the GH3 x GH3 lattice with T_ref = 1/3, i.e. the textbook
w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2); streaming is a periodic roll.
This file shares no code with the C oracle or the HIP path.
"""
import torch

# velocity i = 3a + b, c = (a - 1, b - 1)
_CX = [a - 1 for a in range(3) for b in range(3)]
_CY = [b - 1 for a in range(3) for b in range(3)]
_W1 = [1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0]
_W = [_W1[a] * _W1[b] for a in range(3) for b in range(3)]


def feq(rho, ux, uy):
    """[9, ny, nx] textbook second-order equilibrium."""
    out = []
    usq = ux * ux + uy * uy
    for i in range(9):
        cu = _CX[i] * ux + _CY[i] * uy
        out.append(_W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq))
    return torch.stack(out)


def stream(f):
    """g_i(x) = f_i(x - c_i), periodic (torch.roll shifts by +c)."""
    return torch.stack([torch.roll(f[i], shifts=(_CY[i], _CX[i]), dims=(0, 1)) for i in range(9)])


def macros(g):
    rho = g.sum(0)
    jx = sum(_CX[i] * g[i] for i in range(9))
    jy = sum(_CY[i] * g[i] for i in range(9))
    return rho, jx / rho, jy / rho


def kl(g):
    """Per-cell smooth KL sensor of pre-collision populations g."""
    rho, ux, uy = macros(g)
    fe = feq(rho, ux, uy)
    return (g * torch.log(g / fe) - g + fe).sum(0)


def step(f, tau):
    """One LBGK step; returns (post-collision f, pre-collision g)."""
    g = stream(f)
    rho, ux, uy = macros(g)
    fe = feq(rho, ux, uy)
    return g - (g - fe) / tau, g


def kl_loss(rho0, ux0, uy0, tau, nsteps):
    """L = sum_x S_KL(g_N(x)) after nsteps from equilibrium initial populations."""
    f = feq(rho0, ux0, uy0)
    g = None
    for _ in range(nsteps):
        f, g = step(f, tau)
    return kl(g).sum()


def kl_loss_grad(rho0, ux0, uy0, tau, nsteps):
    """(L, dL/dux0, dL/duy0) by autograd, all float64 CPU tensors."""
    ux = torch.as_tensor(ux0, dtype=torch.float64).clone().requires_grad_(True)
    uy = torch.as_tensor(uy0, dtype=torch.float64).clone().requires_grad_(True)
    rho = torch.as_tensor(rho0, dtype=torch.float64)
    L = kl_loss(rho, ux, uy, tau, nsteps)
    gx, gy = torch.autograd.grad(L, (ux, uy))
    return float(L.detach()), gx.numpy(), gy.numpy()

"""The differentiable torch FP64 D2Q9 reference against the C oracle (forward)
and against central finite differences of the C oracle (gradient of the summed
KL sensor w.r.t. the initial velocity field)."""
import numpy as np
import torch

from oracle import torch_ref
from paper_2603_13618_amd import inputs


def test_forward_matches_c_oracle(orc):
    rho, ux, uy = inputs.smooth_random(16, seed=1, cutoff=4)
    ux, uy = 3 * ux, 3 * uy                  # stronger gradients on a tiny grid
    f0 = orc.equilibrium(9, rho, ux, uy)
    fe = torch_ref.feq(*(torch.from_numpy(a) for a in (rho, ux, uy)))
    np.testing.assert_allclose(fe.numpy(), f0, rtol=1e-14, atol=1e-16)
    out = orc.run(9, f0, 25, tau=0.52)
    f = torch.from_numpy(f0)
    for _ in range(25):
        f, g = torch_ref.step(f, 0.52)
    np.testing.assert_allclose(f.numpy(), out["f"], rtol=1e-12, atol=1e-15)
    kl = torch_ref.kl(g).numpy()
    assert np.abs(kl - out["sens"][0]).max() <= 1e-9 * out["sens"][0].max()
    np.testing.assert_allclose(kl.sum(), out["sums"][-1, 4], rtol=1e-9)


def _loss(orc, rho, ux, uy, steps, tau):
    return orc.run(9, orc.equilibrium(9, rho, ux, uy), steps, tau=tau)["sums"][-1, 4]


def test_autograd_gradient_matches_finite_differences(orc):
    # The 32 x 32 differentiation workload (cutoff 4, tau = 0.52), shortened to
    # 60 steps to keep the CPU suite fast; central differences with eps = 1e-3.
    n, steps, tau, eps = 32, 60, 0.52, 1e-3
    rho, ux, uy = inputs.smooth_random(n, seed=0, cutoff=4)
    L, gx, gy = torch_ref.kl_loss_grad(rho, ux, uy, tau, steps)
    np.testing.assert_allclose(L, _loss(orc, rho, ux, uy, steps, tau), rtol=1e-9)
    rng = np.random.default_rng(5)
    cells = rng.integers(0, n, size=(6, 2))
    for comp, grad in ((0, gx), (1, gy)):
        for (y, x) in cells:
            up, dn = [a.copy() for a in (ux, uy)], [a.copy() for a in (ux, uy)]
            up[comp][y, x] += eps
            dn[comp][y, x] -= eps
            fd = (_loss(orc, rho, *up, steps, tau) - _loss(orc, rho, *dn, steps, tau)) / (2 * eps)
            assert abs(fd - grad[y, x]) <= 1e-3 * np.abs(grad).max()
    # directional derivative along a random smooth direction
    d = inputs.smooth_random(n, seed=9, cutoff=4)[1:]
    dd = np.sum(gx * d[0] + gy * d[1])
    fd = (_loss(orc, rho, ux + eps * d[0], uy + eps * d[1], steps, tau)
          - _loss(orc, rho, ux - eps * d[0], uy - eps * d[1], steps, tau)) / (2 * eps)
    assert abs(fd - dd) <= 1e-4 * abs(dd)

"""GPU parity of the hand-written adjoint (gradient of the summed smooth KL
sensor w.r.t. the initial velocity) against the autograd of the independent
FP64 torch reference and central finite differences of the FP64 C oracle."""
import numpy as np
import pytest
import torch

from oracle import torch_ref
from paper_2603_13618_amd import adjoint, inputs, lks

from gpu_util import to_f64

pytestmark = pytest.mark.gpu


def _grad(rho, ux, uy, tau, steps, K, dtype):
    dev = torch.device("cuda")
    u = torch.tensor(ux, device=dev, requires_grad=True)
    v = torch.tensor(uy, device=dev, requires_grad=True)
    r = torch.tensor(rho, device=dev)
    L = adjoint.kl_sensor_loss(u, v, r, tau=tau, nsteps=steps, checkpoint=K, dtype=dtype)
    L.backward()
    return float(L.detach()), to_f64(u.grad), to_f64(v.grad)


@pytest.mark.parametrize("steps,K", [(30, 7), (1, 5), (12, 12), (25, 1)])
def test_fp64_adjoint_matches_autograd_reference(steps, K):
    rho, ux, uy = inputs.smooth_random(16, seed=3, cutoff=4)
    ux, uy = 3 * ux, 3 * uy
    L, gx, gy = _grad(rho, ux, uy, 0.6, steps, K, "f64")
    Lr, rx, ry = torch_ref.kl_loss_grad(rho, ux, uy, 0.6, steps)
    assert abs(L - Lr) <= 1e-10 * abs(Lr)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    err = max(np.abs(gx - rx).max(), np.abs(gy - ry).max()) / scale
    print(f"steps {steps} K {K}: grad err {err:.2e}", flush=True)
    assert err <= 1e-9


def test_fp32_adjoint_close_to_reference():
    rho, ux, uy = inputs.smooth_random(32, seed=0, cutoff=4)
    L, gx, gy = _grad(rho, ux, uy, 0.52, 60, 20, "f32")
    Lr, rx, ry = torch_ref.kl_loss_grad(rho, ux, uy, 0.52, 60)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    err = max(np.abs(gx - rx).max(), np.abs(gy - ry).max()) / scale
    print(f"FP32 loss rel err {abs(L - Lr) / abs(Lr):.2e}, grad err {err:.2e}", flush=True)
    assert abs(L - Lr) <= 1e-4 * abs(Lr)
    assert err <= 1e-3


def test_differentiation_workload_32_against_finite_differences(orc):
    # 32 x 32 instance of the differentiation workload: 200 steps, checkpoint
    # every 20, tau = 0.52, smooth field with 4 modes; central differences of
    # the FP64 oracle with eps = 1e-3.
    n, steps, tau, eps = 32, 200, 0.52, 1e-3
    rho, ux, uy = inputs.smooth_random(n, seed=0, cutoff=4)

    def loss(a, b):
        return orc.run(9, orc.equilibrium(9, rho, a, b), steps, tau=tau)["sums"][-1, 4]

    L, gx, gy = _grad(rho, ux, uy, tau, steps, 20, "f64")
    L32, gx32, gy32 = _grad(rho, ux, uy, tau, steps, 20, "f32")
    assert abs(L - loss(ux, uy)) <= 1e-10 * abs(L)
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    rng = np.random.default_rng(1)
    worst = worst32 = 0.0
    for comp in (0, 1):
        for (y, x) in rng.integers(0, n, size=(8, 2)):
            a, b = ux.copy(), uy.copy()
            (a if comp == 0 else b)[y, x] += eps
            lp = loss(a, b)
            (a if comp == 0 else b)[y, x] -= 2 * eps
            lm = loss(a, b)
            fd = (lp - lm) / (2 * eps)
            g = (gx if comp == 0 else gy)[y, x]
            g32 = (gx32 if comp == 0 else gy32)[y, x]
            worst = max(worst, abs(fd - g) / scale)
            worst32 = max(worst32, abs(fd - g32) / scale)
    print(f"FD vs adjoint: FP64 {worst:.2e}, FP32 {worst32:.2e}", flush=True)
    assert worst <= 1e-3 and worst32 <= 1e-3


def _one_step_case(nx=24, ny=20, tau=0.6):
    # a non-equilibrium state f_{n-1}, the pre-collision g_n = S f_{n-1} and
    # random directions v, w (all FP64)
    rho, ux, uy = inputs.random_state((ny, nx), 5, (0.9, 1.1), 0.08)
    rng = np.random.default_rng(7)
    f_prev = torch_ref.feq(*(torch.tensor(a) for a in (rho, ux, uy)))
    f_prev = f_prev * (1.0 + 0.05 * torch.tensor(rng.standard_normal(f_prev.shape)))
    v = torch.tensor(rng.standard_normal(f_prev.shape))
    w = torch.tensor(rng.standard_normal(f_prev.shape))
    lat = lks.Lattice(9, nx, ny, "f64", tau=tau)
    w9 = torch.tensor([torch_ref._W[i] for i in range(9)], dtype=torch.float64)
    prev = lat.new_state()
    prev.copy_((f_prev - w9[:, None, None]).to(prev.device))       # deviation storage, rho0 = 1
    return lat, f_prev, torch_ref.stream(f_prev), v, w, prev


def test_fp64_adjoint_step_dot_product_identity():
    # <J v, w> = <v, J^T w> for one step g_n -> g_{n+1} = S C(g_n): the forward
    # derivative of the FP64 torch reference against the library's reverse step
    tau = 0.6
    lat, _, g, v, w, prev = _one_step_case(tau=tau)

    def one_step(gg):
        return torch_ref.stream(gg - (gg - torch_ref.feq(*torch_ref.macros(gg))) / tau)

    _, jv = torch.func.jvp(one_step, (g,), (v,))
    lhs = float((jv * w).sum())
    lam_in, lam_out = lat.new_state(), lat.new_state()
    lam_in.copy_(w.to(lam_in.device))
    lat.adjoint_step(prev, lam_in, lam_out)
    jtw = lam_out.cpu()
    rhs = float((v * jtw).sum())
    scale = float((v * jtw).abs().sum())
    print(f"<Jv,w> {lhs:.15e} <v,J^T w> {rhs:.15e} rel {abs(lhs - rhs) / scale:.2e}", flush=True)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_fp64_adjoint_seed_is_the_kl_gradient():
    # <dS/dg, v> of the summed smooth KL sensor at g_N = S f_{N-1}
    lat, _, g, v, _, prev = _one_step_case()
    _, dl = torch.func.jvp(lambda gg: torch_ref.kl(gg).sum(), (g,), (v,))
    lam = lat.new_state()
    lat.adjoint_seed_kl(prev, lam)
    got = lam.cpu()
    rhs = float((v * got).sum())
    scale = float((v * got).abs().sum())
    print(f"dL.v {float(dl):.15e} <v, seed> {rhs:.15e}", flush=True)
    assert abs(float(dl) - rhs) <= 1e-12 * scale

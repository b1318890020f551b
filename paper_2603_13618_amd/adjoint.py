"""Gradient of the summed smooth KL sensor with respect to the initial velocity
field, by the library's hand-written adjoint kernels behind a
torch.autograd.Function, with checkpointing.

Loss: L(u0) = sum_x S_KL(g_N(x)), g_N the pre-collision populations of the
last of N D2Q9 steps started from the equilibrium of (rho0, u0) (the smooth
S_KL is sum_i f^eq_i phi(f^neq_i / f^eq_i), phi(x) = (1+x) ln(1+x) - x,
which equals the f term of eq. HKL-sensor).

Forward: N fused steps, keeping the state every `checkpoint` steps.
Backward: for each checkpoint segment, newest first, recompute its states
with single fused steps, then run the reverse steps (seed at step N, then one
adjoint step per earlier step) and finally the initial-condition adjoint.
Everything numeric runs in liblks.so; this module only orders the calls and
owns the buffers.
"""
import torch

from . import lks


class _KLSensorLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ux0, uy0, rho0, tau, nsteps, checkpoint, dtype, layout):
        if nsteps < 1 or checkpoint < 1:
            raise ValueError("nsteps and checkpoint must be >= 1")
        ny, nx = ux0.shape
        dev = ux0.device
        lat = lks.Lattice(9, nx, ny, dtype, tau=tau, max_steps=nsteps, layout=layout, device=dev)
        lat.init(rho0, ux0.detach(), uy0.detach())
        ckpts = {0: lat.state.clone()}
        done = 0
        while done < nsteps:
            m = min(checkpoint, nsteps - done)
            lat.step(m)
            done += m
            if done < nsteps:
                ckpts[done] = lat.state.clone()
        loss = lat.sums[(nsteps - 1) % nsteps, 4].clone()
        ctx.lat = lat
        ctx.ckpts = ckpts
        ctx.meta = (nsteps, checkpoint)
        ctx.fields = [t.detach().to(dev, torch.float64).contiguous() for t in (rho0, ux0, uy0)]
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        lat, ckpts = ctx.lat, ctx.ckpts
        nsteps, K = ctx.meta
        rho0, ux0, uy0 = ctx.fields
        seg = [lat.new_state() for _ in range(min(K, nsteps))]
        lam = [lat.new_state() for _ in range(2)]
        cur = 0                      # lam[cur] holds dL/dg_{n+1} entering step n
        for s in sorted(ckpts, reverse=True):
            e = min(s + K - 1, nsteps - 1)          # states f_s .. f_e
            seg[0].copy_(ckpts[s])
            for j in range(1, e - s + 1):
                lat.step_from(seg[j - 1], seg[j])
            for n in range(e + 1, s, -1):           # reverse steps n = e+1 .. s+1
                prev = seg[n - 1 - s]               # f_{n-1}
                if n == nsteps:
                    lat.adjoint_seed_kl(prev, lam[cur])
                else:
                    lat.adjoint_step(prev, lam[cur], lam[1 - cur])
                    cur = 1 - cur
        gux = torch.empty_like(ux0)
        guy = torch.empty_like(uy0)
        lat.adjoint_init(rho0, ux0, uy0, lam[cur], gux, guy)
        g = grad_out.to(torch.float64)
        return gux * g, guy * g, None, None, None, None, None, None


def kl_sensor_loss(ux0, uy0, rho0, tau=0.52, nsteps=200, checkpoint=20, dtype="f32",
                   layout="planes"):
    """L = sum of the smooth KL sensor at the last of nsteps steps (0-dim
    float64 tensor), differentiable w.r.t. ux0 and uy0 ([ny, nx] float64 CUDA
    tensors); rho0 is held fixed.  layout: the population layout of the
    states the forward and reverse steps run on."""
    return _KLSensorLoss.apply(ux0, uy0, rho0, tau, nsteps, checkpoint, dtype, layout)

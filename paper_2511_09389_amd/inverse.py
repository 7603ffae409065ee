"""Gradient-based recovery of an emissivity field through the tracer (Sec. 4).

The paper recovers a scalar amplitude with jacfwd and notes the extension to more
parameters. Here the whole j field is recovered: starting from j = 0, Adam minimises the
mean squared error between the traced field and a target field, with gradients from the
library's adjoint."""

import torch

from .autograd import march_field


def recover_emissivity(kappa_map, target, source_pos, num_rays, step_size, radiation_velocity,
                       time_step, iters=200, lr=1e-2, j_init=None, callback=None):
    """Return (j, losses). kappa_map and target are 3-D float32 device tensors."""
    j = (torch.zeros_like(target) if j_init is None else j_init.clone()).requires_grad_(True)
    opt = torch.optim.Adam([j], lr=lr)
    losses = []
    for it in range(iters):
        opt.zero_grad(set_to_none=True)
        field = march_field(j, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                            time_step)
        loss = torch.mean((field - target) ** 2)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
        if callback is not None:
            callback(it, losses[-1])
    return j.detach(), losses

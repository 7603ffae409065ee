"""Gradient-based recovery of an emissivity field through the tracer (Sec. 4).

The paper recovers a scalar amplitude with forward-mode differentiation and notes the
extension to more parameters. Here the whole j field is recovered: starting from j = 0,
Adam minimises the mean squared error between the traced field and a target field. Every
step runs in the library: the march (rtmi_trace_multi), the loss and its gradient
(rtmi_field_mse), the adjoint (rtmi_trace_vjp) and the Adam update (rtmi_adam_step);
PyTorch only holds the buffers.

The optimiser state (j, both Adam moments, the step count and the loss history) can be
saved and restored, so a long recovery can stop and resume where it left off.
"""

from dataclasses import dataclass, field
from typing import List

import torch

from . import rtmi


@dataclass
class InverseState:
    """Everything a recovery needs to continue: the iterate, Adam's moments and step."""

    j: torch.Tensor
    m: torch.Tensor
    v: torch.Tensor
    step: int = 0
    losses: List[float] = field(default_factory=list)

    @classmethod
    def start(cls, target, j_init=None):
        j = torch.zeros_like(target) if j_init is None else j_init.detach().clone().contiguous()
        return cls(j, torch.zeros_like(j), torch.zeros_like(j), 0, [])

    def state_dict(self):
        return {"j": self.j.detach().cpu(), "m": self.m.detach().cpu(), "v": self.v.detach().cpu(),
                "step": torch.tensor(self.step, dtype=torch.int64),
                "losses": torch.tensor(self.losses, dtype=torch.float64)}

    @classmethod
    def from_state_dict(cls, sd, device):
        return cls(sd["j"].to(device).contiguous(), sd["m"].to(device).contiguous(),
                   sd["v"].to(device).contiguous(), int(sd["step"]), [float(x) for x in sd["losses"]])

    def save(self, path):
        torch.save(self.state_dict(), path)

    @classmethod
    def load(cls, path, device):
        return cls.from_state_dict(torch.load(path, map_location="cpu", weights_only=True), device)


def recover_emissivity(kappa_map, target, source_pos, num_rays, step_size, radiation_velocity,
                       time_step, iters=200, lr=1e-2, j_init=None, callback=None,
                       substep_cap=None, state=None):
    """Run `iters` Adam steps; return (j, losses). kappa_map and target are 3-D float32
    device tensors. Pass `state` (an InverseState) to continue an earlier recovery; it is
    updated in place, and its losses list holds the whole history."""
    st = InverseState.start(target, j_init) if state is None else state
    field_buf = torch.empty_like(target)
    grad = torch.empty_like(target)
    gj, gk = torch.empty_like(target), torch.empty_like(target)
    hist = torch.empty(max(int(iters), 1), dtype=torch.float32, device=target.device)
    scale = 1.0 / target.numel()
    for it in range(iters):
        rtmi.trace_multi(st.j, kappa_map, source_pos, num_rays, step_size, radiation_velocity, time_step,
                         substep_cap=substep_cap, out=field_buf)
        rtmi.field_mse(field_buf, target, scale, grad=grad, loss=hist[it:it + 1])
        rtmi.trace_vjp(st.j, kappa_map, source_pos, num_rays, step_size, radiation_velocity, time_step,
                       grad, substep_cap=substep_cap, grad_j=gj, grad_kappa=gk)
        st.step += 1
        rtmi.adam_step(st.j, st.m, st.v, gj, None, lr, st.step)
        if callback is not None:
            callback(it, float(hist[it]))
    st.losses.extend(float(x) for x in hist[:iters].cpu())
    return st.j, st.losses[-iters:] if iters else []

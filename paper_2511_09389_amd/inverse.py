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


def fit_amplitude_and_opacity(j_template, kappa_template, kappa_scale, targets, source_pos, num_rays,
                              step_size, radiation_velocity, time_step, iters=150, lr=2e-2, start=(1.0, 1.0),
                              substep_cap=None, bin_weights=None):
    """Fit an emissivity amplitude A and a global opacity scale alpha, j = A j_template and
    kappa = alpha kappa_template, to the fields of several frequency bins (kappa_b =
    kappa_scale[b] kappa), by Adam on the sum of per-bin squared errors, each bin's divided
    by its target's sum of squares (or weighted by bin_weights, per voxel). The paper
    recovers a scalar amplitude through the tracer (Sec. 4); the opacity scale and the bins
    are the same gradient with more parameters.

    Every step runs in the library: the fields (rtmi_trace_bins), each bin's loss and
    gradient (rtmi_field_mse), the bins' adjoint (rtmi_trace_bins_vjp),
    dL/dA = <j_template, dL/dj> and dL/dalpha = <kappa_template, dL/dkappa> (rtmi_dot),
    the Adam step on (A, alpha) (rtmi_adam_step) and the scaled maps
    (rtmi_scaled_copy); the parameters never leave the device until the end.
    (The bins' scale gradients of rtmi_trace_bins_vjp give the same dL/dalpha:
    sum_b s_b dL/ds_b = alpha <kappa_template, dL/dkappa>.)
    Returns (A, alpha, losses)."""
    dev = j_template.device
    n_bins = targets.shape[0]
    scale = torch.as_tensor(kappa_scale, dtype=torch.float32).reshape(-1).to(dev)
    if scale.numel() != n_bins:
        raise ValueError("kappa_scale must have one entry per bin")
    cells = targets[0].numel()
    params = torch.tensor([float(start[0]), float(start[1])], dtype=torch.float32, device=dev)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    g = torch.zeros_like(params)
    j, kap = torch.empty_like(j_template), torch.empty_like(kappa_template)
    fields = torch.empty_like(targets)
    grads = torch.empty_like(targets)
    hist = torch.empty((max(int(iters), 1), n_bins), dtype=torch.float32, device=dev)
    weights = []
    for b in range(n_bins):
        if bin_weights is None:   # each bin's error relative to its own target
            ss = float(rtmi.dot(targets[b], targets[b]).cpu())
            weights.append(1.0 / max(ss, 1e-30))
        else:
            weights.append(float(bin_weights[b]) / cells)
    scale_host = scale.cpu().numpy()
    for it in range(iters):
        rtmi.scaled_copy(j_template, params[0:1], out=j)
        rtmi.scaled_copy(kappa_template, params[1:2], out=kap)
        rtmi.trace_bins(j, kap, source_pos, num_rays, step_size, radiation_velocity, time_step,
                        kappa_scale=scale_host, substep_cap=substep_cap, out=fields)
        for b in range(n_bins):
            rtmi.field_mse(fields[b], targets[b], weights[b], grad=grads[b], loss=hist[it, b:b + 1])
        gj, gk, _ = rtmi.trace_bins_vjp(j, kap, source_pos, num_rays, step_size, radiation_velocity, time_step,
                                        grads, kappa_scale=scale_host, substep_cap=substep_cap)
        # j = A j_template and kappa = alpha kappa_template (gk already sums the bins through
        # their scales): dL/dA = <j_template, dL/dj>, dL/dalpha = <kappa_template, dL/dkappa>
        rtmi.dot(j_template, gj, out=g[0:1])
        rtmi.dot(kappa_template, gk, out=g[1:2])
        rtmi.adam_step(params, m, v, g, None, lr, it + 1)
    p = params.cpu()
    return float(p[0]), float(p[1]), [float(x) for x in hist[:iters].cpu().numpy().sum(axis=1)]

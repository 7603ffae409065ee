"""torch.autograd binding of the march: the forward is rtmi_trace_multi, the backward
is the library's hand-written adjoint (rtmi_trace_vjp). Gradients flow to j and kappa."""

import torch

from . import rtmi


class MarchField(torch.autograd.Function):
    """J(j, kappa) for fixed sources; differentiable in j and kappa."""

    @staticmethod
    def forward(ctx, j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                time_step, substep_cap):
        j_map = j_map.contiguous()
        kappa_map = kappa_map.contiguous()
        out = rtmi.trace_multi(j_map, kappa_map, source_pos, num_rays, step_size,
                               radiation_velocity, time_step, substep_cap=substep_cap)
        ctx.save_for_backward(j_map, kappa_map)
        ctx.args = (source_pos, num_rays, step_size, radiation_velocity, time_step, substep_cap)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        j_map, kappa_map = ctx.saved_tensors
        source_pos, num_rays, ds, c, dt, caps = ctx.args
        gj, gk = rtmi.trace_vjp(j_map, kappa_map, source_pos, num_rays, ds, c, dt,
                                grad_out.contiguous().float(), substep_cap=caps)
        return (gj if ctx.needs_input_grad[0] else None,
                gk if ctx.needs_input_grad[1] else None, None, None, None, None, None, None)


def march_field(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                time_step, substep_cap=None):
    return MarchField.apply(j_map, kappa_map, source_pos, num_rays, step_size,
                            radiation_velocity, time_step, substep_cap)

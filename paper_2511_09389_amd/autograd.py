"""torch.autograd binding of the march: the forwards are rtmi_trace_multi and
rtmi_trace_bins, the backwards the library's hand-written adjoints (rtmi_trace_vjp,
rtmi_trace_bins_vjp). Gradients flow to j, kappa and the bins' opacity scales."""

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


class MarchBins(torch.autograd.Function):
    """J_b(j, kappa) of the frequency bins for fixed sources (rtmi_trace_bins), with the
    adjoint of every bin (rtmi_trace_bins_vjp) as its backward. j and kappa are 3-D (shared
    by the bins) or 4-D [B][...]; kappa_scale is a [B] float32 device tensor with a shared
    kappa (kappa_b = kappa_scale[b] kappa), differentiable too, or None with per-bin maps."""

    @staticmethod
    def forward(ctx, j_maps, kappa_maps, kappa_scale, source_pos, num_rays, step_size, radiation_velocity,
                time_step, substep_cap):
        j_maps = j_maps.contiguous()
        kappa_maps = kappa_maps.contiguous()
        scale_host = None if kappa_scale is None else kappa_scale.detach().float().cpu().numpy()
        out = rtmi.trace_bins(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
                              time_step, kappa_scale=scale_host, substep_cap=substep_cap)
        ctx.save_for_backward(j_maps, kappa_maps)
        ctx.scale_host = scale_host
        ctx.args = (source_pos, num_rays, step_size, radiation_velocity, time_step, substep_cap)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        j_maps, kappa_maps = ctx.saved_tensors
        source_pos, num_rays, ds, c, dt, caps = ctx.args
        want_scale = ctx.scale_host is not None and ctx.needs_input_grad[2]
        gj, gk, gs = rtmi.trace_bins_vjp(j_maps, kappa_maps, source_pos, num_rays, ds, c, dt,
                                         grad_out.contiguous().float(), kappa_scale=ctx.scale_host,
                                         substep_cap=caps, scale_grad=want_scale)
        return (gj if ctx.needs_input_grad[0] else None, gk if ctx.needs_input_grad[1] else None,
                gs if want_scale else None, None, None, None, None, None, None)


def march_bins(j_maps, kappa_maps, kappa_scale, source_pos, num_rays, step_size, radiation_velocity,
               time_step, substep_cap=None):
    return MarchBins.apply(j_maps, kappa_maps, kappa_scale, source_pos, num_rays, step_size,
                           radiation_velocity, time_step, substep_cap)

"""Host-side checks of the Python binding (no GPU): every buffer a caller supplies is
checked against the shape the call reads or writes before any pointer reaches the library,
which cannot know buffer sizes. Mis-sized buffers raise ValueError; the bogus CPU tensors
used here never reach a device call."""

import pytest
import torch


@pytest.fixture(scope="module")
def rt():
    from paper_2511_09389_amd import rtmi
    return rtmi


G = (6, 5, 4)


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


def bf16(*shape):
    return torch.zeros(shape, dtype=torch.bfloat16)


def test_march_outputs_are_shape_checked(rt):
    j, k = f32(*G), f32(*G)
    with pytest.raises(ValueError, match="out"):
        rt.trace_single(j, k, (1, 1, 1), 8, 0.5, 2.0, 1.0, out=f32(6, 5, 3))
    with pytest.raises(ValueError, match="out"):
        rt.trace_multi(j, k, [[1, 1, 1]], 8, 0.5, 2.0, 1.0, out=f32(5, 5, 4))
    with pytest.raises(ValueError, match="out"):
        rt.trace_bins(j, k, [[1, 1, 1]], 8, 0.5, 2.0, 1.0, kappa_scale=[1.0, 0.5], out=f32(1, *G))
    with pytest.raises(ValueError, match="kappa_map"):
        rt.trace_multi(j, f32(6, 5, 5), [[1, 1, 1]], 8, 0.5, 2.0, 1.0)


def test_adjoint_buffers_are_shape_checked(rt):
    j, k, g = f32(*G), f32(*G), f32(*G)
    with pytest.raises(ValueError, match="grad_j"):
        rt.trace_vjp(j, k, [[1, 1, 1]], 8, 0.5, 2.0, 1.0, g, grad_j=f32(6, 5))
    with pytest.raises(ValueError, match="grad_kappa"):
        rt.trace_vjp(j, k, [[1, 1, 1]], 8, 0.5, 2.0, 1.0, g, grad_kappa=f32(60, 2))
    with pytest.raises(ValueError, match="grad_field"):
        rt.trace_vjp(j, k, [[1, 1, 1]], 8, 0.5, 2.0, 1.0, f32(6, 5, 3))


def test_conv_buffers_are_shape_checked(rt):
    C = rt.CONV_CHANNELS
    x = bf16(1, 4, 4, 16, C)
    w = bf16(27, C, C)
    with pytest.raises(ValueError, match="y"):
        rt.conv3d_forward(x, w, y=bf16(1, 4, 4, 8, C))
    with pytest.raises(ValueError, match="z"):
        rt.conv3d_forward(x, w, z=f32(1, 4, 4, 15, C))
    with pytest.raises(ValueError, match="w"):
        rt.conv3d_forward(x, bf16(26, C, C))
    with pytest.raises(ValueError, match="dh"):
        rt.conv3d_backward_data(x, w, dh=f32(1, 4, 4, 8, C))
    with pytest.raises(ValueError, match="dz_prev"):
        rt.conv3d_backward_data(x, w, dz_prev=bf16(1, 2, 4, 16, C))
    with pytest.raises(ValueError, match="dw"):
        rt.conv3d_backward_weight(x, x, f32(27, C), f32(C))
    with pytest.raises(ValueError, match="db"):
        rt.conv3d_backward_weight(x, x, f32(27, C, C), f32(C - 1))


def test_loss_adam_and_surrogate_buffers_are_shape_checked(rt):
    C = rt.CONV_CHANNELS
    y = bf16(1, 4, 4, 16, C)
    with pytest.raises(ValueError, match="channels"):
        rt.mse_loss(y, f32(4, 4, 8), 1.0, bf16(1, 4, 4, 16, C), f32(1))
    with pytest.raises(ValueError, match="dz"):
        rt.mse_loss(y, f32(4, 4, 16), 1.0, bf16(1, 4, 4, 8, C), f32(1))
    with pytest.raises(ValueError, match="m"):
        rt.adam_step(f32(10), f32(9), f32(10), f32(10), None, 1e-3, 1)
    with pytest.raises(ValueError, match="w_bf16"):
        rt.adam_step(f32(10), f32(10), f32(10), f32(10), bf16(5), 1e-3, 1)
    j = f32(4, 4, 16)
    with pytest.raises(ValueError, match="cheap"):
        rt.surrogate_features(j, f32(4, 4, 16), f32(4, 4, 8), [0, 1, 1, 0, 1, 1e-6])
    with pytest.raises(ValueError, match="x"):
        rt.surrogate_features(j, j, j, [0, 1, 1, 0, 1, 1e-6], x=bf16(1, 4, 4, 8, C))
    with pytest.raises(ValueError, match="field"):
        rt.surrogate_output(y, j, f32(2), field=f32(4, 4, 8))
    with pytest.raises(ValueError, match="y"):
        rt.surrogate_output(bf16(1, 4, 4, 8, C), j, f32(2))

"""Python binding of librtmi (ctypes): argument marshalling only.

Every step of the march runs in the HIP library; this module checks tensor placement,
dtype and layout, passes raw device pointers, host arrays and the current HIP stream,
and turns non-zero status codes into exceptions. Importing it fails loudly when the
library has not been built: there is no fallback implementation.
"""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtmi.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_SHAPE = -2
ERR_NONFINITE = -3
ERR_HIP = -4
ERR_UNSUPPORTED = -5
ERR_RANGE = -6
ACCUM_ATOMIC = 0
ACCUM_DETERMINISTIC = 1
PATH_TILED = 0
PATH_DIRECT = 1
KERNEL_RECORD = 0
KERNEL_TILE = 1
KERNEL_DIRECT = 2
KERNEL_TABLE = 3
KERNEL_GATHER = 4


class RtmiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librtmi error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("accum_mode", ctypes.c_int32), ("directions", ctypes.c_void_p),
                ("ray_weight", ctypes.c_float), ("path", ctypes.c_int32),
                ("tile_item_chunks", ctypes.c_int32), ("record_capacity", ctypes.c_int64),
                ("gather_table", ctypes.c_int32), ("sources_per_launch", ctypes.c_int32),
                ("tile_groups_per_cu", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_09389_amd.build` "
                          "(or __graft_entry__.build()); there is no non-HIP fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    sig = {
        "rtmi_last_error": (ctypes.c_char_p, []),
        "rtmi_version": (I32, []),
        "rtmi_num_substeps": (I64, [F32, F32, F32, I32]),
        "rtmi_fibonacci_directions": (I32, [I32, P]),
        "rtmi_prepare": (I32, [I32]),
        "rtmi_reserve": (I32, [I64]),
        "rtmi_release_workspaces": (I32, []),
        "rtmi_dropped_records": (I32, [ctypes.POINTER(ctypes.c_int64)]),
        "rtmi_trace_single": (I32, [P, P, I32, I32, I32, P, I32, F32, F32, F32, P, P]),
        "rtmi_trace_multi": (I32, [P, P, I32, I32, I32, I32, P, P, P, F32, F32, F32, P, P]),
        "rtmi_trace_bins": (I32, [P, I64, P, I64, P, I32, I32, I32, I32, I32, P, P, P, F32, F32,
                                  F32, P, ctypes.POINTER(Options), P]),
        "rtmi_trace_bins_static": (I32, [P, I64, P, I64, P, I32, I32, I32, I32, I32, P, P, P, F32, F32,
                                         F32, P, ctypes.POINTER(Options), P]),
        "rtmi_static_scratch_bytes": (I64, []),
        "rtmi_field_mse": (I32, [P, P, I64, F32, P, P, P]),
        "rtmi_dot": (I32, [P, P, I64, P, P]),
        "rtmi_scaled_copy": (I32, [P, P, P, I64, P]),
        "rtmi_debug_rays": (I32, [P, P, I32, I32, I32, P, I32, F32, F32, F32, I32, P, P, P]),
        "rtmi_trace_vjp": (I32, [P, P, I32, I32, I32, I32, P, P, P, F32, F32, F32, P, P, P, P]),
        "rtmi_trace_bins_vjp": (I32, [P, I64, P, I64, P, I32, I32, I32, I32, I32, P, P, P, F32, F32, F32,
                                      P, P, P, P, P]),
        "rtmi_plan_create": (I32, [I32, I32, I32, I32, P, P, P, I32, I64, I64, P, F32, F32, F32,
                                   ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p)]),
        "rtmi_plan_execute": (I32, [P, P, P, P, P]),
        "rtmi_plan_workspace_bytes": (I64, [P]),
        "rtmi_plan_destroy": (I32, [P]),
        "rtmi_conv3d_forward": (I32, [P, P, P, P, I32, I32, I32, I32, I32, P, P, P]),
        "rtmi_conv3d_backward_data": (I32, [P, P, P, P, I32, I32, I32, I32, P, P, P]),
        "rtmi_conv3d_backward_weight": (I32, [P, P, I32, I32, I32, I32, P, P, P]),
        "rtmi_mse_loss": (I32, [P, P, I64, F32, P, P, P]),
        "rtmi_adam_step": (I32, [P, P, P, P, P, I64, F32, F32, F32, F32, I32, P]),
        "rtmi_surrogate_features": (I32, [P, P, P, I64, P, P, P, P]),
        "rtmi_surrogate_output": (I32, [P, P, I64, P, P, P, P]),
        "rtmi_timing_enable": (I32, [I32]),
        "rtmi_timing_read": (I32, [I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(code):
    if code != OK:
        raise RtmiError(int(code), lib.rtmi_last_error().decode())


def _dev(t, name, ndim=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (C order)")
    if ndim is not None and t.dim() not in ((ndim,) if isinstance(ndim, int) else ndim):
        raise ValueError(f"{name} has {t.dim()} dims, expected {ndim}")
    return ctypes.c_void_p(t.data_ptr())


def _same(t, name, shape, device):
    """A caller-supplied buffer must have exactly the shape the call reads or writes, on
    the call's device: the library trusts its sizes, so a short buffer would be overrun."""
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _host_f32(a, shape_last=None):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape_last is not None:
        arr = arr.reshape(-1, shape_last)
    return arr


def version():
    return int(lib.rtmi_version())


def num_substeps(step_size, radiation_velocity, time_step, cap=0):
    n = int(lib.rtmi_num_substeps(step_size, radiation_velocity, time_step, int(cap)))
    if n < 0:
        raise RtmiError(n, lib.rtmi_last_error().decode())
    return n


def fibonacci_directions(n):
    out = np.empty((int(n), 3), dtype=np.float32)
    _check(lib.rtmi_fibonacci_directions(int(n), out.ctypes.data_as(ctypes.c_void_p)))
    return out


def prepare(num_rays, device=None):
    with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
        _check(lib.rtmi_prepare(int(num_rays)))


def reserve(nbytes, device=None):
    """Grow the device's workspace pool to at least nbytes (tiled path)."""
    with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
        _check(lib.rtmi_reserve(int(nbytes)))


def release_workspaces(device=None):
    """Wait for the device, then free the workspaces stateless calls keep per stream."""
    with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
        _check(lib.rtmi_release_workspaces())


def dropped_records(device=None):
    """Wait for the device; return (and reset) the chunk records that stateless tiled calls
    could not store since the last query. 0 means no deposit was lost."""
    n = ctypes.c_int64(0)
    with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
        code = lib.rtmi_dropped_records(ctypes.byref(n))
    if code not in (OK, ERR_RANGE):
        _check(code)
    return int(n.value)


def _new_field(shape, like):
    return torch.empty(shape, dtype=torch.float32, device=like.device)


def trace_single(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                 time_step, out=None):
    """The single-source kernel; returns J as a float32 tensor shaped like j_map."""
    if tuple(kappa_map.shape) != tuple(j_map.shape):
        raise ValueError("j_map and kappa_map must have the same shape")
    nx, ny, nz = j_map.shape
    _same(kappa_map, "kappa_map", j_map.shape, j_map.device)
    out = _new_field(j_map.shape, j_map) if out is None else _same(out, "out", j_map.shape, j_map.device)
    src = _host_f32(source_pos).reshape(3)
    with torch.cuda.device(j_map.device):
        _check(lib.rtmi_trace_single(_dev(j_map, "j_map", 3), _dev(kappa_map, "kappa_map", 3),
                                     nx, ny, nz, src.ctypes.data_as(ctypes.c_void_p), int(num_rays),
                                     step_size, radiation_velocity, time_step,
                                     _dev(out, "out", 3), _stream(j_map.device)))
    return out


def _per_source(source_pos, num_rays, substep_cap):
    src = _host_f32(source_pos, 3)
    n_src = src.shape[0]
    nr = np.ascontiguousarray(np.broadcast_to(np.asarray(num_rays, np.int32), (n_src,)))
    cap = None
    if substep_cap is not None:
        cap = np.ascontiguousarray(np.broadcast_to(np.asarray(substep_cap, np.int32), (n_src,)))
    return src, nr, cap


def trace_multi(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                time_step, substep_cap=None, out=None):
    """Sum over sources of the single-source kernel with a shared j_map."""
    if tuple(kappa_map.shape) != tuple(j_map.shape):
        raise ValueError("j_map and kappa_map must have the same shape")
    nx, ny, nz = j_map.shape
    src, nr, cap = _per_source(source_pos, num_rays, substep_cap)
    _same(kappa_map, "kappa_map", j_map.shape, j_map.device)
    out = _new_field(j_map.shape, j_map) if out is None else _same(out, "out", j_map.shape, j_map.device)
    with torch.cuda.device(j_map.device):
        _check(lib.rtmi_trace_multi(_dev(j_map, "j_map", 3), _dev(kappa_map, "kappa_map", 3),
                                    nx, ny, nz, src.shape[0], src.ctypes.data_as(ctypes.c_void_p),
                                    nr.ctypes.data_as(ctypes.c_void_p),
                                    None if cap is None else cap.ctypes.data_as(ctypes.c_void_p),
                                    step_size, radiation_velocity, time_step, _dev(out, "out", 3),
                                    _stream(j_map.device)))
    return out


def trace_bins(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
               time_step, kappa_scale=None, substep_cap=None, out=None, deterministic=False,
               directions=None, ray_weight=0.0, path=PATH_TILED, tile_item_chunks=0, record_capacity=0,
               gather_table=0, sources_per_launch=0, tile_groups_per_cu=0):
    """Frequency bins as a batch axis. j_maps / kappa_maps are 3-D (shared by all bins) or
    4-D [B][nx][ny][nz]; a 3-D kappa with kappa_scale gives kappa_b = kappa * scale[b].
    Returns a [B][nx][ny][nz] float32 tensor."""
    return _bins_call(lib.rtmi_trace_bins, j_maps, kappa_maps, source_pos, num_rays, step_size,
                      radiation_velocity, time_step, kappa_scale, substep_cap, out, deterministic,
                      directions, ray_weight, path, tile_item_chunks, record_capacity, gather_table,
                      sources_per_launch, tile_groups_per_cu)


def trace_bins_static(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
                      time_step, kappa_scale=None, substep_cap=None, out=None, deterministic=False,
                      path=PATH_TILED, tile_item_chunks=0, record_capacity=0, gather_table=0,
                      sources_per_launch=0):
    """trace_bins through rtmi_trace_bins_static, which allocates nothing: its scratch is
    the library's static per-device array (static_scratch_bytes()). Every N_Omega must have
    been prepared (prepare()); pass `out` to keep this call free of allocation in torch too."""
    return _bins_call(lib.rtmi_trace_bins_static, j_maps, kappa_maps, source_pos, num_rays, step_size,
                      radiation_velocity, time_step, kappa_scale, substep_cap, out, deterministic,
                      None, 0.0, path, tile_item_chunks, record_capacity, gather_table, sources_per_launch)


def static_scratch_bytes():
    return int(lib.rtmi_static_scratch_bytes())


def _bins_call(entry, j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
               time_step, kappa_scale, substep_cap, out, deterministic, directions, ray_weight, path,
               tile_item_chunks, record_capacity, gather_table=0, sources_per_launch=0, tile_groups_per_cu=0):
    grid = tuple(j_maps.shape[-3:])
    if tuple(kappa_maps.shape[-3:]) != grid:
        raise ValueError("j and kappa grids differ")
    cells = grid[0] * grid[1] * grid[2]
    b_j = j_maps.shape[0] if j_maps.dim() == 4 else 1
    b_k = kappa_maps.shape[0] if kappa_maps.dim() == 4 else 1
    scale = None
    if kappa_maps.dim() == 4:
        if kappa_scale is not None:
            raise ValueError("kappa_scale applies to a shared 3-D kappa only")
    elif kappa_scale is not None:
        scale = _host_f32(kappa_scale).ravel()
    n_bins = max(b_j, b_k, 1 if scale is None else scale.size)
    for nb, what in ((b_j, "j_maps"), (b_k, "kappa_maps")):
        if nb not in (1, n_bins):
            raise ValueError(f"{what} has {nb} bins, expected 1 or {n_bins}")
    if scale is not None and scale.size != n_bins:
        raise ValueError("kappa_scale must have one entry per bin")
    src, nr, cap = _per_source(source_pos, num_rays, substep_cap)
    if kappa_maps.device != j_maps.device:
        raise ValueError("j_maps and kappa_maps must be on one device")
    out = _new_field((n_bins,) + grid, j_maps) if out is None else \
        _same(out, "out", (n_bins,) + grid, j_maps.device)
    opts = Options(ACCUM_DETERMINISTIC if deterministic else ACCUM_ATOMIC, None, float(ray_weight),
                   int(path), int(tile_item_chunks), int(record_capacity), int(gather_table),
                   int(sources_per_launch), int(tile_groups_per_cu))
    dirs = None
    if directions is not None:
        dirs = _host_f32(directions, 3)
        opts.directions = dirs.ctypes.data
    with torch.cuda.device(j_maps.device):
        _check(entry(
            _dev(j_maps, "j_maps", (3, 4)), cells if (j_maps.dim() == 4 and b_j > 1) else 0,
            _dev(kappa_maps, "kappa_maps", (3, 4)), cells if (kappa_maps.dim() == 4 and b_k > 1) else 0,
            None if scale is None else scale.ctypes.data_as(ctypes.c_void_p), n_bins,
            grid[0], grid[1], grid[2], src.shape[0], src.ctypes.data_as(ctypes.c_void_p),
            nr.ctypes.data_as(ctypes.c_void_p),
            None if cap is None else cap.ctypes.data_as(ctypes.c_void_p),
            step_size, radiation_velocity, time_step, _dev(out, "out", 4), ctypes.byref(opts),
            _stream(j_maps.device)))
    return out


class Plan:
    """The batched march prepared once (rtmi_plan_*): sources with their own N_Omega and
    substep caps, times bins, as trace_bins computes them. execute() only enqueues kernels
    on the current stream, so it can be captured in a torch.cuda.CUDAGraph and replayed.
    Executions of one plan must be stream-ordered (they share its workspace)."""

    def __init__(self, grid, source_pos, num_rays, step_size, radiation_velocity, time_step,
                 n_bins=1, kappa_scale=None, per_bin_j=False, per_bin_kappa=False,
                 substep_cap=None, deterministic=False, directions=None, ray_weight=0.0,
                 tile_item_chunks=0, gather_table=0, sources_per_launch=0, tile_groups_per_cu=0,
                 device=None):
        self.grid = tuple(int(v) for v in grid)
        cells = self.grid[0] * self.grid[1] * self.grid[2]
        src, nr, cap = _per_source(source_pos, num_rays, substep_cap)
        scale = None
        if kappa_scale is not None:
            if per_bin_kappa:
                raise ValueError("kappa_scale applies to a shared kappa only")
            scale = _host_f32(kappa_scale).ravel()
            if scale.size != n_bins:
                raise ValueError("kappa_scale must have one entry per bin")
        self.n_bins = int(n_bins)
        self.per_bin_j, self.per_bin_kappa = bool(per_bin_j), bool(per_bin_kappa)
        opts = Options(ACCUM_DETERMINISTIC if deterministic else ACCUM_ATOMIC, None,
                       float(ray_weight), PATH_TILED, int(tile_item_chunks), 0, int(gather_table),
                       int(sources_per_launch), int(tile_groups_per_cu))
        dirs = None
        if directions is not None:
            dirs = _host_f32(directions, 3)
            opts.directions = dirs.ctypes.data
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.rtmi_plan_create(
                self.grid[0], self.grid[1], self.grid[2], src.shape[0],
                src.ctypes.data_as(ctypes.c_void_p), nr.ctypes.data_as(ctypes.c_void_p),
                None if cap is None else cap.ctypes.data_as(ctypes.c_void_p), self.n_bins,
                cells if per_bin_j else 0, cells if per_bin_kappa else 0,
                None if scale is None else scale.ctypes.data_as(ctypes.c_void_p),
                step_size, radiation_velocity, time_step, ctypes.byref(opts), ctypes.byref(handle)))
        self._handle = handle

    @property
    def workspace_bytes(self):
        return int(lib.rtmi_plan_workspace_bytes(self._handle))

    def execute(self, j_maps, kappa_maps, out=None):
        if self._handle is None:
            raise RuntimeError("plan is closed")
        for t, per_bin, name in ((j_maps, self.per_bin_j, "j_maps"), (kappa_maps, self.per_bin_kappa, "kappa_maps")):
            want = ((self.n_bins,) + self.grid) if per_bin else self.grid
            if tuple(t.shape) != want:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want}")
        if out is None:
            out = _new_field((self.n_bins,) + self.grid, j_maps)
        elif tuple(out.shape) != (self.n_bins,) + self.grid:
            raise ValueError(f"out has shape {tuple(out.shape)}, expected {(self.n_bins,) + self.grid}")
        with torch.cuda.device(self.device):
            _check(lib.rtmi_plan_execute(self._handle, _dev(j_maps, "j_maps", (3, 4)),
                                         _dev(kappa_maps, "kappa_maps", (3, 4)), _dev(out, "out", 4),
                                         _stream(self.device)))
        return out

    def close(self):
        if getattr(self, "_handle", None) is not None:
            lib.rtmi_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trace_vjp(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity, time_step,
              grad_field, substep_cap=None, grad_j=None, grad_kappa=None):
    """Adjoint of trace_multi: (dL/dj, dL/dkappa) for dL/dJ = grad_field (all 3-D float32)."""
    if tuple(kappa_map.shape) != tuple(j_map.shape) or tuple(grad_field.shape) != tuple(j_map.shape):
        raise ValueError("j_map, kappa_map and grad_field must have the same shape")
    nx, ny, nz = j_map.shape
    src, nr, cap = _per_source(source_pos, num_rays, substep_cap)
    for t, name in ((kappa_map, "kappa_map"), (grad_field, "grad_field")):
        _same(t, name, j_map.shape, j_map.device)
    grad_j = _new_field(j_map.shape, j_map) if grad_j is None else _same(grad_j, "grad_j", j_map.shape, j_map.device)
    grad_kappa = _new_field(j_map.shape, j_map) if grad_kappa is None else \
        _same(grad_kappa, "grad_kappa", j_map.shape, j_map.device)
    with torch.cuda.device(j_map.device):
        _check(lib.rtmi_trace_vjp(_dev(j_map, "j_map", 3), _dev(kappa_map, "kappa_map", 3),
                                  nx, ny, nz, src.shape[0], src.ctypes.data_as(ctypes.c_void_p),
                                  nr.ctypes.data_as(ctypes.c_void_p),
                                  None if cap is None else cap.ctypes.data_as(ctypes.c_void_p),
                                  step_size, radiation_velocity, time_step,
                                  _dev(grad_field, "grad_field", 3), _dev(grad_j, "grad_j", 3),
                                  _dev(grad_kappa, "grad_kappa", 3), _stream(j_map.device)))
    return grad_j, grad_kappa


def trace_bins_vjp(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity, time_step,
                   grad_fields, kappa_scale=None, substep_cap=None, scale_grad=False, grad_j=None,
                   grad_kappa=None, grad_kappa_scale=None):
    """Adjoint of trace_bins for dL/dJ_b = grad_fields ([B][nx][ny][nz]). j_maps and
    kappa_maps are 3-D (shared by the bins) or 4-D [B][...], as for trace_bins. Returns
    (dL/dj, dL/dkappa, dL/dkappa_scale): gradients of shared maps are 3-D (summed over bins,
    kappa's through each bin's scale), of per-bin maps 4-D; the scale gradient is a [B]
    float32 device tensor when scale_grad is set (a shared kappa only), else None."""
    grid = tuple(j_maps.shape[-3:])
    if tuple(kappa_maps.shape[-3:]) != grid:
        raise ValueError("j and kappa grids differ")
    cells = grid[0] * grid[1] * grid[2]
    n_bins = grad_fields.shape[0] if grad_fields.dim() == 4 else 0
    if n_bins < 1:
        raise ValueError("grad_fields must be [B][nx][ny][nz]")
    _same(grad_fields, "grad_fields", (n_bins,) + grid, j_maps.device)
    for t, what in ((j_maps, "j_maps"), (kappa_maps, "kappa_maps")):
        if t.dim() == 4 and t.shape[0] != n_bins:
            raise ValueError(f"{what} has {t.shape[0]} bins, expected {n_bins}")
        if t.device != j_maps.device:
            raise ValueError("j_maps and kappa_maps must be on one device")
    per_j, per_k = j_maps.dim() == 4, kappa_maps.dim() == 4
    scale = None
    if per_k:
        if kappa_scale is not None or scale_grad:
            raise ValueError("kappa_scale and its gradient apply to a shared 3-D kappa only")
    elif kappa_scale is not None:
        scale = _host_f32(kappa_scale).ravel()
        if scale.size != n_bins:
            raise ValueError("kappa_scale must have one entry per bin")
    src, nr, cap = _per_source(source_pos, num_rays, substep_cap)
    gj_shape = (n_bins,) + grid if per_j else grid
    gk_shape = (n_bins,) + grid if per_k else grid
    grad_j = _new_field(gj_shape, j_maps) if grad_j is None else _same(grad_j, "grad_j", gj_shape, j_maps.device)
    grad_kappa = _new_field(gk_shape, j_maps) if grad_kappa is None else \
        _same(grad_kappa, "grad_kappa", gk_shape, j_maps.device)
    gs = None
    if scale_grad:
        gs = _new_field((n_bins,), j_maps) if grad_kappa_scale is None else \
            _same(grad_kappa_scale, "grad_kappa_scale", (n_bins,), j_maps.device)
    with torch.cuda.device(j_maps.device):
        _check(lib.rtmi_trace_bins_vjp(
            _dev(j_maps, "j_maps", (3, 4)), cells if per_j else 0,
            _dev(kappa_maps, "kappa_maps", (3, 4)), cells if per_k else 0,
            None if scale is None else scale.ctypes.data_as(ctypes.c_void_p), n_bins,
            grid[0], grid[1], grid[2], src.shape[0], src.ctypes.data_as(ctypes.c_void_p),
            nr.ctypes.data_as(ctypes.c_void_p), None if cap is None else cap.ctypes.data_as(ctypes.c_void_p),
            step_size, radiation_velocity, time_step, _dev(grad_fields, "grad_fields", 4),
            _dev(grad_j, "grad_j", (3, 4)), _dev(grad_kappa, "grad_kappa", (3, 4)),
            None if gs is None else _dev(gs, "grad_kappa_scale", 1), _stream(j_maps.device)))
    return grad_j, grad_kappa, gs


def dot(a, b, out=None):
    """out[0] = sum(a * b) over two equal-sized float32 device tensors (binary64 sum)."""
    if a.numel() != b.numel() or a.numel() < 1:
        raise ValueError("dot needs two non-empty tensors of one size")
    out = torch.empty(1, dtype=torch.float32, device=a.device) if out is None else _same(out, "out", (1,), a.device)
    with torch.cuda.device(a.device):
        _check(lib.rtmi_dot(_dev(a, "a"), _dev(_same(b, "b", tuple(b.shape), a.device), "b"), a.numel(),
                            _dev(out, "out", 1), _stream(a.device)))
    return out


def scaled_copy(x, scale, out=None):
    """out = scale[0] * x, with scale a float32 device tensor of at least one element."""
    if scale.numel() < 1:
        raise ValueError("scale needs one element")
    out = torch.empty_like(x) if out is None else _same(out, "out", tuple(x.shape), x.device)
    with torch.cuda.device(x.device):
        _check(lib.rtmi_scaled_copy(_dev(x, "x"), _dev(_same(scale, "scale", tuple(scale.shape), x.device), "scale"),
                                    _dev(out, "out"), x.numel(), _stream(x.device)))
    return out


def field_mse(field, target, scale=None, grad=None, loss=None):
    """(loss, grad): loss = scale * sum (field - target)^2 written to a one-element device
    tensor, grad = dL/dfield. scale defaults to 1 / numel (the mean squared error)."""
    dev = field.device
    _same(target, "target", field.shape, dev)
    grad = torch.empty_like(field) if grad is None else _same(grad, "grad", field.shape, dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev) if loss is None else _same(loss, "loss", (1,), dev)
    scale = 1.0 / field.numel() if scale is None else float(scale)
    with torch.cuda.device(dev):
        _check(lib.rtmi_field_mse(_dev(field, "field"), _dev(target, "target"), field.numel(), scale,
                                  _dev(grad, "grad"), _dev(loss, "loss"), _stream(dev)))
    return loss, grad


def debug_rays(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
               time_step, cap=0):
    """Per-ray I_{k+1} and tau_{k+1} of one source, lattice order: two [N][N_s] tensors."""
    nx, ny, nz = j_map.shape
    _same(kappa_map, "kappa_map", j_map.shape, j_map.device)
    n_s = num_substeps(step_size, radiation_velocity, time_step, cap)
    rays = torch.zeros((int(num_rays), n_s), dtype=torch.float32, device=j_map.device)
    tau = torch.zeros_like(rays)
    src = _host_f32(source_pos).reshape(3)
    with torch.cuda.device(j_map.device):
        _check(lib.rtmi_debug_rays(_dev(j_map, "j_map", 3), _dev(kappa_map, "kappa_map", 3),
                                   nx, ny, nz, src.ctypes.data_as(ctypes.c_void_p), int(num_rays),
                                   step_size, radiation_velocity, time_step, int(cap),
                                   _dev(rays, "out_rays", 2), _dev(tau, "out_tau", 2),
                                   _stream(j_map.device)))
    return rays, tau


# ---- surrogate network building blocks (channels-last, 32 channels) ----

CONV_CHANNELS = 32


def _act(t, name, dtype, ndim=5):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and (t.dim() != ndim or t.shape[-1] != CONV_CHANNELS):
        raise ValueError(f"{name} must be [n][d][h][w][{CONV_CHANNELS}] (got {tuple(t.shape)})")
    return ctypes.c_void_p(t.data_ptr())


def _opt(t, name, dtype, ndim=5):
    return None if t is None else _act(t, name, dtype, ndim)


WEIGHT_SHAPE = (27, CONV_CHANNELS, CONV_CHANNELS)


def _optsame(t, name, shape, device):
    return None if t is None else _same(t, name, shape, device)


def conv3d_forward(x, w, bias=None, residual=None, gelu=False, z=None, y=None):
    """y = act(conv(x, w) + bias) + residual, bf16 channels-last; z (fp32) if given."""
    n, d, h, wd, _ = x.shape
    dev = x.device
    _same(w, "w", WEIGHT_SHAPE, dev)
    _optsame(bias, "bias", (CONV_CHANNELS,), dev)
    _optsame(residual, "residual", x.shape, dev)
    _optsame(z, "z", x.shape, dev)
    y = torch.empty_like(x) if y is None else _same(y, "y", x.shape, dev)
    with torch.cuda.device(dev):
        _check(lib.rtmi_conv3d_forward(_act(x, "x", torch.bfloat16), _act(w, "w", torch.bfloat16, None),
                                       _opt(bias, "bias", torch.float32, None),
                                       _opt(residual, "residual", torch.bfloat16), int(bool(gelu)),
                                       n, d, h, wd, _act(y, "y", torch.bfloat16),
                                       _opt(z, "z", torch.float32), _stream(dev)))
    return y


def conv3d_backward_data(dz, w, residual=None, zprev=None, dh=None, dz_prev=None):
    n, d, h, wd, _ = dz.shape
    dev = dz.device
    _same(w, "w", WEIGHT_SHAPE, dev)
    for t, name in ((residual, "residual"), (zprev, "zprev"), (dh, "dh"), (dz_prev, "dz_prev")):
        _optsame(t, name, dz.shape, dev)
    with torch.cuda.device(dev):
        _check(lib.rtmi_conv3d_backward_data(_act(dz, "dz", torch.bfloat16), _act(w, "w", torch.bfloat16, None),
                                             _opt(residual, "residual", torch.float32),
                                             _opt(zprev, "zprev", torch.float32), n, d, h, wd,
                                             _opt(dh, "dh", torch.float32),
                                             _opt(dz_prev, "dz_prev", torch.bfloat16), _stream(dev)))
    return dh, dz_prev


def conv3d_backward_weight(x, dz, dw, db):
    n, d, h, wd, _ = x.shape
    dev = x.device
    _same(dz, "dz", x.shape, dev)
    _same(dw, "dw", WEIGHT_SHAPE, dev)
    _same(db, "db", (CONV_CHANNELS,), dev)
    with torch.cuda.device(dev):
        _check(lib.rtmi_conv3d_backward_weight(_act(x, "x", torch.bfloat16), _act(dz, "dz", torch.bfloat16),
                                               n, d, h, wd, _act(dw, "dw", torch.float32, None),
                                               _act(db, "db", torch.float32, None), _stream(dev)))
    return dw, db


def mse_loss(y, target, scale, dz, loss):
    nvox = target.numel()
    dev = y.device
    if y.dim() != 5 or y.numel() != nvox * CONV_CHANNELS:
        raise ValueError(f"y must hold {CONV_CHANNELS} channels per target voxel (got {tuple(y.shape)})")
    _same(target, "target", target.shape, dev)
    _same(dz, "dz", y.shape, dev)
    if loss.numel() < 1:
        raise ValueError("loss must hold one element")
    _same(loss, "loss", loss.shape, dev)
    with torch.cuda.device(dev):
        _check(lib.rtmi_mse_loss(_act(y, "y", torch.bfloat16), _act(target, "target", torch.float32, None),
                                 nvox, float(scale), _act(dz, "dz", torch.bfloat16),
                                 _act(loss, "loss", torch.float32, None), _stream(dev)))
    return loss


def adam_step(w, m, v, g, w_bf16, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    dev = w.device
    for t, name in ((m, "m"), (v, "v"), (g, "g")):
        _same(t, name, w.shape, dev)
    _optsame(w_bf16, "w_bf16", w.shape, dev)
    with torch.cuda.device(dev):
        _check(lib.rtmi_adam_step(_act(w, "w", torch.float32, None), _act(m, "m", torch.float32, None),
                                  _act(v, "v", torch.float32, None), _act(g, "g", torch.float32, None),
                                  _opt(w_bf16, "w_bf16", torch.bfloat16, None), w.numel(), float(lr),
                                  float(beta1), float(beta2), float(eps), int(step), _stream(dev)))


def surrogate_features(j, kappa, cheap, stats, x=None, scale_sums=None):
    """(x, scale_sums): bf16 [1][d][h][w][32] network input from fp32 j, kappa and the
    cheap field (3-D), and the device sums that fix the sample's scale."""
    d, h, w = j.shape
    dev = j.device
    _same(kappa, "kappa", j.shape, dev)
    _same(cheap, "cheap", j.shape, dev)
    xs = (1, d, h, w, CONV_CHANNELS)
    x = torch.empty(xs, dtype=torch.bfloat16, device=dev) if x is None else _same(x, "x", xs, dev)
    scale_sums = torch.empty(2, dtype=torch.float32, device=dev) if scale_sums is None else \
        _same(scale_sums, "scale_sums", (2,), dev)
    st = np.ascontiguousarray(np.asarray(stats, np.float32).reshape(6))
    with torch.cuda.device(dev):
        _check(lib.rtmi_surrogate_features(_dev(j, "j", 3), _dev(kappa, "kappa", 3), _dev(cheap, "cheap", 3),
                                           j.numel(), st.ctypes.data_as(ctypes.c_void_p),
                                           _act(scale_sums, "scale_sums", torch.float32, None),
                                           _act(x, "x", torch.bfloat16), _stream(dev)))
    return x, scale_sums


def surrogate_output(y, cheap, scale_sums, field=None, check=None):
    """(field, check sums): prediction from the network output and the error-check sums."""
    dev = cheap.device
    _same(y, "y", (1,) + tuple(cheap.shape) + (CONV_CHANNELS,), dev)
    _same(scale_sums, "scale_sums", (2,), dev)
    field = torch.empty_like(cheap) if field is None else _same(field, "field", cheap.shape, dev)
    check = torch.zeros(2, dtype=torch.float32, device=dev) if check is None else _same(check, "check", (2,), dev)
    with torch.cuda.device(dev):
        _check(lib.rtmi_surrogate_output(_act(y, "y", torch.bfloat16), _dev(cheap, "cheap", 3), cheap.numel(),
                                         _act(scale_sums, "scale_sums", torch.float32, None),
                                         _dev(field, "field", 3), _act(check, "check", torch.float32, None),
                                         _stream(dev)))
    return field, check


def timing_enable(on=True):
    """Bracket every march launch with HIP events on its stream (measurement only)."""
    _check(lib.rtmi_timing_enable(1 if on else 0))


def timing_read(kind):
    """(total milliseconds, launch count) of the launches of one kernel kind (KERNEL_RECORD,
    KERNEL_TILE or KERNEL_DIRECT) timed since the last read of that kind."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib.rtmi_timing_read(int(kind), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value

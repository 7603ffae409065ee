"""FP64 vector-Jacobian product of the march (test infrastructure only).

The paper differentiates its tracer end to end with JAX (Sec. 4, "Gradient-based
inversion"; "Coupling to differentiable hydro"). Here the derivative of the single-source
field J(j, kappa) is written out by the chain rule on Eq. (2), for an upstream gradient
G = dL/dJ. With a_k = exp(-kappa_k ds), E_k = exp(-tau_k), c = 4 pi / N and w_kv the
trilinear weights of sample k:

  direct sensitivity of I_{k+1}:   g_{k+1} = c * sum_v w_kv G[v]            (same weights)
  adjoint of I_{k+1}:             Ibar_{k+1} = g_{k+1} + Ibar_{k+2} a_{k+1}  (reverse in k)
  dL/dj[v]     += w_kv Ibar_{k+1} E_k ds                                    (j enters via j_k)
  dL/dkappa_k   = -ds (Ibar_{k+1} I_k a_k + sum_{k'>k} Ibar_{k'+1} j_{k'} E_{k'} ds)
                  (kappa_k attenuates step k and every later emission through tau)
  dL/dkappa[nearest voxel of sample k] += dL/dkappa_k

The forward quantities are those of oracle.march.trace_single (same readings, same
binary32 sample points). Pinned by tests against the exact Jacobian transpose (unit
impulses through the forward oracle) and against central finite differences in FP64.
"""

import numpy as np

from . import march


def trace_single_vjp(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                     time_step, grad_field, cap=0, geometry="fp32", directions=None,
                     weight=None):
    """Return (dL/dj, dL/dkappa) as FP64 arrays for dL/dJ = grad_field."""
    j = np.ascontiguousarray(j_map, dtype=np.float64)
    kap = np.ascontiguousarray(kappa_map, dtype=np.float64)
    G = np.ascontiguousarray(grad_field, dtype=np.float64).ravel()
    shape = np.array(j.shape, dtype=np.int64)
    jf, kf = j.ravel(), kap.ravel()
    n_s = march.num_substeps(step_size, radiation_velocity, time_step, cap)
    ds = float(np.float32(step_size))
    dirs = march.fibonacci_directions(num_rays) if directions is None else \
        np.asarray(directions, dtype=np.float64).reshape(-1, 3)
    n_rays = dirs.shape[0]
    c = march.FOUR_PI / n_rays if weight is None else float(weight)

    # forward sweep, keeping every per-step quantity (small problems only)
    flats, wts, nears, j_ks, a_ks, I_prev, E_k = [], [], [], [], [], [], []
    intensity = np.zeros(n_rays)
    tau = np.zeros(n_rays)
    corners = [(cx, cy, cz) for cx in (0, 1) for cy in (0, 1) for cz in (0, 1)]
    for k in range(n_s):
        x = march._positions(k, source_pos, dirs, ds, geometry)
        i0 = np.floor(x)
        frac = x - i0
        lo = np.clip(i0, 0, shape - 1).astype(np.int64)
        hi = np.clip(i0 + 1, 0, shape - 1).astype(np.int64)
        fl, ww = [], []
        for (cx, cy, cz) in corners:
            ia = hi[:, 0] if cx else lo[:, 0]
            ib = hi[:, 1] if cy else lo[:, 1]
            ic = hi[:, 2] if cz else lo[:, 2]
            fl.append((ia * shape[1] + ib) * shape[2] + ic)
            ww.append((frac[:, 0] if cx else 1.0 - frac[:, 0]) *
                      (frac[:, 1] if cy else 1.0 - frac[:, 1]) *
                      (frac[:, 2] if cz else 1.0 - frac[:, 2]))
        m = np.clip(np.rint(x), 0, shape - 1).astype(np.int64)
        near = (m[:, 0] * shape[1] + m[:, 1]) * shape[2] + m[:, 2]
        j_k = sum(w * jf[idx] for idx, w in zip(fl, ww))
        a_k = np.exp(-kf[near] * ds)
        E = np.exp(-tau)
        flats.append(fl)
        wts.append(ww)
        nears.append(near)
        j_ks.append(j_k)
        a_ks.append(a_k)
        I_prev.append(intensity.copy())
        E_k.append(E)
        intensity = intensity * a_k + j_k * E * ds
        tau = tau + kf[near] * ds

    # reverse sweep
    dj = np.zeros(jf.size)
    dk = np.zeros(kf.size)
    ibar_next = np.zeros(n_rays)      # Ibar_{k+2}
    a_next = np.zeros(n_rays)         # a_{k+1}
    suffix = np.zeros(n_rays)         # sum_{k'>k} Ibar_{k'+1} j_{k'} E_{k'} ds
    for k in range(n_s - 1, -1, -1):
        g = c * sum(w * G[idx] for idx, w in zip(flats[k], wts[k]))
        ibar = g + ibar_next * a_next
        for idx, w in zip(flats[k], wts[k]):
            np.add.at(dj, idx, w * ibar * E_k[k] * ds)
        np.add.at(dk, nears[k], -ds * (ibar * I_prev[k] * a_ks[k] + suffix))
        suffix = suffix + ibar * j_ks[k] * E_k[k] * ds
        ibar_next = ibar
        a_next = a_ks[k]
    return dj.reshape(j.shape), dk.reshape(kap.shape)


def trace_multi_vjp(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                    time_step, grad_field, caps=None, **kw):
    """VJP of the multi-source field: the sum of the single-source VJPs."""
    src = np.asarray(source_pos, dtype=np.float64).reshape(-1, 3)
    nr = np.broadcast_to(np.asarray(num_rays), (src.shape[0],))
    cp = np.zeros(src.shape[0], dtype=np.int64) if caps is None else \
        np.broadcast_to(np.asarray(caps), (src.shape[0],))
    dj = np.zeros(np.shape(j_map))
    dk = np.zeros(np.shape(kappa_map))
    for s in range(src.shape[0]):
        a, b = trace_single_vjp(j_map, kappa_map, src[s], int(nr[s]), step_size,
                                radiation_velocity, time_step, grad_field, cap=int(cp[s]), **kw)
        dj += a
        dk += b
    return dj, dk



def trace_bins_vjp(j_maps, kappa_map, kappa_scale, source_pos, num_rays, step_size,
                   radiation_velocity, time_step, grad_fields, caps=None, kappa_maps=None, **kw):
    """VJP of the frequency-bin march (oracle.march.trace_bins) for upstream gradients
    G_b = dL/dJ_b, grad_fields of shape (B, nx, ny, nz).

    Each bin is an independent multi-source problem (Sec. 2, "Frequency-bin agnosticism"),
    so its derivative is the single-bin one, and the shared inputs collect the bins'
    contributions by the chain rule:
      j shared by the bins:       dL/dj = sum_b dL/dj_b      (a 4-D j_maps: dL/dj_b each)
      kappa_b = s_b kappa:        dL/dkappa = sum_b s_b dL/dkappa_b,
                                  dL/ds_b   = sum_v kappa[v] dL/dkappa_b[v]
      per-bin kappa maps:         dL/dkappa_b each (no scales)
    where dL/dj_b, dL/dkappa_b are trace_multi_vjp at (j_b, kappa_b). Returns (dj, dk, ds),
    ds an array of B values, or None with per-bin kappa maps.
    """
    G = np.asarray(grad_fields, dtype=np.float64)
    n_bins = G.shape[0]
    jm = np.asarray(j_maps, dtype=np.float64)
    if kappa_maps is not None:
        km = np.asarray(kappa_maps, dtype=np.float64)
        kappas = [km[b] for b in range(n_bins)]
        scales = None
    else:
        base = np.asarray(kappa_map, dtype=np.float64)
        scales = [float(np.float32(v)) for v in np.asarray(kappa_scale, dtype=np.float64).ravel()]
        kappas = [base * scales[b] for b in range(n_bins)]
    dj = np.zeros(jm.shape)
    dk = np.zeros((n_bins,) + jm.shape[-3:]) if scales is None else np.zeros(jm.shape[-3:])
    ds = None if scales is None else np.zeros(n_bins)
    for b in range(n_bins):
        j_b = jm if jm.ndim == 3 else jm[b]
        a, k = trace_multi_vjp(j_b, kappas[b], source_pos, num_rays, step_size, radiation_velocity,
                               time_step, G[b], caps=caps, **kw)
        if jm.ndim == 3:
            dj += a
        else:
            dj[b] = a
        if scales is None:
            dk[b] = k
        else:
            dk += scales[b] * k
            ds[b] = float(np.sum(base * k))
    return dj, dk, ds

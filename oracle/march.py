"""Plain FP64 marcher (test infrastructure only; see the package docstring).

Each function follows the paper's Sec. 2 in its own order and notation. Nothing here is
blocked, fused or reordered beyond that description: the loop over substeps k is the
outer loop, and at each k every ray does position -> stencil -> gather -> update ->
deposit, exactly as the paragraph after Eq. (2) lists them. Rays are independent given
the medium (Sec. 2, "Vectorization, memory, and speed"), so one substep is evaluated for
all rays at once with NumPy arrays; that is the same arithmetic as a loop over rays.

Readings of points the paper leaves open (each is also listed in the design notes):
  * Grid convention: voxel (a, b, c) of a C-order [nx][ny][nz] array sits at grid
    coordinate (a, b, c); source positions are in these grid coordinates (Appendix A,
    "source_pos").
  * Fibonacci lattice: offset variant z_i = 1 - (2i+1)/N, azimuth i times the golden
    angle, polar axis = array axis 2 (Sec. 2 cites the golden-angle lattice without
    fixing the variant; this choice gives every point an equal-area z band of 4*pi/N,
    matching the 4*pi/N_Omega weight).
  * kappa "at the cell index used for the previous position": kappa is read at the
    nearest lattice point of x_k (round half to even), clamped to the box.
  * j is gathered and I_{k+1} deposited with the trilinear weights of x_k (Eq. (2) reads
    j(x_k); the deposit uses "the same trilinear weights").
  * Clamping: each stencil index is clamped per axis; rays are not stopped when they
    leave the box, they keep marching and deposit on the nearest boundary voxels.
  * Initial state: x_0 = source position, tau_0 = 0, I_0 = 0.
  * The 4*pi/N_Omega factor multiplies every deposit (with the source's own N_Omega).
  * Positions follow the "fp32 geometry" by default: t = fl32(k * ds), p = fl32(t * n),
    x = fl32(src + p), with n the FP64 direction rounded to binary32. These are the
    sample points a binary32 implementation produces; index decisions (floor, round)
    are discontinuous in x, so both sides must decide them on the same numbers. The
    "fp64" geometry (x = src + k ds n in binary64) is kept to measure that sensitivity.
"""

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def num_substeps(step_size, radiation_velocity, time_step, cap=0):
    """N_s = ceil(c * dt / ds) (Sec. 2 after Eq. (2); Appendix A, "N_s"), min'd with cap.

    The arguments are the binary32 values a caller passes; the quotient and the ceiling
    are taken in binary64. A cap <= 0 means "no cap".
    """
    ds = float(np.float32(step_size))
    c = float(np.float32(radiation_velocity))
    dt = float(np.float32(time_step))
    if not (ds > 0.0) or c < 0.0 or dt < 0.0:
        raise ValueError("need step_size > 0, radiation_velocity >= 0, time_step >= 0")
    n = int(math.ceil((c * dt) / ds))
    if cap > 0:
        n = min(n, int(cap))
    return n


def fibonacci_directions(n):
    """N nearly uniform unit vectors on the sphere, golden-angle lattice (Sec. 2).

    Point i has z_i = 1 - (2i + 1)/N, radius r_i = sqrt(1 - z_i^2) and azimuth
    phi_i = 2*pi * frac(i * g) with g = (3 - sqrt(5))/2 the golden-angle fraction of a
    turn. Returns an (N, 3) float64 array of (r cos phi, r sin phi, z) on array axes
    (0, 1, 2). Each step is evaluated per point with Python's libm-backed math module.
    """
    n = int(n)
    if n <= 0:
        raise ValueError("need at least one direction")
    g = (3.0 - math.sqrt(5.0)) / 2.0
    two_pi = 2.0 * math.pi
    out = np.empty((n, 3), dtype=np.float64)
    for i in range(n):
        z = 1.0 - (2.0 * i + 1.0) / n
        r = math.sqrt(max(0.0, 1.0 - z * z))
        ig = i * g
        phi = two_pi * (ig - math.floor(ig))
        out[i, 0] = r * math.cos(phi)
        out[i, 1] = r * math.sin(phi)
        out[i, 2] = z
    return out


def _positions(k, src, dirs, ds, geometry):
    """x_k = x_0 + k ds n (Eq. (2), first relation unrolled), as FP64 numbers."""
    if geometry == "fp32":
        t = np.float32(np.float32(k) * np.float32(ds))
        p = (t * dirs.astype(np.float32)).astype(np.float32)
        x = (np.asarray(src, dtype=np.float32)[None, :] + p).astype(np.float32)
        return x.astype(np.float64)
    if geometry == "fp64":
        return np.asarray(src, dtype=np.float64)[None, :] + (k * float(ds)) * dirs
    raise ValueError("geometry must be 'fp32' or 'fp64'")


def trace_single(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                 time_step, cap=0, geometry="fp32", kappa_rule="rint", directions=None,
                 weight=None, return_rays=False):
    """One source, one time step: the single-source kernel of Sec. 2.

    Arguments mirror the paper's signature (j_map, kappa_map, source_pos, num_rays,
    step_size, radiation_velocity, time_step). j_map and kappa_map are 3-D arrays
    (C order, [nx][ny][nz]); their values are read exactly as binary64. source_pos is a
    grid-coordinate triple. `directions` (N, 3) replaces the Fibonacci set and `weight`
    replaces 4*pi/N (test hooks). Returns J as an FP64 array of the grid's shape; with
    return_rays also the per-ray I_{k+1} and tau_{k+1} as (N, N_s) arrays.
    """
    j = np.ascontiguousarray(j_map, dtype=np.float64)
    kap = np.ascontiguousarray(kappa_map, dtype=np.float64)
    if j.ndim != 3 or j.shape != kap.shape:
        raise ValueError("j_map and kappa_map must be 3-D arrays of the same shape")
    shape = np.array(j.shape, dtype=np.int64)
    jf = j.ravel()
    kf = kap.ravel()

    n_s = num_substeps(step_size, radiation_velocity, time_step, cap)
    ds = float(np.float32(step_size))
    if directions is None:
        dirs = fibonacci_directions(num_rays)
    else:
        dirs = np.asarray(directions, dtype=np.float64).reshape(-1, 3)
    n_rays = dirs.shape[0]
    w_ray = FOUR_PI / n_rays if weight is None else float(weight)

    field = np.zeros(jf.size, dtype=np.float64)
    intensity = np.zeros(n_rays)          # I_k, with I_0 = 0
    tau = np.zeros(n_rays)                # tau_k, with tau_0 = 0
    if return_rays:
        rays_i = np.zeros((n_rays, n_s))
        rays_tau = np.zeros((n_rays, n_s))

    corners = [(cx, cy, cz) for cx in (0, 1) for cy in (0, 1) for cz in (0, 1)]
    for k in range(n_s):
        # position x_k
        x = _positions(k, source_pos, dirs, ds, geometry)

        # trilinear stencil, each index clamped to the box
        i0 = np.floor(x)
        frac = x - i0
        lo = np.clip(i0, 0, shape - 1).astype(np.int64)
        hi = np.clip(i0 + 1, 0, shape - 1).astype(np.int64)
        flat = []
        wts = []
        for (cx, cy, cz) in corners:
            ia = hi[:, 0] if cx else lo[:, 0]
            ib = hi[:, 1] if cy else lo[:, 1]
            ic = hi[:, 2] if cz else lo[:, 2]
            wa = frac[:, 0] if cx else 1.0 - frac[:, 0]
            wb = frac[:, 1] if cy else 1.0 - frac[:, 1]
            wc = frac[:, 2] if cz else 1.0 - frac[:, 2]
            flat.append((ia * shape[1] + ib) * shape[2] + ic)
            wts.append(wa * wb * wc)

        # j(x_k) by trilinear interpolation
        j_k = np.zeros(n_rays)
        for idx, w in zip(flat, wts):
            j_k += w * jf[idx]

        # kappa(x_k), nearest neighbour, clamped
        if kappa_rule == "rint":
            near = np.rint(x)
        elif kappa_rule == "floor":
            near = np.floor(x)
        else:
            raise ValueError("kappa_rule must be 'rint' or 'floor'")
        m = np.clip(near, 0, shape - 1).astype(np.int64)
        kappa_k = kf[(m[:, 0] * shape[1] + m[:, 1]) * shape[2] + m[:, 2]]

        # Eq. (2): I_{k+1} = I_k exp(-kappa ds) + j exp(-tau_k) ds ; tau_{k+1} = tau_k + kappa ds
        intensity = intensity * np.exp(-kappa_k * ds) + j_k * np.exp(-tau) * ds
        tau = tau + kappa_k * ds
        if return_rays:
            rays_i[:, k] = intensity
            rays_tau[:, k] = tau

        # deposit the post-attenuation I_{k+1} with the same weights, times 4 pi / N
        for idx, w in zip(flat, wts):
            np.add.at(field, idx, w_ray * w * intensity)

    field = field.reshape(j.shape)
    if return_rays:
        return field, rays_i, rays_tau
    return field


def trace_multi(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                time_step, caps=None, **kw):
    """Multi-source routine: the sum of single-source fields (Sec. 2, loop-and-sum).

    source_pos is (n_src, 3); num_rays and caps are per-source sequences (caps may be
    None). Every source sees the same j_map.
    """
    src = np.asarray(source_pos, dtype=np.float64).reshape(-1, 3)
    n_src = src.shape[0]
    nr = np.broadcast_to(np.asarray(num_rays), (n_src,))
    cp = np.zeros(n_src, dtype=np.int64) if caps is None else np.broadcast_to(np.asarray(caps), (n_src,))
    total = np.zeros(np.shape(j_map), dtype=np.float64)
    for s in range(n_src):
        total += trace_single(j_map, kappa_map, src[s], int(nr[s]), step_size,
                              radiation_velocity, time_step, cap=int(cp[s]), **kw)
    return total


def trace_bins(j_maps, kappa_map, kappa_scale, source_pos, num_rays, step_size,
               radiation_velocity, time_step, caps=None, kappa_maps=None, **kw):
    """Frequency bins as a batch axis (Sec. 2, "Frequency-bin agnosticism").

    Bin b is an independent multi-source problem with emissivity j_b and opacity
    kappa_b. j_maps is either one 3-D map (shared by all bins) or a (B, nx, ny, nz)
    stack. kappa_b = kappa * kappa_scale[b], or kappa_maps[b] when kappa_maps is given.
    Returns a (B, nx, ny, nz) FP64 array.
    """
    jm = np.asarray(j_maps)
    if kappa_maps is not None:
        km = np.asarray(kappa_maps, dtype=np.float64)
        n_bins = km.shape[0]
        kappas = [km[b] for b in range(n_bins)]
    else:
        scale = np.asarray(kappa_scale, dtype=np.float64).ravel()
        n_bins = scale.size
        base = np.asarray(kappa_map, dtype=np.float64)
        kappas = [base * float(np.float32(scale[b])) for b in range(n_bins)]
    out = []
    for b in range(n_bins):
        j_b = jm if jm.ndim == 3 else jm[b]
        out.append(trace_multi(j_b, kappas[b], source_pos, num_rays, step_size,
                               radiation_velocity, time_step, caps=caps, **kw))
    return np.stack(out)


def trace_voxels(j_map, kappa_map, source_pos, num_rays, step_size, radiation_velocity,
                 time_step, voxels, caps=None, kappa_scale=1.0):
    """J at a few interior voxels of the multi-source field (Sec. 2, loop-and-sum), in FP64.

    The same march as trace_single (fp32 geometry, rint kappa, Eq. (2), deposit of I_{k+1}
    with x_k's weights, 4 pi / N per deposit), restricted to what can reach the requested
    voxels: an interior voxel v (1 <= v_a <= n_a - 2 on every axis) is a stencil corner of
    sample x exactly when v_a - 1 <= x_a < v_a + 1 on every axis, so only rays whose
    segment passes through that cube (widened by 1e-3 for the binary32 rounding of x) can
    deposit on it, and only up to the last substep that can reach it. Those rays are
    marched from k = 0 like every other ray; deposits on other voxels are dropped. This
    lets a field whose full oracle would take hours be checked voxel by voxel.

    voxels: (m, 3) integer array. kappa_scale multiplies kappa as trace_bins's bin scale
    does. Returns an (m,) FP64 array.
    """
    j = np.ascontiguousarray(j_map, dtype=np.float64)
    kap = np.asarray(kappa_map, dtype=np.float64) * float(np.float32(kappa_scale))
    shape = np.array(j.shape, dtype=np.int64)
    jf, kf = j.ravel(), kap.ravel()
    vox = np.asarray(voxels, dtype=np.int64).reshape(-1, 3)
    if np.any(vox < 1) or np.any(vox > shape - 2):
        raise ValueError("trace_voxels takes interior voxels only (1 <= v <= n - 2 per axis)")
    vflat = (vox[:, 0] * shape[1] + vox[:, 1]) * shape[2] + vox[:, 2]
    order = np.argsort(vflat, kind="stable")
    vsorted = vflat[order]
    if np.any(np.diff(vsorted) == 0):
        raise ValueError("voxels must be distinct")
    out_sorted = np.zeros(vflat.size)

    src_all = np.asarray(source_pos, dtype=np.float64).reshape(-1, 3)
    n_src = src_all.shape[0]
    nr = np.broadcast_to(np.asarray(num_rays), (n_src,))
    cp = np.zeros(n_src, dtype=np.int64) if caps is None else np.broadcast_to(np.asarray(caps), (n_src,))
    ds = float(np.float32(step_size))
    corners = [(cx, cy, cz) for cx in (0, 1) for cy in (0, 1) for cz in (0, 1)]
    margin = 1e-3
    for s in range(n_src):
        n_s = num_substeps(step_size, radiation_velocity, time_step, int(cp[s]))
        if n_s == 0:
            continue
        src = src_all[s].astype(np.float32).astype(np.float64)
        dirs = fibonacci_directions(int(nr[s]))
        n32 = dirs.astype(np.float32).astype(np.float64)
        tmax = (n_s - 1) * ds
        # per (ray, voxel): the parameter interval inside v's cube, intersected with [0, tmax]
        t0 = np.zeros((n32.shape[0], vox.shape[0]))
        t1 = np.full((n32.shape[0], vox.shape[0]), tmax)
        for a in range(3):
            lo = vox[None, :, a] - 1.0 - margin - src[a]
            hi = vox[None, :, a] + 1.0 + margin - src[a]
            na = n32[:, a][:, None]
            with np.errstate(divide="ignore", invalid="ignore"):
                ta, tb = lo / na, hi / na
            ta = np.where(na == 0.0, np.where((lo <= 0) & (hi >= 0), -np.inf, np.inf), ta)
            tb = np.where(na == 0.0, np.where((lo <= 0) & (hi >= 0), np.inf, -np.inf), tb)
            t0 = np.maximum(t0, np.minimum(ta, tb))
            t1 = np.minimum(t1, np.maximum(ta, tb))
        reach = t0 <= t1
        rays = np.flatnonzero(reach.any(axis=1))
        if rays.size == 0:
            continue
        k_last = np.minimum(n_s - 1, np.ceil(np.where(reach[rays], t1[rays], -np.inf).max(axis=1) / ds) + 1)
        steps = int(k_last.max()) + 1
        d = dirs[rays]
        w_ray = FOUR_PI / dirs.shape[0]
        intensity = np.zeros(rays.size)
        tau = np.zeros(rays.size)
        for k in range(steps):
            x = _positions(k, src_all[s], d, ds, "fp32")
            i0 = np.floor(x)
            frac = x - i0
            lo = np.clip(i0, 0, shape - 1).astype(np.int64)
            hi = np.clip(i0 + 1, 0, shape - 1).astype(np.int64)
            flat, wts = [], []
            for (cx, cy, cz) in corners:
                ia = hi[:, 0] if cx else lo[:, 0]
                ib = hi[:, 1] if cy else lo[:, 1]
                ic = hi[:, 2] if cz else lo[:, 2]
                flat.append((ia * shape[1] + ib) * shape[2] + ic)
                wts.append((frac[:, 0] if cx else 1.0 - frac[:, 0]) *
                           (frac[:, 1] if cy else 1.0 - frac[:, 1]) *
                           (frac[:, 2] if cz else 1.0 - frac[:, 2]))
            j_k = np.zeros(rays.size)
            for idx, w in zip(flat, wts):
                j_k += w * jf[idx]
            m = np.clip(np.rint(x), 0, shape - 1).astype(np.int64)
            kappa_k = kf[(m[:, 0] * shape[1] + m[:, 1]) * shape[2] + m[:, 2]]
            intensity = intensity * np.exp(-kappa_k * ds) + j_k * np.exp(-tau) * ds
            tau = tau + kappa_k * ds
            for idx, w in zip(flat, wts):
                pos = np.minimum(np.searchsorted(vsorted, idx), vsorted.size - 1)
                hit = vsorted[pos] == idx
                if hit.any():
                    np.add.at(out_sorted, pos[hit], (w_ray * w * intensity)[hit])
    out = np.empty_like(out_sorted)
    out[order] = out_sorted
    return out

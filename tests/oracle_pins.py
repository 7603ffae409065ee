"""Pins for the FP64 oracle: checks that do not re-type the oracle's own code.

Each pin takes a module `m` exposing num_substeps, fibonacci_directions and trace_single
(the oracle, or a deliberately broken copy of it in the mutation test) and raises on
failure. They check the oracle against what the paper and the mathematics fix:
closed forms of Eq. (2), invariants of the deposit, symmetry, and a brute-force
gather-form evaluator written independently as scalar Python loops.
"""

import math
from fractions import Fraction

import numpy as np

FOUR_PI = 4.0 * math.pi
GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


# ----------------------------------------------------------------------------------------
# Independent scalar walker (pure Python): positions, stencil and samples of one ray.
# ----------------------------------------------------------------------------------------
def f32_position(src, n, k, ds):
    """The binary32 sample point of substep k: fl(src + fl(fl(k ds) n))."""
    t = np.float32(np.float32(k) * np.float32(ds))
    return [float(np.float32(np.float32(src[a]) + np.float32(t * np.float32(n[a])))) for a in range(3)]


def stencil(x, shape):
    """[(flat index, weight)] of the clamped trilinear stencil at x (8 entries)."""
    out = []
    base = [math.floor(v) for v in x]
    frac = [x[a] - base[a] for a in range(3)]
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                idx = []
                w = 1.0
                for a, c in enumerate((cx, cy, cz)):
                    i = min(max(base[a] + c, 0), shape[a] - 1)
                    idx.append(i)
                    w *= frac[a] if c else (1.0 - frac[a])
                out.append(((idx[0] * shape[1] + idx[1]) * shape[2] + idx[2], w))
    return out


def nearest(x, shape):
    idx = [min(max(int(round(v)), 0), shape[a] - 1) for a, v in enumerate(x)]  # round() is half-even
    return (idx[0] * shape[1] + idx[1]) * shape[2] + idx[2]


def walk(jf, kf, shape, src, n, ds, n_s):
    """Return per-step (stencil, j_k, kappa_k) of one ray (x_0 = src)."""
    steps = []
    for k in range(n_s):
        x = f32_position(src, n, k, ds)
        st = stencil(x, shape)
        j_k = sum(w * jf[i] for i, w in st)
        steps.append((st, j_k, kf[nearest(x, shape)]))
    return steps


def closed_form_intensity(steps, ds):
    """I_{k+1} = exp(-tau_{k+1}) * sum_{m<=k} j_m exp(kappa_m ds) ds, tau_{k+1} = ds sum kappa_m."""
    out = []
    tau = 0.0
    acc = 0.0
    for (_, j_k, kap) in steps:
        tau += kap * ds
        acc += j_k * math.exp(kap * ds) * ds
        out.append(math.exp(-tau) * acc)
    return out


def rand_medium(shape, seed, kappa_scale=0.3):
    rng = np.random.default_rng(seed)
    j = rng.random(shape).astype(np.float32)
    kap = (kappa_scale * rng.random(shape)).astype(np.float32)
    return j, kap


# ----------------------------------------------------------------------------------------
# Pins
# ----------------------------------------------------------------------------------------
def pin_num_substeps(m):
    assert m.num_substeps(0.5, 16.0, 1.0) == 32
    assert m.num_substeps(0.5, 128.0, 1.0) == 256
    # ceil of the exact quotient of the binary32 inputs (10 * fl32(0.3) / 0.5 = 6.0000002)
    for ds, c, dt in [(0.5, 10.0, 0.3), (0.25, 1.0, 1.1), (0.3, 7.0, 0.9), (0.5, 3.0, 0.5)]:
        q = Fraction(float(np.float32(c))) * Fraction(float(np.float32(dt))) / Fraction(float(np.float32(ds)))
        assert m.num_substeps(ds, c, dt) == math.ceil(q), (ds, c, dt)
    assert m.num_substeps(0.5, 10.0, 0.3) == 7
    assert m.num_substeps(0.5, 256.0, 1.0, cap=100) == 100
    assert m.num_substeps(0.5, 16.0, 1.0, cap=1000) == 32
    assert m.num_substeps(0.5, 16.0, 0.0) == 0


def pin_fibonacci(m):
    for n in (1, 2, 7, 64, 256, 1000):
        d = m.fibonacci_directions(n)
        assert d.shape == (n, 3)
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
        # equal-area bands: z_i are the midpoints of N equal slices of [-1, 1]
        z_expected = np.array([1.0 - (2 * i + 1) / n for i in range(n)])
        assert np.allclose(d[:, 2], z_expected, atol=1e-15)
        assert abs(d[:, 2].sum()) < 1e-12
        if n >= 2:
            # successive azimuths advance by the golden angle, counter-clockwise about +z
            phi = np.arctan2(d[:, 1], d[:, 0])
            step = np.mod(np.diff(phi), 2 * math.pi)
            assert np.allclose(step, GOLDEN_ANGLE, atol=1e-9)
            assert abs(phi[0]) < 1e-15   # phase: the first point sits at azimuth 0
    d = m.fibonacci_directions(256)
    assert abs(np.mean(d[:, 0] ** 2) - 1.0 / 3.0) < 1e-4
    assert np.linalg.norm(d.sum(axis=0)) / 256 < 1e-2


def pin_uniform_total(m):
    """Uniform j, kappa: every ray has I_{k+1} = (k+1) j0 ds e^{-k kappa0 ds}, so
    sum J = 4 pi j0 ds sum_k (k+1) e^{-k kappa0 ds}, whatever the directions and clamping."""
    for shape, src, kap0, c, n_rays in [((8, 9, 10), (4.0, 4.5, 5.0), 0.1, 8.0, 37),
                                        ((6, 6, 6), (0.3, 5.2, 2.9), 0.0, 10.0, 20),
                                        ((5, 7, 4), (2.0, 3.0, 1.0), 0.7, 5.0, 64)]:
        j0 = 0.75
        j = np.full(shape, j0, np.float32)
        kap = np.full(shape, kap0, np.float32)
        ds = 0.5
        n_s = int(math.ceil(c / ds))
        got = m.trace_single(j, kap, src, n_rays, ds, c, 1.0).sum()
        a = math.exp(-float(np.float32(kap0)) * ds)
        want = FOUR_PI * float(np.float32(j0)) * ds * sum((k + 1) * a ** k for k in range(n_s))
        assert abs(got - want) <= 1e-12 * abs(want), (got, want)


def pin_recurrence(m):
    """Per-ray traces follow the closed form of Eq. (2) built from an independent walk."""
    shape = (9, 8, 7)
    j, kap = rand_medium(shape, 11)
    src = (4.3, 3.9, 3.1)
    n_rays, ds, c = 24, 0.5, 6.0
    n_s = int(math.ceil(c / ds))
    _, rays_i, rays_tau = m.trace_single(j, kap, src, n_rays, ds, c, 1.0, return_rays=True)
    dirs = m.fibonacci_directions(n_rays)
    jf, kf = j.ravel().astype(float), kap.ravel().astype(float)
    for r in (0, 5, 13, 23):
        steps = walk(jf, kf, shape, src, dirs[r], ds, n_s)
        want = closed_form_intensity(steps, ds)
        assert np.allclose(rays_i[r], want, rtol=1e-12, atol=0), r
        assert np.allclose(rays_tau[r], np.cumsum([s[2] * ds for s in steps]), rtol=1e-12), r


def pin_conservation(m):
    """sum J = (4 pi / N) sum_rays sum_k I_{k+1}: the clamped weights partition unity."""
    shape = (10, 6, 8)
    j, kap = rand_medium(shape, 5)
    for src in [(5.0, 3.0, 4.0), (0.2, 5.9, 7.7), (-1.5, 2.0, 9.5)]:
        field, rays_i, _ = m.trace_single(j, kap, src, 33, 0.5, 12.0, 1.0, return_rays=True)
        want = FOUR_PI / 33 * rays_i.sum()
        assert abs(field.sum() - want) <= 1e-12 * want


def pin_axis_ray(m):
    """One ray along +x (N = 1, weight 4 pi) from an integer source, j = j0 at the source only,
    uniform kappa, ds = 0.5: I_1 = j0 ds, I_{k+1} = 1.5 j0 ds e^{-k kappa ds} for k >= 1,
    J[s] = 4 pi (I_1 + I_2 / 2), J[s+m] = 4 pi 1.5 j0 ds e^{-kappa m}(1 + cosh(kappa ds))
    before the wall, and the rest of the march piles up on the boundary voxel."""
    n = 12
    shape = (n, 5, 6)
    s = (3, 2, 4)
    kap0 = float(np.float32(0.2))
    j0 = 2.0
    ds = 0.5
    j = np.zeros(shape, np.float32)
    j[s] = j0
    kap = np.full(shape, kap0, np.float32)
    n_s = 30
    field = m.trace_single(j, kap, s, 1, ds, float(n_s) * ds, 1.0, directions=[[1.0, 0.0, 0.0]],
                           weight=FOUR_PI)
    a = math.exp(-kap0 * ds)
    i_k = [j0 * ds] + [1.5 * j0 * ds * a ** k for k in range(1, n_s)]
    line = field[:, s[1], s[2]]
    assert abs(line[s[0]] - FOUR_PI * (i_k[0] + 0.5 * i_k[1])) < 1e-12 * line[s[0]]
    for mm in range(1, n - 1 - s[0]):
        want = FOUR_PI * 1.5 * j0 * ds * math.exp(-kap0 * mm) * (1.0 + math.cosh(kap0 * ds))
        assert abs(line[s[0] + mm] - want) < 1e-12 * want, mm
    # the boundary voxel collects its own neighbourhood plus every deposit past the wall
    k_wall = 2 * (n - 1 - s[0]) - 1
    want_wall = FOUR_PI * (0.5 * i_k[k_wall] + sum(i_k[k_wall + 1:]))
    assert abs(line[n - 1] - want_wall) < 1e-12 * want_wall
    assert np.count_nonzero(field) == n - s[0]


def pin_free_streaming(m):
    """kappa = 0 and j on one voxel: each ray's I is constant once past the stencil of the
    source voxel (after 4 substeps of 0.5), and equals ds times the sum of its first samples."""
    shape = (15, 15, 15)
    j = np.zeros(shape, np.float32)
    j[7, 7, 7] = 1.0
    kap = np.zeros(shape, np.float32)
    _, rays_i, _ = m.trace_single(j, kap, (7.0, 7.0, 7.0), 50, 0.5, 6.0, 1.0, return_rays=True)
    assert np.all(rays_i[:, 3:] == rays_i[:, 3:4])
    assert np.allclose(rays_i[:, 0], 0.5)                 # I_1 = j(src) ds
    assert np.all(rays_i[:, 3] > 0.5)


def pin_linearity(m):
    """J is linear in j; multi-source fields add up (Sec. 2, loop-and-sum)."""
    shape = (7, 9, 8)
    j1, kap = rand_medium(shape, 21)
    j2, _ = rand_medium(shape, 22)
    args = ((3.2, 4.4, 3.9), 40, 0.5, 7.0, 1.0)
    f1 = m.trace_single(j1, kap, *args)
    f2 = m.trace_single(j2, kap, *args)
    f12 = m.trace_single((2.0 * j1.astype(np.float64) - 0.5 * j2), kap, *args)
    assert np.allclose(f12, 2.0 * f1 - 0.5 * f2, rtol=1e-11, atol=1e-13 * np.abs(f1).max())


def pin_axis_permutation(m):
    """Permuting the axes of (j, kappa, source, directions) permutes J."""
    shape = (6, 8, 10)
    j, kap = rand_medium(shape, 31)
    dirs = np.random.default_rng(3).normal(size=(17, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    src = np.array([2.7, 4.1, 5.6])
    base = m.trace_single(j, kap, src, 17, 0.5, 8.0, 1.0, directions=dirs)
    for perm in [(1, 2, 0), (2, 0, 1), (0, 2, 1)]:
        got = m.trace_single(np.transpose(j, perm), np.transpose(kap, perm), src[list(perm)], 17,
                             0.5, 8.0, 1.0, directions=dirs[:, list(perm)])
        assert np.allclose(got, np.transpose(base, perm), rtol=1e-12, atol=1e-14 * base.max())


def pin_reflection(m):
    """Mirroring one axis (x -> n-1-x, n_x -> -n_x) mirrors J; exact in the fp64 geometry on
    odd grids, where round-half-to-even is itself mirror symmetric."""
    shape = (9, 7, 11)
    j, kap = rand_medium(shape, 41)
    dirs = np.random.default_rng(4).normal(size=(13, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    src = np.array([3.0, 2.5, 6.0])
    base = m.trace_single(j, kap, src, 13, 0.5, 9.0, 1.0, directions=dirs, geometry="fp64")
    for ax in range(3):
        d2 = dirs.copy()
        d2[:, ax] = -d2[:, ax]
        s2 = src.copy()
        s2[ax] = shape[ax] - 1 - s2[ax]
        got = m.trace_single(np.flip(j, ax), np.flip(kap, ax), s2, 13, 0.5, 9.0, 1.0,
                             directions=d2, geometry="fp64")
        assert np.allclose(got, np.flip(base, ax), rtol=1e-10, atol=1e-13 * base.max()), ax


def pin_brute_force(m):
    """Gather-form brute force on a small non-cubic grid: J[v] = sum over rays and substeps of
    W(x_k, v) (4 pi / N) I_{k+1}, with I from the closed form of an independent walk."""
    shape = (7, 8, 9)
    j, kap = rand_medium(shape, 51)
    src = (3.4, 2.2, 5.1)
    n_rays, ds, c = 12, 0.5, 5.5
    n_s = int(math.ceil(c / ds))
    dirs = m.fibonacci_directions(n_rays)
    got = m.trace_single(j, kap, src, n_rays, ds, c, 1.0).ravel()
    jf, kf = j.ravel().astype(float), kap.ravel().astype(float)
    samples = []
    for r in range(n_rays):
        steps = walk(jf, kf, shape, src, dirs[r], ds, n_s)
        for (st, _, _), i_next in zip(steps, closed_form_intensity(steps, ds)):
            samples.append((dict_of(st), i_next))
    want = np.zeros(jf.size)
    for v in range(jf.size):
        acc = 0.0
        for weights, i_next in samples:
            w = weights.get(v)
            if w is not None:
                acc += w * FOUR_PI / n_rays * i_next
        want[v] = acc
    assert np.allclose(got, want, rtol=1e-12, atol=1e-14 * want.max())


def dict_of(st):
    d = {}
    for i, w in st:
        d[i] = d.get(i, 0.0) + w
    return d


ALL_PINS = [pin_num_substeps, pin_fibonacci, pin_uniform_total, pin_recurrence, pin_conservation,
            pin_axis_ray, pin_free_streaming, pin_linearity, pin_axis_permutation, pin_reflection,
            pin_brute_force]

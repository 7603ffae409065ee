"""CPU pins of the FP64 adjoint (vector-Jacobian product) of the march."""

import types

import numpy as np
import pytest

import oracle
from oracle import adjoint as oracle_adjoint

from oracle_pins import rand_medium


def _jacobian_wrt_j(kap, shape, src, n_rays, ds, c):
    """J = A j: column v of A is the field of a unit impulse at voxel v (the field is linear in j)."""
    cols = []
    for v in range(int(np.prod(shape))):
        e = np.zeros(int(np.prod(shape)))
        e[v] = 1.0
        cols.append(oracle.trace_single(e.reshape(shape), kap, src, n_rays, ds, c, 1.0).ravel())
    return np.stack(cols, axis=1)


def pin_jacobian_transpose(m):
    shape = (5, 6, 4)
    j, kap = rand_medium(shape, 61)
    src = (2.3, 2.9, 1.6)
    G = np.random.default_rng(5).normal(size=shape)
    A = _jacobian_wrt_j(kap, shape, src, 9, 0.5, 4.5)
    dj, _ = m.trace_single_vjp(j, kap, src, 9, 0.5, 4.5, 1.0, G)
    want = A.T @ G.ravel()
    assert np.allclose(dj.ravel(), want, rtol=1e-11, atol=1e-13 * np.abs(want).max())


def pin_kappa_finite_differences(m):
    shape = (6, 5, 7)
    j, kap = rand_medium(shape, 62, kappa_scale=0.4)
    kap = kap.astype(np.float64)
    src = (2.7, 2.2, 3.4)
    G = np.random.default_rng(6).normal(size=shape)
    _, dk = m.trace_single_vjp(j, kap, src, 11, 0.5, 5.0, 1.0, G)
    loss = lambda kk: float(np.sum(G * oracle.trace_single(j, kk, src, 11, 0.5, 5.0, 1.0)))
    h = 1e-5
    checked = 0
    for v in np.argsort(-np.abs(dk.ravel()))[:12]:
        e = np.zeros(kap.size)
        e[v] = h
        fd = (loss(kap + e.reshape(shape)) - loss(kap - e.reshape(shape))) / (2 * h)
        assert abs(fd - dk.ravel()[v]) <= 1e-6 * max(1.0, abs(fd)), (v, fd, dk.ravel()[v])
        checked += 1
    assert checked == 12
    # voxels no ray samples have zero gradient
    assert np.count_nonzero(dk) < kap.size


def pin_amplitude_inversion(m):
    """Sec. 4: j = A e0 with a fixed template. J(A e0) = A F, so the MSE minimiser is
    <F, I_ref>/<F, F>, and dL/dA = <dL/dj, e0> = <G, F>."""
    shape = (7, 7, 7)
    e0 = np.zeros(shape)
    e0[3, 3, 3] = 1.0
    e0[3, 4, 3] = 0.5
    kap = np.full(shape, 0.1)
    F = oracle.trace_single(e0, kap, (3.0, 3.0, 3.0), 20, 0.5, 4.0, 1.0)
    a_true, a = 2.5, 1.2
    ref = a_true * F
    G = 2.0 * (a * F - ref)
    dj, _ = m.trace_single_vjp(a * e0, kap, (3.0, 3.0, 3.0), 20, 0.5, 4.0, 1.0, G)
    assert np.isclose(np.sum(dj * e0), np.sum(G * F), rtol=1e-12)
    assert np.isclose(np.sum(F * ref) / np.sum(F * F), a_true, rtol=1e-14)


ADJ_PINS = [pin_jacobian_transpose, pin_kappa_finite_differences, pin_amplitude_inversion]


@pytest.mark.parametrize("pin", ADJ_PINS, ids=lambda p: p.__name__)
def test_adjoint_pin(pin):
    pin(oracle)


def test_multi_vjp_is_sum():
    shape = (6, 6, 6)
    j, kap = rand_medium(shape, 63)
    G = np.random.default_rng(7).normal(size=shape)
    src = np.array([[2.0, 3.0, 1.5], [4.5, 1.0, 4.0]])
    dj, dk = oracle.trace_multi_vjp(j, kap, src, [7, 12], 0.5, 4.0, 1.0, G, caps=[0, 5])
    a = oracle.trace_single_vjp(j, kap, src[0], 7, 0.5, 4.0, 1.0, G)
    b = oracle.trace_single_vjp(j, kap, src[1], 12, 0.5, 4.0, 1.0, G, cap=5)
    assert np.allclose(dj, a[0] + b[0]) and np.allclose(dk, a[1] + b[1])


ADJ_MUTANTS = {
    "no kappa suffix (tau) term": ("-ds * (ibar * I_prev[k] * a_ks[k] + suffix)", "-ds * (ibar * I_prev[k] * a_ks[k])"),
    "adjoint propagates without attenuation": ("ibar = g + ibar_next * a_next", "ibar = g + ibar_next"),
    "dj without exp(-tau_k)": ("np.add.at(dj, idx, w * ibar * E_k[k] * ds)", "np.add.at(dj, idx, w * ibar * ds)"),
    "dkappa uses I_{k+1}": ("ibar * I_prev[k] * a_ks[k]", "ibar * (I_prev[k] * a_ks[k] + j_ks[k] * E_k[k] * ds)"),
    "G gathered without 4pi/N": ("g = c * sum(", "g = sum("),
}


@pytest.mark.parametrize("name", sorted(ADJ_MUTANTS))
def test_adjoint_pins_catch_mutant(name):
    src = open(oracle_adjoint.__file__).read()
    old, new = ADJ_MUTANTS[name]
    assert old in src
    mod = types.ModuleType("adjoint_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new, 1), "adjoint_mutant", "exec"), mod.__dict__)
    failed = []
    for pin in ADJ_PINS:
        try:
            pin(mod)
        except Exception:  # noqa: BLE001
            failed.append(pin.__name__)
    assert failed, f"no pin catches: {name}"


# ---- frequency bins (Sec. 2: bins are independent copies of the problem) ----

BIN_SCALES = np.array([1.0, 0.296875, 0.125], np.float32)   # exact in binary32


def _bins_case(seed):
    shape = (5, 4, 6)
    j, kap = rand_medium(shape, seed, kappa_scale=0.5)
    src = np.array([[2.2, 1.7, 2.9], [1.1, 2.6, 3.8]])
    G = np.random.default_rng(seed + 1).normal(size=(3,) + shape)
    return shape, j.astype(np.float64), kap.astype(np.float64), src, G


def _bins_loss(j, kap_maps, src, G):
    """sum_b <G_b, J_b> with bin b's opacity given as a full FP64 map."""
    J = oracle.trace_bins(j, None, None, src, [9, 6], 0.5, 3.0, 1.0, caps=[0, 5], kappa_maps=kap_maps)
    return float(np.sum(G * J))


def pin_bins_scale_finite_differences(m):
    """dL/ds_b against central differences in the bin scale (opacity maps kappa (s_b +- h))."""
    shape, j, kap, src, G = _bins_case(71)
    _, _, ds = m.trace_bins_vjp(j, kap, BIN_SCALES, src, [9, 6], 0.5, 3.0, 1.0, G, caps=[0, 5])
    h = 1e-6
    for b in range(3):
        maps = [kap * float(s) for s in BIN_SCALES]
        up = [mm.copy() for mm in maps]
        dn = [mm.copy() for mm in maps]
        up[b] = kap * (float(BIN_SCALES[b]) + h)
        dn[b] = kap * (float(BIN_SCALES[b]) - h)
        fd = (_bins_loss(j, np.stack(up), src, G) - _bins_loss(j, np.stack(dn), src, G)) / (2 * h)
        assert abs(fd - ds[b]) <= 1e-6 * max(1.0, abs(fd)), (b, fd, ds[b])


def pin_bins_kappa_finite_differences(m):
    """dL/dkappa of the shared base opacity (every bin scales it) against central differences."""
    shape, j, kap, src, G = _bins_case(72)
    _, dk, _ = m.trace_bins_vjp(j, kap, BIN_SCALES, src, [9, 6], 0.5, 3.0, 1.0, G, caps=[0, 5])
    h = 1e-6
    for v in np.argsort(-np.abs(dk.ravel()))[:8]:
        e = np.zeros(kap.size)
        e[v] = h
        e = e.reshape(shape)
        fd = (_bins_loss(j, np.stack([(kap + e) * float(s) for s in BIN_SCALES]), src, G) -
              _bins_loss(j, np.stack([(kap - e) * float(s) for s in BIN_SCALES]), src, G)) / (2 * h)
        assert abs(fd - dk.ravel()[v]) <= 1e-6 * max(1.0, abs(fd)), (v, fd, dk.ravel()[v])


def pin_bins_j_jacobian_transpose(m):
    """L is linear in j: dL/dj[v] = sum_b <G_b, J_b(e_v)> by unit impulses, for a j shared by
    the bins and, per bin, for a stack of j maps."""
    shape, j, kap, src, G = _bins_case(73)
    maps = np.stack([kap * float(s) for s in BIN_SCALES])
    dj, _, _ = m.trace_bins_vjp(j, kap, BIN_SCALES, src, [9, 6], 0.5, 3.0, 1.0, G, caps=[0, 5])
    stack = np.stack([j, 0.5 * j, 2.0 * j])
    djb, dkb, dsb = m.trace_bins_vjp(stack, None, None, src, [9, 6], 0.5, 3.0, 1.0, G, caps=[0, 5],
                                     kappa_maps=maps)
    assert dsb is None and dkb.shape == (3,) + shape
    for v in range(int(np.prod(shape))):
        e = np.zeros(int(np.prod(shape)))
        e[v] = 1.0
        J = oracle.trace_bins(e.reshape(shape), None, None, src, [9, 6], 0.5, 3.0, 1.0, caps=[0, 5],
                              kappa_maps=maps)
        per_bin = np.sum(G * J, axis=(1, 2, 3))
        assert np.isclose(dj.ravel()[v], per_bin.sum(), rtol=1e-10, atol=1e-12)
        assert np.allclose(djb.reshape(3, -1)[:, v], per_bin, rtol=1e-10, atol=1e-12)


BIN_PINS = [pin_bins_scale_finite_differences, pin_bins_kappa_finite_differences, pin_bins_j_jacobian_transpose]


@pytest.mark.parametrize("pin", BIN_PINS, ids=lambda p: p.__name__)
def test_bins_adjoint_pin(pin):
    pin(oracle)


BIN_MUTANTS = {
    "shared kappa gradient without the bin scale": ("dk += scales[b] * k", "dk += k"),
    "scale gradient against the scaled kappa": ("ds[b] = float(np.sum(base * k))",
                                                "ds[b] = float(np.sum(kappas[b] * k))"),
    "shared j keeps one bin": ("            dj += a\n", "            dj = a\n"),
    "bins read the base kappa": ("kappas = [base * scales[b] for b in range(n_bins)]",
                                 "kappas = [base for b in range(n_bins)]"),
}


@pytest.mark.parametrize("name", sorted(BIN_MUTANTS))
def test_bins_adjoint_pins_catch_mutant(name):
    src = open(oracle_adjoint.__file__).read()
    old, new = BIN_MUTANTS[name]
    assert old in src
    mod = types.ModuleType("adjoint_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new, 1), "adjoint_mutant", "exec"), mod.__dict__)
    failed = []
    for pin in BIN_PINS:
        try:
            pin(mod)
        except Exception:  # noqa: BLE001
            failed.append(pin.__name__)
    assert failed, f"no pin catches: {name}"

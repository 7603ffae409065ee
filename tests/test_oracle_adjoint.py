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

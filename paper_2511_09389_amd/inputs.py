"""Seeded synthetic inputs for the ray march (no part of the method's arithmetic).

The paper's turbulent media come from hydro snapshots that are not available, so these
generators stand in for them (Sec. 3, "Turbulent snapshots from hydro"): a lognormal
opacity built from a Gaussian random field with a Kolmogorov-like k^(-11/3) spectrum,
Gaussian emissivity blobs, and sources at blob centres or at the highest-opacity voxels
("top 0.1 % density peaks"). Everything is produced on the host with NumPy's PCG64 from a
fixed seed and handed as plain float32 arrays to both the GPU library and the CPU oracle.

Workloads (grid n^3, unit cells):
  uniform_blob  32^3, kappa = 0.05, one Gaussian j (sigma 1.5, amplitude 1) at (16,16,16),
                source at (16,16,16), 256 rays, ds 0.5, c dt 16 (32 substeps).
  turbulent     128^3 lognormal kappa (mean 0.02, sigma_ln 1), 16 random blobs and sources,
                4096 rays per source, ds 0.5, c dt 128 (256 substeps).
  uneven_bins   256^3 lognormal kappa (mean 0.01), 64 sources with N_Omega drawn from
                {1024, ..., 16384} and substep caps from [64, 512], 4 bins with
                kappa_nu = kappa (nu/nu0)^-3, nu/nu0 in {1, 1.5, 2, 3}, c dt 256.
  inverse       64^3 lognormal kappa (mean 0.03), 8 sources, 2048 rays, 128 substeps.
  surrogate     64^3 turbulent-style samples, 4096 rays, 128 substeps.
  peaks         128^3 turbulent kappa, 2097 sources at the largest-kappa voxels (0.1 %),
                unit Gaussians sigma 1 there, 4096 rays, 256 substeps.
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 1000


@dataclass
class Workload:
    """One synthetic problem: maps, sources and march parameters (all host arrays)."""

    name: str
    j_map: np.ndarray                    # float32 [nx][ny][nz]
    kappa_map: np.ndarray                # float32 [nx][ny][nz]
    source_pos: np.ndarray               # float32 [n_src][3], grid coordinates
    num_rays: np.ndarray                 # int32 [n_src]
    step_size: float
    radiation_velocity: float
    time_step: float
    substep_cap: Optional[np.ndarray] = None    # int32 [n_src] or None
    kappa_scale: Optional[np.ndarray] = None    # float32 [n_bins] or None
    notes: dict = field(default_factory=dict)

    @property
    def shape(self):
        return tuple(self.j_map.shape)

    @property
    def n_src(self):
        return int(self.source_pos.shape[0])

    @property
    def n_bins(self):
        return 1 if self.kappa_scale is None else int(self.kappa_scale.size)


def lognormal_kappa(n, mean, sigma_ln, rng, slope=-11.0 / 3.0):
    """Lognormal field exp(sigma_ln g) scaled to the given mean; g is a unit Gaussian
    random field on the periodic n^3 box with power spectrum P(k) ~ |k|^slope."""
    noise = rng.standard_normal((n, n, n))
    spec = np.fft.rfftn(noise)
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    kk = np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (slope / 2.0)
    g = np.fft.irfftn(spec * amp, s=(n, n, n), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    e = np.exp(sigma_ln * g)
    return (mean * e / e.mean()).astype(np.float32)


def gaussian_blobs(n, centres, sigmas, amps, cutoff=6.0):
    """Sum of A exp(-|x - c|^2 / (2 sigma^2)) at integer grid points, each blob cut off
    beyond `cutoff` sigma (below 1.6e-8 of its peak). Evaluated in float64, cast to float32."""
    out = np.zeros((n, n, n), dtype=np.float64)
    for c, s, a in zip(np.asarray(centres, np.float64), sigmas, amps):
        r = int(np.ceil(cutoff * s))
        lo = np.maximum(np.floor(c).astype(int) - r, 0)
        hi = np.minimum(np.floor(c).astype(int) + r + 2, n)
        if np.any(hi <= lo):
            continue
        axes = [np.exp(-((np.arange(lo[d], hi[d]) - c[d]) ** 2) / (2.0 * s * s)) for d in range(3)]
        out[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += a * axes[0][:, None, None] * axes[1][None, :, None] * axes[2][None, None, :]
    return out.astype(np.float32)


def _rng(config_id, sub=0):
    ss = np.random.SeedSequence(SEED_BASE + config_id)
    return np.random.default_rng(ss.spawn(sub + 1)[sub])


def uniform_blob(n=32, kappa=0.05, sigma=1.5, num_rays=256, ds=0.5, c=16.0, dt=1.0):
    """Uniform opacity, one Gaussian blob and one source at the grid centre n/2."""
    centre = np.array([n // 2] * 3, dtype=np.float32)
    j = gaussian_blobs(n, [centre], [sigma], [1.0], cutoff=1e9)
    kap = np.full((n, n, n), kappa, dtype=np.float32)
    return Workload("uniform_blob", j, kap, centre[None, :].copy(),
                    np.array([num_rays], np.int32), ds, c, dt)


def turbulent(n=128, n_src=16, kappa_mean=0.02, sigma_ln=1.0, num_rays=4096, ds=0.5,
              c=128.0, dt=1.0, config_id=2, sample=0):
    """Lognormal turbulent opacity, n_src random Gaussian blobs with a source at each centre:
    sigma ~ U[1, 3], amplitude ~ lognormal(0, 0.5), centre ~ U[0, n-1]^3."""
    rng_k = _rng(config_id, 2 * sample)
    rng_b = _rng(config_id, 2 * sample + 1)
    kap = lognormal_kappa(n, kappa_mean, sigma_ln, rng_k)
    centres = rng_b.uniform(0.0, n - 1, size=(n_src, 3)).astype(np.float32)
    sig = rng_b.uniform(1.0, 3.0, size=n_src)
    amp = np.exp(rng_b.normal(0.0, 0.5, size=n_src))
    j = gaussian_blobs(n, centres, sig, amp)
    return Workload("turbulent", j, kap, centres, np.full(n_src, num_rays, np.int32),
                    ds, c, dt, notes={"sigma": sig, "amplitude": amp})


def uneven_bins(n=256, n_src=64, kappa_mean=0.01, ds=0.5, c=256.0, dt=1.0,
                ray_choices=(1024, 2048, 4096, 8192, 16384), cap_range=(64, 512),
                nu=(1.0, 1.5, 2.0, 3.0), config_id=3):
    """Uneven batch: per-source N_Omega and substep caps, frequency bins scaling kappa."""
    w = turbulent(n=n, n_src=n_src, kappa_mean=kappa_mean, num_rays=1, ds=ds, c=c, dt=dt,
                  config_id=config_id)
    rng = _rng(config_id, 7)
    w.name = "uneven_bins"
    w.num_rays = rng.choice(np.asarray(ray_choices), size=n_src).astype(np.int32)
    w.substep_cap = rng.integers(cap_range[0], cap_range[1] + 1, size=n_src).astype(np.int32)
    w.kappa_scale = np.asarray([v ** -3.0 for v in nu], dtype=np.float32)
    return w


def inverse(n=64, n_src=8, kappa_mean=0.03, num_rays=2048, ds=0.5, c=64.0, dt=1.0):
    """Inverse-problem medium: turbulent kappa and a seeded 'true' j of 8 blobs."""
    w = turbulent(n=n, n_src=n_src, kappa_mean=kappa_mean, num_rays=num_rays, ds=ds, c=c,
                  dt=dt, config_id=4)
    w.name = "inverse"
    return w


def surrogate_sample(seed, n=64, n_src=16, num_rays=4096, ds=0.5, c=64.0, dt=1.0):
    """One training/evaluation sample for the surrogate (turbulent-style generator)."""
    w = turbulent(n=n, n_src=n_src, num_rays=num_rays, ds=ds, c=c, dt=dt, config_id=5,
                  sample=int(seed))
    w.name = "surrogate"
    return w


def peaks(n=128, frac=0.001, sigma=1.0, num_rays=4096, ds=0.5, c=128.0, dt=1.0):
    """Sources at the largest-kappa voxels (the top `frac` of the grid), unit Gaussian j there."""
    rng_k = _rng(6, 0)
    kap = lognormal_kappa(n, 0.02, 1.0, rng_k)
    count = int(np.floor(frac * n ** 3))
    flat = np.argsort(kap.ravel(), kind="stable")[::-1][:count]
    centres = np.stack(np.unravel_index(flat, kap.shape), axis=1).astype(np.float32)
    j = gaussian_blobs(n, centres, np.full(count, sigma), np.ones(count))
    return Workload("peaks", j, kap, centres, np.full(count, num_rays, np.int32), ds, c, dt)


def by_name(name, **kw):
    return {"uniform_blob": uniform_blob, "turbulent": turbulent, "uneven_bins": uneven_bins,
            "inverse": inverse, "peaks": peaks}[name](**kw)


def small_turbulent(n=24, n_src=3, num_rays=96, c=20.0, seed_sample=0, ds=0.5):
    """A reduced turbulent case the oracle finishes in well under a second."""
    return turbulent(n=n, n_src=n_src, num_rays=num_rays, c=c, ds=ds, config_id=2,
                     sample=100 + seed_sample)

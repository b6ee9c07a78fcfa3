"""Seeded synthetic inputs for the messenger-field Gibbs sampler.

This module only builds problem *inputs* (data d, per-voxel noise variance N
with +inf marking unobserved voxels, and an initial power-spectrum guess).  It
holds none of the sampler's arithmetic and is shared by the HIP path, the CPU
oracle and the benchmark.

The paper's mock (Sec. "Generation of a mock galaxy catalogue") uses an
Eisenstein-Hu LCDM spectrum, the SDSS DR7 completeness map and a Schechter
selection function, none of which is available here.  The stand-ins are:

* signal: a Gaussian random field with P(k) = A k^n exp(-(k/kc)^2), P(0) = 0;
* data model d = R s + eps with R = 1 on observed voxels, noise variance N_i
  (the count-noise form N_bar R_i of the mock section moved into N_i);
* survey geometry: either a random fraction of unobserved voxels, or a sphere
  of radius 0.45 L about the box centre minus a seeded 30-degree azimuthal
  wedge with a Gaussian radial selection, N_i = 1 / (nbar sel(r_i) V_cell).

All randomness comes from numpy's PCG64 seeded with the workload seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # grid side
    box: float             # box side L in h^-1 Mpc
    n_bins: int            # linear |k| bins on (0, sqrt(3) k_Nyquist]
    amp: float = 1.0e4     # A of P(k) = A k^n exp(-(k/kc)^2)
    index: float = -1.5    # n
    kc: float = 0.3        # h/Mpc
    mask: str = "random"   # "random" | "survey" | "none"
    mask_frac: float = 0.2         # unobserved fraction for mask="random"
    noise_lo: float = 0.5          # N_i = sigma2 * U[noise_lo, noise_hi] (random)
    noise_hi: float = 2.0
    sigma2: float = 1.0
    nbar: float = 3.0e-4           # (h/Mpc)^3, survey mask
    sel_r0: float = 400.0          # sel(r) = exp(-(r/sel_r0)^2)
    pk_init_frac: float = 0.1      # initial P guess = frac * truth at bin centres
    precision: str = "fp32"        # "fp64" | "fp32" (FP32 fields, FP64 shells/draws)
    sweeps: int = 10
    seed: int = 1000               # mock seed (PCG64)
    rng_seed: int = 2000           # Philox key of the chain

    @property
    def m(self) -> int:
        return self.n ** 3

    @property
    def cell_volume(self) -> float:
        return (self.box / self.n) ** 3


# The configurations the sampler is measured and checked on.
SMALL_FP64 = Workload("gibbs-32^3-fp64", n=32, box=500.0, n_bins=16, mask="random",
                      mask_frac=0.2, precision="fp64", sweeps=100, seed=1001, rng_seed=2001)
SURVEY_128_FP32 = Workload("gibbs-128^3-fp32-survey", n=128, box=1000.0, n_bins=32,
                           mask="survey", precision="fp32", sweeps=1000, seed=1002,
                           rng_seed=2002)
SURVEY_256_MIXED = Workload("gibbs-256^3-fp32-survey", n=256, box=2000.0, n_bins=64,
                            index=-1.0, mask="survey", precision="fp32", sweeps=500,
                            seed=1003, rng_seed=2003)

WORKLOADS = {w.name: w for w in (SMALL_FP64, SURVEY_128_FP32, SURVEY_256_MIXED)}


def power_spectrum(k: np.ndarray, w: Workload) -> np.ndarray:
    """Physical P(k) in h^-3 Mpc^3; P(0) = 0 (the field mean is not a mode)."""
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    nz = k > 0
    out[nz] = w.amp * k[nz] ** w.index * np.exp(-(k[nz] / w.kc) ** 2)
    return out


def wavenumber_grid(n: int, box: float, half: bool = False) -> np.ndarray:
    """|k| in h/Mpc on the DFT grid (full, or the iz <= n/2 half)."""
    kf = 2.0 * math.pi / box
    m = np.fft.fftfreq(n, d=1.0 / n)
    mz = np.arange(n // 2 + 1) if half else m
    kx = m[:, None, None]
    ky = m[None, :, None]
    kz = mz[None, None, :]
    return kf * np.sqrt(kx * kx + ky * ky + kz * kz)


def bin_centres(w: Workload) -> np.ndarray:
    """Centres of the n_bins equal-width |k| bins spanning (0, sqrt(3) k_Ny]."""
    k_ny = math.pi * w.n / w.box
    dk = math.sqrt(3.0) * k_ny / w.n_bins
    return (np.arange(w.n_bins) + 0.5) * dk


def gaussian_field(w: Workload, rng: np.random.Generator) -> np.ndarray:
    """Real field whose unnormalised DFT has E|s_k|^2 = M P(k) / V_cell."""
    white = rng.standard_normal((w.n, w.n, w.n))
    p_grid = power_spectrum(wavenumber_grid(w.n, w.box, half=True), w) / w.cell_volume
    return np.fft.irfftn(np.fft.rfftn(white) * np.sqrt(p_grid), s=(w.n,) * 3, axes=(0, 1, 2))


def voxel_centres(w: Workload):
    c = (np.arange(w.n) + 0.5) * (w.box / w.n) - 0.5 * w.box
    return c[:, None, None], c[None, :, None], c[None, None, :]


def survey_geometry(w: Workload, rng: np.random.Generator):
    """Observed mask and noise variance of the sphere-minus-wedge footprint."""
    x, y, z = voxel_centres(w)
    r = np.sqrt(x * x + y * y + z * z)
    phi = np.degrees(np.arctan2(y, x)) % 360.0
    phi0 = rng.uniform(0.0, 360.0)
    in_wedge = ((phi - phi0) % 360.0) < 30.0
    observed = (r < 0.45 * w.box) & ~np.broadcast_to(in_wedge, r.shape)
    sel = np.exp(-(r / w.sel_r0) ** 2)
    noise = 1.0 / (w.nbar * sel * w.cell_volume)
    return observed, np.broadcast_to(noise, r.shape)


def make_problem(w: Workload, seed: Optional[int] = None) -> dict:
    """Build (d, N, P_init, s_true) for a workload.

    Returns float64 arrays in C order (ix, iy, iz), iz fastest; N is +inf on
    unobserved voxels and d is 0 there.
    """
    rng = np.random.default_rng(w.seed if seed is None else seed)
    s_true = gaussian_field(w, rng)
    shape = (w.n,) * 3
    if w.mask == "none":
        observed = np.ones(shape, dtype=bool)
        noise = np.full(shape, w.sigma2, dtype=np.float64)
    elif w.mask == "random":
        observed = np.ones(w.m, dtype=bool)
        observed[rng.permutation(w.m)[: int(round(w.mask_frac * w.m))]] = False
        observed = observed.reshape(shape)
        noise = w.sigma2 * rng.uniform(w.noise_lo, w.noise_hi, size=shape)
    elif w.mask == "survey":
        observed, noise = survey_geometry(w, rng)
    else:
        raise ValueError(f"unknown mask kind {w.mask!r}")
    eps = rng.standard_normal(shape)
    noise_var = np.where(observed, noise, np.inf).astype(np.float64)
    data = np.where(observed, s_true + np.sqrt(np.where(observed, noise, 0.0)) * eps, 0.0)
    pk_init = w.pk_init_frac * power_spectrum(bin_centres(w), w)
    return {
        "data": np.ascontiguousarray(data, dtype=np.float64),
        "noise_var": np.ascontiguousarray(noise_var),
        "pk_init": pk_init.astype(np.float64),
        "s_true": s_true,
        "observed": observed,
    }


def small_workload(n: int, n_bins: int, mask: str = "random", precision: str = "fp64",
                   seed: int = 7, rng_seed: int = 11, box: Optional[float] = None,
                   **kw) -> Workload:
    """A reduced-size workload (tests): cell of 15.625 h^-1 Mpc unless box given."""
    return Workload(f"test-{n}^3", n=n, box=box if box is not None else 15.625 * n,
                    n_bins=n_bins, mask=mask, precision=precision, seed=seed,
                    rng_seed=rng_seed, **kw)


# Batched independent chains of several grid sides in one graph: per chain its
# own seed, random mask fraction in [0.1, 0.4] and noise level sigma^2
# log-uniform in [0.25, 4]; cell 15.625 h^-1 Mpc, P(k) with n = -1.5, 16 bins.
BATCHED_SIZES = ((64, 32), (48, 8), (80, 8), (96, 8))   # (grid side, chains)


def batched_chain(n: int, chain: int, base_seed: int = 3000, precision: str = "fp32") -> Workload:
    rng = np.random.default_rng(base_seed + 1000 * n + chain)
    frac = float(rng.uniform(0.1, 0.4))
    sigma2 = float(np.exp(rng.uniform(np.log(0.25), np.log(4.0))))
    return Workload(f"batch-{n}^3-{chain}", n=n, box=15.625 * n, n_bins=16, mask="random",
                    mask_frac=frac, sigma2=sigma2, precision=precision, sweeps=200,
                    seed=base_seed + 1000 * n + chain, rng_seed=base_seed)

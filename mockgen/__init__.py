"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only *draws inputs*: log-normal particle catalogues standing in
for the N-body snapshot the paper measures on (Sec. 3, the MDPL2 z=0
subsample), uniform random catalogues, and random fields for the small
field-level checks.  It holds none of the estimator's arithmetic (no deposit,
no multipole kernel, no contraction), so the CPU oracle and the GPU library
can both be fed from it without sharing any code with each other.

Recipe for a log-normal catalogue (all steps in float64):
  1. white noise w ~ N(0,1) on the analysis grid (n^3 cells, cell a = box/n);
  2. Gaussian spectrum P(k) = k^-1.5 exp(-(k R)^2), k in h/Mpc, P(0) = 0;
  3. amplitude A = n^3 / sum_{k != 0} P(k), so the expected grid variance of
     G is one;
  4. G = Re ifftn( fftn(w) sqrt(A P) );
  5. 1 + delta_LN = exp(G - 1/2);
  6. cell counts ~ Multinomial(N_p, (1 + delta_LN) / sum(1 + delta_LN));
  7. each particle uniform inside its cell, positions rounded to float32 and
     wrapped into [0, box);
  8. weights one, or uniform in [0.5, 1.5) rounded to float32.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "lognormal_catalogue", "uniform_catalogue",
    "workload_catalogue", "batch_sizes", "random_field", "band_limited_field",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: grid, box, multipole order, radial bins."""
    name: str
    box: float          # periodic box side, Mpc/h
    n: int              # grid points per side
    lmax: int           # multipole truncation L
    r_lo: float         # first bin edge, Mpc/h
    r_hi: float         # last bin edge, Mpc/h
    nbins: int          # number of linear radial bins
    n_particles: int    # particles per catalogue
    smoothing: float    # Gaussian smoothing R of the input spectrum, Mpc/h
    weights: str        # "unit" or "uniform"
    form: str           # summation form the workload is quoted with
    seed_base: int      # seeds: field = base+1, sample = base+2, weights = base+3, randoms = base+4

    @property
    def edges(self) -> np.ndarray:
        return np.linspace(self.r_lo, self.r_hi, self.nbins + 1)

    @property
    def cell(self) -> float:
        return self.box / self.n

    @property
    def units(self) -> float:
        """Work units of one evaluation: N_g (L+1)^2 N_r."""
        return float(self.n) ** 3 * (self.lmax + 1) ** 2 * self.nbins


WORKLOADS = {
    # small plain-FP64 case; grid summation; 10k uniform randoms alongside
    "box250_n32_l4": Workload("box250_n32_l4", 250.0, 32, 4, 10.0, 60.0, 6,
                              2_000, 4.0, "unit", "gamma", 1000),
    # particle summation, 1e6 particles on 128^3
    "box1000_n128_l10": Workload("box1000_n128_l10", 1000.0, 128, 10, 20.0, 150.0, 15,
                                 1_000_000, 8.0, "unit", "particle", 2000),
    # grid summation, 256^3, L = 10, 20 bins: the throughput workload
    "box2000_n256_l10": Workload("box2000_n256_l10", 2000.0, 256, 10, 20.0, 200.0, 20,
                                 8_000_000, 8.0, "unit", "nodal", 3000),
    # particle summation, 512^3, 5e7 weighted particles
    "box3000_n512_l10": Workload("box3000_n512_l10", 3000.0, 512, 10, 20.0, 200.0, 20,
                                 50_000_000, 8.0, "uniform", "particle", 4000),
    # 64 mocks of uneven size through one batched call, forward + adjoint
    "batch64_n128_l8": Workload("batch64_n128_l8", 1000.0, 128, 8, 20.0, 140.0, 12,
                                0, 8.0, "unit", "nodal", 5000),
}


def _gaussian_field(n: int, box: float, smoothing: float, rng: np.random.Generator) -> np.ndarray:
    noise = rng.standard_normal((n, n, n))
    f = np.fft.fftfreq(n, d=1.0 / n)
    kf = 2.0 * np.pi / box
    k2 = (f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2) * kf * kf
    k = np.sqrt(k2)
    spec = np.zeros_like(k)
    nz = k > 0
    spec[nz] = k[nz] ** -1.5 * np.exp(-(k[nz] * smoothing) ** 2)
    amp = n ** 3 / spec.sum()
    g_hat = np.fft.fftn(noise) * np.sqrt(amp * spec)
    g_hat[0, 0, 0] = 0.0
    return np.fft.ifftn(g_hat).real


def _wrap32(pos: np.ndarray, box: float) -> np.ndarray:
    p = pos.astype(np.float32)
    b = np.float32(box)
    p = np.where(p >= b, p - b, p)
    p = np.where(p < 0, p + b, p)
    p = np.where(p >= b, np.float32(0.0), p)
    return np.ascontiguousarray(p, dtype=np.float32)


def lognormal_catalogue(n: int, box: float, n_particles: int, smoothing: float,
                        seed_field: int, seed_sample: int,
                        seed_weights: int | None = None,
                        weight_range: tuple[float, float] | None = None):
    """Log-normal catalogue: (pos [N_p,3] float32, w [N_p] float32)."""
    g = _gaussian_field(n, box, smoothing, np.random.default_rng(seed_field))
    rho = np.exp(g - 0.5).ravel()
    del g
    p = rho / rho.sum()
    rng = np.random.default_rng(seed_sample)
    counts = rng.multinomial(n_particles, p)
    del p, rho
    cells = np.repeat(np.arange(n ** 3, dtype=np.int64), counts)
    del counts
    ix, rem = np.divmod(cells, n * n)
    iy, iz = np.divmod(rem, n)
    del cells, rem
    a = box / n
    pos = np.empty((n_particles, 3), dtype=np.float64)
    jit = rng.random((n_particles, 3))
    pos[:, 0] = (ix + jit[:, 0]) * a
    pos[:, 1] = (iy + jit[:, 1]) * a
    pos[:, 2] = (iz + jit[:, 2]) * a
    del jit, ix, iy, iz
    pos32 = _wrap32(pos, box)
    if weight_range is None:
        w = np.ones(n_particles, dtype=np.float32)
    else:
        lo, hi = weight_range
        w = np.random.default_rng(seed_weights).uniform(lo, hi, n_particles).astype(np.float32)
    return pos32, w


def uniform_catalogue(n_particles: int, box: float, seed: int):
    """Uniform random catalogue in [0, box)^3 (float32 positions, unit weights)."""
    pos = np.random.default_rng(seed).random((n_particles, 3)) * box
    return _wrap32(pos, box), np.ones(n_particles, dtype=np.float32)


def batch_sizes(count: int = 64, seed: int = 5999, lo: int = 200_000, hi: int = 1_000_000) -> np.ndarray:
    """Uneven per-mock particle counts for the batched workload."""
    return np.random.default_rng(seed).integers(lo, hi + 1, count)


def workload_catalogue(wl: Workload, index: int = 0, n_particles: int | None = None):
    """Catalogue for a named workload.  ``index`` selects a mock of a batch."""
    if wl.name.startswith("batch"):
        sizes = batch_sizes()
        npart = int(sizes[index]) if n_particles is None else n_particles
        base = wl.seed_base + 10 * index
    else:
        npart = wl.n_particles if n_particles is None else n_particles
        base = wl.seed_base
    wr = (0.5, 1.5) if wl.weights == "uniform" else None
    return lognormal_catalogue(wl.n, wl.box, npart, wl.smoothing,
                               base + 1, base + 2, base + 3, wr)


def random_field(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Zero-mean white-noise field on an n^3 grid."""
    f = np.random.default_rng(seed).standard_normal((n, n, n))
    f -= f.mean()
    return np.ascontiguousarray(f.astype(dtype))


def band_limited_field(n: int, seed: int, kmax_frac: float = 0.5) -> np.ndarray:
    """Real zero-mean field whose spectrum vanishes on and near the Nyquist planes.

    Only modes with |n_d| < kmax_frac * n/2 on every axis are kept.
    """
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n))
    fh = np.fft.fftn(f)
    fr = np.abs(np.fft.fftfreq(n, d=1.0 / n))
    keep = fr < kmax_frac * n / 2
    mask = keep[:, None, None] & keep[None, :, None] & keep[None, None, :]
    fh = np.where(mask, fh, 0.0)
    fh[0, 0, 0] = 0.0
    return np.ascontiguousarray(np.fft.ifftn(fh).real)

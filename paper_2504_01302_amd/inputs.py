"""Seeded synthetic inputs for the JAM-cyl forward model.

This module only draws numbers: Multi-Gaussian-expansion (MGE) parameters,
sky grids, a sampled PSF kernel, bin maps and per-model parameters.  It holds
none of the model's arithmetic (no deprojection, no potential, no moments), so
that both the GPU path and the FP64 oracle can consume the same inputs without
sharing any computation.

The shapes follow the paper's kinematic workload (App. "Simulated mock
datasets": a single Gaussian kinematic PSF of FWHM 0.14 arcsec, Voronoi bins
over a small field of view; Sect. 3.2: MGEs of the light and of the mass, the
two sets differing in size).  The paper's RXJ1131 data are not available, so
every input here is synthetic and drawn from a seeded generator:

* MGE dispersions sigma' log-uniform in [0.02, 5] arcsec, apparent axis
  ratios q' uniform in [0.6, 0.95], luminous peaks I0 log-uniform over 3 dex,
  mass peaks Sigma0 log-uniform over 3 dex in Msun/pc^2;
* one central black-hole Gaussian of dispersion 0.01 arcsec, q' = 1;
* square pixel grids centred on the galaxy, optional supersampling;
* a Gaussian PSF sampled at sub-pixel centres and normalised to unit sum;
* bins built by assigning every pixel to its nearest random generator point
  (a Voronoi tessellation, hence contiguous), standing in for VorBin;
* per-model inclination, anisotropy, mass scale and BH mass drawn as listed
  for each workload below.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

# Ranges of the synthetic MGEs.
SIGMA_RANGE = (0.02, 5.0)          # arcsec, log-uniform
Q_RANGE = (0.6, 0.95)              # apparent axis ratio, uniform
LOG_I0_RANGE = (0.0, 3.0)          # dex, luminous peak (arbitrary units)
LOG_S0_RANGE = (1.0, 4.0)          # dex, mass peak in Msun/pc^2
BH_SIGMA = 0.01                    # arcsec
DISTANCE_MPC = 1000.0              # 1 Gpc


@dataclass
class Geometry:
    """Everything about one galaxy model that a sampler does not vary.

    Pixel ``(ix, iy)`` of the field of view has its centre at
    ``x = xc + (ix - (nx-1)/2) * pixsize``, ``y = yc + (iy - (ny-1)/2) * pixsize``
    (arcsec; x along the projected major axis).  ``bin_index[iy, ix]`` is the
    bin of that pixel, -1 meaning excluded.  ``psf`` is an odd square kernel
    sampled on the sub-pixel grid (pitch ``pixsize / supersample``).
    """
    lum_sigma: np.ndarray
    lum_q: np.ndarray
    lum_I0: np.ndarray
    mass_sigma: np.ndarray
    mass_q: np.ndarray
    mass_S0: np.ndarray
    bh_sigma: float
    distance_mpc: float
    nx: int
    ny: int
    pixsize: float
    xc: float
    yc: float
    supersample: int
    psf: np.ndarray
    n_bins: int
    bin_index: np.ndarray
    n_u: int

    @property
    def n_lum(self) -> int:
        return int(self.lum_sigma.shape[0])

    @property
    def n_mass(self) -> int:
        return int(self.mass_sigma.shape[0])

    @property
    def psf_n(self) -> int:
        return int(self.psf.shape[0])


@dataclass
class Params:
    """What a sampler proposes for one model.

    ``inc`` in radians (pi/2 = edge-on); ``beta`` one anisotropy per luminous
    Gaussian; ``mass_scale`` multiplies every stellar/dark mass Gaussian (not
    the BH); ``m_bh`` in Msun.  ``lum_I0`` / ``mass_S0`` override the
    geometry's default amplitudes when given.
    """
    inc: float
    beta: np.ndarray
    mass_scale: float
    m_bh: float
    lum_I0: Optional[np.ndarray] = None
    mass_S0: Optional[np.ndarray] = None


@dataclass
class Workload:
    name: str
    geometries: List[Geometry]
    geom_idx: np.ndarray          # [n_models] int32
    params: List[Params] = field(default_factory=list)


def _rng(cfg: int, seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(seed)]))


def _log_uniform(rng, lo, hi, n):
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n)


def draw_mge(rng, n_lum: int, n_mass: int):
    """Luminous and mass MGE components with the ranges stated above."""
    lum_sigma = np.sort(_log_uniform(rng, *SIGMA_RANGE, n_lum))
    lum_q = rng.uniform(*Q_RANGE, n_lum)
    lum_I0 = 10.0 ** rng.uniform(*LOG_I0_RANGE, n_lum)
    mass_sigma = np.sort(_log_uniform(rng, *SIGMA_RANGE, n_mass))
    mass_q = rng.uniform(*Q_RANGE, n_mass)
    mass_S0 = 10.0 ** rng.uniform(*LOG_S0_RANGE, n_mass)
    return lum_sigma, lum_q, lum_I0, mass_sigma, mass_q, mass_S0


def gaussian_psf(fwhm: float, pitch: float, n: int) -> np.ndarray:
    """Odd ``n x n`` Gaussian kernel sampled at sub-pixel centres, unit sum."""
    if n % 2 != 1:
        raise ValueError("PSF size must be odd")
    sig = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    h = (n - 1) // 2
    o = np.arange(-h, h + 1) * pitch
    k = np.exp(-0.5 * (o[None, :] ** 2 + o[:, None] ** 2) / sig ** 2)
    return k / k.sum()


def psf_size_for(fwhm: float, pitch: float) -> int:
    """Half-width ceil(4 sigma / pitch), as an odd kernel size."""
    sig = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    return 2 * int(np.ceil(4.0 * sig / pitch)) + 1


def voronoi_bins(rng, nx: int, ny: int, n_bins: int) -> np.ndarray:
    """Nearest-generator bin map ``[ny, nx]``; redrawn until no bin is empty.

    Ties go to the lower generator index (``argmin`` keeps the first).
    """
    if n_bins > nx * ny:
        raise ValueError("more bins than pixels")
    iy, ix = np.mgrid[0:ny, 0:nx]
    px = ix.ravel().astype(np.float64)
    py = iy.ravel().astype(np.float64)
    for _ in range(1000):
        gx = rng.uniform(-0.5, nx - 0.5, n_bins)
        gy = rng.uniform(-0.5, ny - 0.5, n_bins)
        best = np.zeros(px.shape, dtype=np.int64)
        bestd = np.full(px.shape, np.inf)
        for b in range(n_bins):        # chunked argmin keeps memory small
            d = (px - gx[b]) ** 2 + (py - gy[b]) ** 2
            upd = d < bestd
            best[upd] = b
            bestd[upd] = d[upd]
        counts = np.bincount(best, minlength=n_bins)
        if np.all(counts > 0):
            return best.reshape(ny, nx).astype(np.int32)
    raise RuntimeError("could not draw a bin map without empty bins")


def draw_inclination(rng, q_min: float, lo_deg=45.0, hi_deg=85.0, margin=0.02) -> float:
    """Uniform inclination, redrawn from the same stream until the flattest
    Gaussian stays deprojectable with a margin: cos(i) < q'_min - margin."""
    for _ in range(100000):
        i = np.deg2rad(rng.uniform(lo_deg, hi_deg))
        if np.cos(i) < q_min - margin:
            return float(i)
    raise RuntimeError("no admissible inclination")


def _geometry(rng, n_lum, n_mass, n, pixsize, ss, psf_fwhm, psf_n, n_bins, n_u):
    ls, lq, li, ms, mq, mS = draw_mge(rng, n_lum, n_mass)
    if psf_n is None:
        psf_n = psf_size_for(psf_fwhm, pixsize / ss)
    psf = gaussian_psf(psf_fwhm, pixsize / ss, psf_n)
    bins = voronoi_bins(rng, n, n, n_bins)
    return Geometry(ls, lq, li, ms, mq, mS, BH_SIGMA, DISTANCE_MPC,
                    n, n, pixsize, 0.0, 0.0, ss, psf, n_bins, bins, n_u)


def _q_min(g: Geometry) -> float:
    return float(np.concatenate([g.lum_q, g.mass_q]).min())


def _proposal(rng, g: Geometry) -> Params:
    """Sampler-like draw: inclination 45-85 deg (redrawn, see above), beta_k
    uniform in [-0.2, 0.4], mass scale uniform in [0.8, 1.2], BH mass
    log-uniform in [1e7, 10^9.5] Msun."""
    inc = draw_inclination(rng, _q_min(g))
    beta = rng.uniform(-0.2, 0.4, g.n_lum)
    ml = float(rng.uniform(0.8, 1.2))
    mbh = float(10.0 ** rng.uniform(7.0, 9.5))
    return Params(inc, beta, ml, mbh)


# --------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------

def config1(seed: int = 0) -> Workload:
    """Single small forward: 10 luminous + 12 mass Gaussians + BH (10^8.5 Msun),
    i = 60 deg, beta_k = 0.1, 30x30 grid at 0.05", 100 u-nodes, Gaussian PSF
    FWHM 0.1" (9x9), 20 bins."""
    rng = _rng(1, seed)
    g = _geometry(rng, 10, 12, 30, 0.05, 1, 0.1, None, 20, 100)
    p = Params(np.deg2rad(60.0), np.full(10, 0.1), 1.0, 10.0 ** 8.5)
    return Workload("cfg1", [g], np.zeros(1, np.int32), [p])


def config2(seed: int = 0) -> Workload:
    """IFU scale: 40 luminous x 40 mass Gaussians + BH (10^8.5 Msun), 200x200
    grid at 0.025" with 2x supersampling, 128 u-nodes, 31x31 Gaussian PSF of
    FWHM 0.14" on the sub-grid, 60 bins; inclination 45-85 deg (redrawn),
    beta_k uniform in [-0.2, 0.4]."""
    rng = _rng(2, seed)
    g = _geometry(rng, 40, 40, 200, 0.025, 2, 0.14, 31, 60, 128)
    inc = draw_inclination(rng, _q_min(g))
    beta = rng.uniform(-0.2, 0.4, 40)
    p = Params(inc, beta, 1.0, 10.0 ** 8.5)
    return Workload("cfg2", [g], np.zeros(1, np.int32), [p])


def config3(n_models: int = 4096, seed: int = 0) -> Workload:
    """Batched proposals on the config-1 geometry, one draw per model."""
    base = config1(seed).geometries[0]
    rng = _rng(3, seed)
    params = [_proposal(rng, base) for _ in range(n_models)]
    return Workload("cfg3", [base], np.zeros(n_models, np.int32), params)


def config4(n_models: int = 1024, seed: int = 0) -> Workload:
    """Uneven batch: per model K, J uniform in 5..60, square grids 32..256,
    64..160 u-nodes, 10..100 bins; pitch 0.05", Gaussian PSF FWHM 0.1" (9x9),
    no supersampling; parameters drawn as for config 3."""
    rng = _rng(4, seed)
    geoms, params = [], []
    for _ in range(n_models):
        K = int(rng.integers(5, 61))
        J = int(rng.integers(5, 61))
        n = int(rng.integers(32, 257))
        nu = int(rng.integers(64, 161))
        nb = int(rng.integers(10, min(100, n * n) + 1))
        g = _geometry(rng, K, J, n, 0.05, 1, 0.1, 9, nb, nu)
        geoms.append(g)
        params.append(_proposal(rng, g))
    return Workload("cfg4", geoms, np.arange(n_models, dtype=np.int32), params)


def config5(n_models: int = 256, seed: int = 0) -> Workload:
    """Gradient workload: config-1 geometry, config-3 style draws."""
    w = config3(n_models, seed + 1000)
    w.name = "cfg5"
    return w


def config_composite(seed: int = 0) -> Workload:
    """The IFU-scale grid of config 2 with the Gaussian counts of the paper's
    composite lens model (42 light and 95 mass Gaussians + BH), for timing
    the spherically aligned path at the size the paper quotes."""
    rng = _rng(6, seed)
    g = _geometry(rng, 42, 95, 200, 0.025, 2, 0.14, 31, 60, 128)
    inc = draw_inclination(rng, _q_min(g))
    beta = rng.uniform(-0.2, 0.4, 42)
    p = Params(inc, beta, 1.0, 10.0 ** 8.5)
    return Workload("composite", [g], np.zeros(1, np.int32), [p])


def cotangent(n_bins: int, n_models: int, seed: int = 0) -> np.ndarray:
    """Seeded N(0,1) cotangent per bin and model, ``[n_models, n_bins]``."""
    return _rng(5, seed).standard_normal((n_models, n_bins))


# Synthetic kinematic data for the goodness of fit of eq. (chi2_dyn); the
# measured v_rms of the paper's lens and their covariance are not available.
VRMS_OBS_RANGE = (200.0, 400.0)    # km/s, uniform per bin
VRMS_REL_ERR = (0.04, 0.06)        # 1-sigma error per bin, relative, uniform
VRMS_SYS_REL = 0.02                # error common to all bins, relative


def kinematic_data(n_bins: int, seed: int = 0):
    """Observed v_rms per bin [km/s] and the covariance of their errors
    [(km/s)^2]: independent per-bin errors of 4-6 % plus a 2 % error shared
    by all bins, cov = diag(e_b^2) + 0.02^2 v v^T (symmetric positive
    definite)."""
    rng = _rng(11, seed)
    v = rng.uniform(*VRMS_OBS_RANGE, n_bins)
    e = rng.uniform(*VRMS_REL_ERR, n_bins) * v
    cov = np.diag(e ** 2) + VRMS_SYS_REL ** 2 * np.outer(v, v)
    return v, cov


def with_overrides(p: Params, **kw) -> Params:
    return replace(p, **kw)


def small_geometry(seed: int = 0, n_lum=3, n_mass=2, nx=9, ny=7, ss=1,
                   psf_n=3, n_bins=4, n_u=24, pixsize=0.1, xc=0.0, yc=0.0,
                   psf_fwhm=0.15) -> Geometry:
    """A tiny, possibly off-centre, non-square geometry for unit tests."""
    rng = _rng(9, seed)
    ls, lq, li, ms, mq, mS = draw_mge(rng, n_lum, n_mass)
    psf = gaussian_psf(psf_fwhm, pixsize / ss, psf_n)
    bins = voronoi_bins(rng, nx, ny, n_bins)
    return Geometry(ls, lq, li, ms, mq, mS, BH_SIGMA, DISTANCE_MPC,
                    nx, ny, pixsize, xc, yc, ss, psf, n_bins, bins, n_u)


def small_params(g: Geometry, seed: int = 0) -> Params:
    rng = _rng(10, seed)
    return _proposal(rng, g)

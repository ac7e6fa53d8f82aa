"""Plain FP64 CPU oracle of the cylindrically aligned JAM projected second
moment, PSF convolution and luminosity-weighted binning.

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU library.  Only
the test suite, the package smoke check and the benchmark's CPU-baseline leg
may import it; the product path never does.  It shares no code with the GPU
path: it is written directly from the paper's equations and from the
derivation stated below, with PyTorch CPU tensors in float64 so that autograd
yields the exact gradient of the same arithmetic.

What is computed (paper Sect. 2.4, App. A):

* The observed MGEs of the light, eq. (sb_mge_2D), and of the mass,
  eq. (smd_mge), are deprojected at inclination i (App. A):
  q = sqrt(q'^2 - cos^2 i) / sin i, requiring cos^2 i < q'^2_min, with peak
  density q' I0 / (sqrt(2 pi) sigma q), eq. (sb_mge_3D) / (smd_3D).
* The paper refers the potential and the Jeans solution to the JAM
  literature instead of printing them.  This oracle uses the standard
  potential of a deprojected Gaussian of total mass M (oblate homoeoid
  theorem; reduces to -G M erf(r / sqrt(2) sigma) / r when q = 1):
      Phi(R, z) = -sqrt(2/pi) G M / sigma
                  * int_0^1 exp(-u^2 (R^2 + z^2 / h) / (2 sigma^2)) / sqrt(h) du,
      h = 1 - (1 - q^2) u^2.
* Cylindrically aligned Jeans equations with v_R^2 = b_k v_z^2 per luminous
  Gaussian, b_k = 1 / (1 - beta_k):
      nu v_z^2 = int_z^inf nu dPhi/dz dz,
      nu (v_phi^2 - v_R^2) = b_k R d(nu v_z^2)/dR + R nu dPhi/dR.
* The line-of-sight second moment, with the line of sight along
  (0, sin i, cos i) in galaxy coordinates, is
      v_los^2 = cos^2 i v_z^2 + sin^2 i [v_R^2 + (v_phi^2 - v_R^2) x'^2 / R^2],
  and eq. (VLos) integrates rho_* v_los^2 along the line of sight.
* For each luminous Gaussian k, mass Gaussian j and quadrature node u, the
  z-integral and the line-of-sight integral are Gaussian and close exactly;
  the integrand of the u-integral is
      sqrt(pi / a) exp(-c1 x'^2 - gamma y'^2) (P + Q x'^2)
  with c1, A, a, gamma, g, w, P, Q as in ``term_coefficients``.  The
  u-integral is an n_u-node Gauss-Legendre rule on [0, 1].
* Finally the PSF-convolved, bin-summed ratio of the two maps (Sect. 2.4,
  unnumbered equation before eq. (Vrms)) gives v_rms^2 per bin.

Readings where the paper is silent: the PSF acts on both the numerator map
I v_los^2 and on I, evaluated on a grid padded by the kernel half-width
('valid' convolution); supersampled sub-pixels inherit their parent pixel's
bin; the mass scale multiplies every mass Gaussian except the BH.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import numpy as np
import torch

DT = torch.float64

# ---------------------------------------------------------------------------
# Units.  Lengths on the sky in arcsec, masses in Msun, velocities in km/s.
# G in pc (km/s)^2 / Msun from the IAU nominal solar mass parameter and the
# IAU astronomical unit; 1 pc = 648000/pi au.
# ---------------------------------------------------------------------------
GM_SUN_SI = 1.3271244e20            # m^3 s^-2
AU_M = 149597870700.0               # m
PC_M = AU_M * 648000.0 / math.pi    # m
G_PC_KMS2 = GM_SUN_SI / (PC_M * 1.0e6)   # ~4.30091e-3


def pc_per_arcsec(distance_mpc: float) -> float:
    """Physical length of one arcsec at angular-diameter distance D."""
    return distance_mpc * 1.0e6 * math.pi / 648000.0


def gauss_legendre_unit(n: int):
    """n-node Gauss-Legendre rule mapped to [0, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _t(v):
    if isinstance(v, torch.Tensor):
        return v.to(DT)
    return torch.as_tensor(np.asarray(v, dtype=np.float64), dtype=DT)


# ---------------------------------------------------------------------------
# App. A: deprojection of an observed Gaussian.
# ---------------------------------------------------------------------------

def intrinsic_axis_ratio(q_obs, inc):
    """q = sqrt(q'^2 - cos^2 i) / sin i (App. A); needs cos^2 i < q'^2."""
    c2 = torch.cos(inc) ** 2
    if torch.any(q_obs ** 2 <= c2):
        raise ValueError("inclination below the deprojection limit cos^2 i < q'^2_min")
    return torch.sqrt(q_obs ** 2 - c2) / torch.sin(inc)


def peak_density(amp, sigma, q_obs, q_intr):
    """Central 3-D density of a deprojected Gaussian, eq. (sb_mge_3D):
    q' I0 / (sqrt(2 pi) sigma q)   [amplitude units per arcsec]."""
    return q_obs * amp / (math.sqrt(2.0 * math.pi) * sigma * q_intr)


def gaussian_total_mass(S0, sigma_obs, q_obs, pc_as):
    """Total mass of one term of eq. (smd_mge): 2 pi Sigma0 (s sigma')^2 q'."""
    return 2.0 * math.pi * S0 * (pc_as * sigma_obs) ** 2 * q_obs


# ---------------------------------------------------------------------------
# The model for one set of parameters.
# ---------------------------------------------------------------------------

def _param_tensors(geom, params, overrides=None):
    """Torch views of everything the model depends on (leaf tensors allowed
    through ``overrides`` for autograd)."""
    o = dict(overrides or {})
    I0 = params.lum_I0 if params.lum_I0 is not None else geom.lum_I0
    S0 = params.mass_S0 if params.mass_S0 is not None else geom.mass_S0
    return dict(
        inc=o.get("inc", _t(params.inc)),
        beta=o.get("beta", _t(params.beta)),
        mass_scale=o.get("mass_scale", _t(params.mass_scale)),
        m_bh=o.get("m_bh", _t(params.m_bh)),
        lum_I0=o.get("lum_I0", _t(I0)),
        mass_S0=o.get("mass_S0", _t(S0)),
    )


def mass_gaussians(geom, pt):
    """Intrinsic dispersion [arcsec], axis ratio and total mass [Msun] of
    every mass Gaussian, the BH appended last (q' = 1)."""
    s = pc_per_arcsec(geom.distance_mpc)
    inc = pt["inc"]
    q_obs = _t(geom.mass_q)
    sig = _t(geom.mass_sigma)
    q = intrinsic_axis_ratio(q_obs, inc)
    M = pt["mass_scale"] * gaussian_total_mass(pt["mass_S0"], sig, q_obs, s)
    sig_all = torch.cat([sig, _t([geom.bh_sigma])])
    q_all = torch.cat([q, torch.ones(1, dtype=DT)])
    M_all = torch.cat([M, pt["m_bh"].reshape(1)])
    return sig_all, q_all, M_all


def tracer_gaussians(geom, pt):
    """Intrinsic dispersion, axis ratio, peak density and b_k of the light."""
    q_obs = _t(geom.lum_q)
    sig = _t(geom.lum_sigma)
    q = intrinsic_axis_ratio(q_obs, pt["inc"])
    nu0 = peak_density(pt["lum_I0"], sig, q_obs, q)
    b = 1.0 / (1.0 - pt["beta"])
    return sig, q, nu0, b


def term_coefficients(geom, pt):
    """Per (k, j, n) coefficients of the u-integrand, shape [K, J+1, n_u].

    Returns (c1, gamma, C0, C1) such that the sky numerator is
        N(x', y') = sum_{k,j,n} exp(-c1 x'^2 - gamma y'^2) (C0 + C1 x'^2).

    Derivation per term (sigma_k, q_k, nu0_k tracer; sigma_j, q_j, M_j mass):
      K_j = sqrt(2/pi) G M_j / (s sigma_j)               potential scale
      nu_k dPhi_j/dz   = nu0 K u^2 z / (sigma_j^2 h^{3/2}) exp(-c1 R^2 - A z^2)
      nu_k v_z^2       = g exp(-c1 R^2 - A z^2),  g = nu0 K u^2 / (2 A sigma_j^2 h^{3/2})
      nu_k (1/R) dPhi_j/dR = w exp(...),         w = nu0 K u^2 / (sigma_j^2 h^{1/2})
      with c1 = 1/(2 sigma_k^2) + u^2/(2 sigma_j^2),
           A  = 1/(2 sigma_k^2 q_k^2) + u^2/(2 sigma_j^2 h),  h = 1 - (1-q_j^2) u^2.
      nu v_los^2 = (P + Q x'^2) exp(-c1 R^2 - A z^2),
           P = (cos^2 i + b sin^2 i) g,   Q = sin^2 i (w - 2 c1 b g).
      Along the line of sight R^2 = x'^2 + (z' sin i - y' cos i)^2 and
      z = y' sin i + z' cos i, so the z'-integral gives
      sqrt(pi/a) exp(-c1 x'^2 - gamma y'^2) with a = c1 sin^2 i + A cos^2 i,
      gamma = c1 A / a.
    The quadrature weight w_n and sqrt(pi/a) are folded into C0, C1.
    """
    s = pc_per_arcsec(geom.distance_mpc)
    inc = pt["inc"]
    si2 = torch.sin(inc) ** 2
    ci2 = torch.cos(inc) ** 2
    sk, qk, nu0, b = tracer_gaussians(geom, pt)
    sj, qj, Mj = mass_gaussians(geom, pt)
    u_np, w_np = gauss_legendre_unit(geom.n_u)
    u = _t(u_np)
    wq = _t(w_np)

    Kj = math.sqrt(2.0 / math.pi) * G_PC_KMS2 * Mj / (s * sj)      # [(km/s)^2]
    # broadcast to [K, J+1, n_u]
    sk_ = sk[:, None, None]
    qk_ = qk[:, None, None]
    nu_ = nu0[:, None, None]
    b_ = b[:, None, None]
    sj_ = sj[None, :, None]
    e2_ = (1.0 - qj ** 2)[None, :, None]
    K_ = Kj[None, :, None]
    u2 = (u ** 2)[None, None, :]

    h = 1.0 - e2_ * u2
    c1 = 1.0 / (2.0 * sk_ ** 2) + u2 / (2.0 * sj_ ** 2)
    A = 1.0 / (2.0 * sk_ ** 2 * qk_ ** 2) + u2 / (2.0 * sj_ ** 2 * h)
    a = c1 * si2 + A * ci2
    gamma = c1 * A / a
    g = nu_ * K_ * u2 / (2.0 * A * sj_ ** 2 * h ** 1.5)
    w = nu_ * K_ * u2 / (sj_ ** 2 * torch.sqrt(h))
    P = (ci2 + b_ * si2) * g
    Q = si2 * (w - 2.0 * c1 * b_ * g)
    f = wq[None, None, :] * torch.sqrt(math.pi / a)
    return c1, gamma, f * P, f * Q


def numerator(coeffs, x, y, chunk: Optional[int] = None):
    """N(x', y') = int rho_* v_los^2 dz' at the points (x[i], y[i]).

    Points are processed in chunks that keep the [terms x points] temporaries
    near 2^24 elements; the sum over terms of every point is unchanged."""
    c1, gam, C0, C1 = (t.reshape(-1) for t in coeffs)
    x = _t(x).reshape(-1)
    y = _t(y).reshape(-1)
    if chunk is None:
        chunk = max(1, min(4096, (1 << 24) // max(1, c1.shape[0])))
    out = []
    for s in range(0, x.shape[0], chunk):
        xx = (x[s:s + chunk] ** 2)[None, :]
        yy = (y[s:s + chunk] ** 2)[None, :]
        e = torch.exp(-c1[:, None] * xx - gam[:, None] * yy)
        out.append(torch.sum(e * (C0[:, None] + C1[:, None] * xx), dim=0))
    return torch.cat(out) if out else torch.zeros(0, dtype=DT)


def surface_brightness(geom, I0, x, y):
    """eq. (sb_mge_2D): I(x', y') = sum_k I0_k exp(-(x'^2 + y'^2/q'^2)/(2 sigma'^2))."""
    x = _t(x).reshape(-1)[None, :]
    y = _t(y).reshape(-1)[None, :]
    sig = _t(geom.lum_sigma)[:, None]
    q = _t(geom.lum_q)[:, None]
    I0 = _t(I0)[:, None]
    return torch.sum(I0 * torch.exp(-(x ** 2 + y ** 2 / q ** 2) / (2.0 * sig ** 2)), dim=0)


# ---------------------------------------------------------------------------
# Sky sampling, PSF and bins.
# ---------------------------------------------------------------------------

def padded_subgrid(geom):
    """Sub-pixel centre coordinates of the field of view extended by the PSF
    half-width h on every side: (x [nxp], y [nyp], h)."""
    ss = geom.supersample
    h = (geom.psf_n - 1) // 2
    pitch = geom.pixsize / ss
    mx = np.arange(-h, geom.nx * ss + h, dtype=np.float64)
    my = np.arange(-h, geom.ny * ss + h, dtype=np.float64)
    x = geom.xc + (mx - (geom.nx * ss - 1) / 2.0) * pitch
    y = geom.yc + (my - (geom.ny * ss - 1) / 2.0) * pitch
    return x, y, h


def convolve_valid(m_pad, psf, h: int):
    """True 2-D convolution restricted to the field of view:
    C[p] = sum_o psf[o + h] * M[p - o], o in [-h, h]^2."""
    psf = _t(psf)
    nyp, nxp = m_pad.shape
    ny, nx = nyp - 2 * h, nxp - 2 * h
    out = torch.zeros((ny, nx), dtype=DT)
    for oy in range(-h, h + 1):
        for ox in range(-h, h + 1):
            out = out + psf[oy + h, ox + h] * m_pad[h - oy:h - oy + ny, h - ox:h - ox + nx]
    return out


def subpixel_bins(geom) -> np.ndarray:
    """Bin index of every field-of-view sub-pixel (parent pixel's bin)."""
    ss = geom.supersample
    return np.repeat(np.repeat(geom.bin_index, ss, axis=0), ss, axis=1)


def bin_sums(c_map, geom):
    """Sum a field-of-view sub-pixel map over every bin (index -1 dropped)."""
    bins = torch.as_tensor(subpixel_bins(geom).reshape(-1).astype(np.int64))
    vals = c_map.reshape(-1)
    keep = bins >= 0
    out = torch.zeros(geom.n_bins, dtype=DT)
    return out.index_add(0, bins[keep], vals[keep])


# ---------------------------------------------------------------------------
# Public oracle entry points.
# ---------------------------------------------------------------------------

def maps(geom, params, overrides=None):
    """(N, I) on the padded sub-pixel grid, shape [nyp, nxp] each."""
    pt = _param_tensors(geom, params, overrides)
    x, y, _ = padded_subgrid(geom)
    X, Y = np.meshgrid(x, y)
    coeffs = term_coefficients(geom, pt)
    N = numerator(coeffs, X.ravel(), Y.ravel()).reshape(X.shape)
    I = surface_brightness(geom, pt["lum_I0"], X.ravel(), Y.ravel()).reshape(X.shape)
    return N, I


def vrms2(geom, params, overrides=None):
    """v_rms^2 per bin [(km/s)^2] (Sect. 2.4, eqs. VLos and Vrms)."""
    N, I = maps(geom, params, overrides)
    h = (geom.psf_n - 1) // 2
    Nb = bin_sums(convolve_valid(N, geom.psf, h), geom)
    Ib = bin_sums(convolve_valid(I, geom.psf, h), geom)
    return Nb / Ib


GRAD_KEYS = ("inc", "beta", "mass_scale", "m_bh", "lum_I0", "mass_S0")


def vrms2_and_grad(geom, params, cot):
    """v_rms^2 and the gradient of sum_b cot_b v_rms^2_b with respect to the
    inclination, every beta_k, the mass scale, the BH mass and every luminous
    and mass amplitude (exact autograd of the FP64 arithmetic above)."""
    pt0 = _param_tensors(geom, params)
    leaves = {k: pt0[k].detach().clone().requires_grad_(True) for k in GRAD_KEYS}
    V = vrms2(geom, params, overrides=leaves)
    L = torch.sum(V * _t(cot))
    grads = torch.autograd.grad(L, [leaves[k] for k in GRAD_KEYS])
    return V.detach(), {k: g.detach() for k, g in zip(GRAD_KEYS, grads)}


def needed_padded_mask(geom, bins: Sequence[int]):
    """Padded sub-pixels whose values enter the convolved map on the given
    bins (the bins' sub-pixels dilated by the PSF footprint)."""
    h = (geom.psf_n - 1) // 2
    sb = subpixel_bins(geom)
    sel = np.isin(sb, np.asarray(bins))
    ny, nx = sel.shape
    need = np.zeros((ny + 2 * h, nx + 2 * h), dtype=bool)
    for oy in range(-h, h + 1):
        for ox in range(-h, h + 1):
            need[h - oy:h - oy + ny, h - ox:h - ox + nx] |= sel
    return need


def vrms2_bins(geom, params, bins: Sequence[int]):
    """v_rms^2 of selected bins only, evaluating N and I just where the
    convolution on those bins reads them (for large grids)."""
    pt = _param_tensors(geom, params)
    x, y, h = padded_subgrid(geom)
    X, Y = np.meshgrid(x, y)
    need = needed_padded_mask(geom, bins)
    coeffs = term_coefficients(geom, pt)
    N = torch.zeros(X.shape, dtype=DT)
    I = torch.zeros(X.shape, dtype=DT)
    idx = np.nonzero(need.ravel())[0]
    N.view(-1)[idx] = numerator(coeffs, X.ravel()[idx], Y.ravel()[idx])
    I.view(-1)[idx] = surface_brightness(geom, pt["lum_I0"], X.ravel()[idx], Y.ravel()[idx])
    Nb = bin_sums(convolve_valid(N, geom.psf, h), geom)
    Ib = bin_sums(convolve_valid(I, geom.psf, h), geom)
    b = torch.as_tensor(np.asarray(bins, dtype=np.int64))
    return (Nb / Ib)[b]


def point_values(geom, params, x, y):
    """(N, I) at arbitrary sky points (no PSF), for sampled comparisons."""
    pt = _param_tensors(geom, params)
    coeffs = term_coefficients(geom, pt)
    return numerator(coeffs, x, y), surface_brightness(geom, pt["lum_I0"], x, y)


# ---------------------------------------------------------------------------
# Goodness of fit of the dynamical model, eq. (chi2_dyn).
# ---------------------------------------------------------------------------

def chi2_dyn(V, vrms_obs, cov):
    """chi^2 = (v_obs - v_pre)^T Sigma_kin^-1 (v_obs - v_pre), eq. (chi2_dyn),
    with the predicted v_rms = sqrt of the binned second moment, eq. (Vrms).
    ``cov`` is the covariance of the measured v_rms [(km/s)^2]; the product
    with its inverse is a linear solve."""
    V = torch.as_tensor(V, dtype=DT)
    r = _t(vrms_obs) - torch.sqrt(V)
    return torch.dot(r, torch.linalg.solve(_t(cov), r))


def chi2_and_grad(geom, params, vrms_obs, cov):
    """chi^2 of one model (eq. chi2_dyn on eq. Vrms of the binned moments) and
    its gradient with respect to the parameters of ``GRAD_KEYS`` (exact
    autograd of the FP64 arithmetic)."""
    pt0 = _param_tensors(geom, params)
    leaves = {k: pt0[k].detach().clone().requires_grad_(True) for k in GRAD_KEYS}
    V = vrms2(geom, params, overrides=leaves)
    c2 = chi2_dyn(V, vrms_obs, cov)
    grads = torch.autograd.grad(c2, [leaves[k] for k in GRAD_KEYS])
    return float(c2.detach()), {k: g.detach() for k, g in zip(GRAD_KEYS, grads)}

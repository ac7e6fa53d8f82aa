"""Plain FP64 CPU oracle of the spherically aligned JAM projected second
moment (the paper's dynamics, Sect. 2.4, eqs. J1 and J2), on the same MGE
deprojection, potential, PSF and bins as the cylindrical oracle.

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU library; only
the test suite may import it.  It shares no code with the GPU path (it reuses
the cylindrical oracle's deprojection, potential constants, sub-pixel grid,
convolution and bin sums, which are themselves oracle code).

The solution of eqs. J1, J2 used here (derived; the paper refers it to the
JAM literature):

* Eliminating nu v_phi^2 between J2 and J1 leaves, for P = nu v_r^2 of one
  tracer Gaussian with constant beta,
      d_r P - (1 - beta) (tan(theta) / r) d_theta P + 2 beta P / r = S,
      S = -nu d_r Phi + (tan(theta) / r) nu d_theta Phi = -nu (d_z Phi) / cos(theta).
* Its characteristics are the curves r^(1 - beta) sin(theta) = const; along
  them d(r^(2 beta) P)/dr = r^(2 beta) S, so with P -> 0 at infinity
      P(r, theta) = r^(-2 beta) int_r^inf r'^(2 beta) nu (d_z Phi) / cos(theta') dr',
      sin(theta') = sin(theta) (r / r')^(1 - beta).
  For the MGE potential (d_z Phi) / cos(theta) = r G(R, z) with
      G = sum_j K_j int_0^1 u^2 / (sigma_j^2 h^(3/2)) E du,
      E = exp(-u^2 (R^2 + z^2 / h) / (2 sigma_j^2)),  h = 1 - e_j^2 u^2.
* Differentiating along theta at fixed r (d_theta R = z, d_theta z = -R)
  multiplies the Gaussians' integrands by polynomials, so
      d_theta P = r^(1 - 3 beta) cos(theta) I_D,
      I_D = int_r^inf r'^(3 beta + 1) R' nu [G_theta + G (1/q_k^2 - 1)/sigma_k^2] dr',
      G_theta = sum_j K_j int_0^1 e_j^2 u^6 / (sigma_j^4 h^(5/2)) E du,
  and J2 gives
      nu v_phi^2 = (1 - beta) P + (1 - beta) sin(theta) r^(1 - 3 beta) I_D - nu R^2 G_phi,
      G_phi = sum_j K_j int_0^1 e_j^2 u^4 / (sigma_j^2 h^(3/2)) E du;
  nu v_theta^2 = (1 - beta) P by the definition of beta.
* With the line of sight n = (0, sin i, cos i) in galaxy coordinates (the
  cylindrical oracle's convention), the projected second moment is
      nu v_los^2 = (n.e_r)^2 nu v_r^2 + (n.e_theta)^2 nu v_theta^2 + (n.e_phi)^2 nu v_phi^2,
  n.e_r = sin i sin(theta) sin(phi) + cos i cos(theta),
  n.e_theta = sin i cos(theta) sin(phi) - cos i sin(theta),  n.e_phi = sin i cos(phi),
  and N(x', y') = int nu v_los^2 dz'.

Discretisation (the paper fixes a non-adaptive mesh for the intrinsic
moments but not its layout; these are the readings both sides use):
* r' integral: tau = ln(r'/r) on [0, ln(r_max / r)], r_max^2 = r^2 + 50 sigma_k^2
  (along a characteristic nu_k falls at least as fast as exp(-r'^2 / (2 sigma_k^2)),
  so the integrand has dropped by e^-25 there), SEG_TAU segments of NODE_TAU
  Gauss-Legendre nodes each;
* u integral: the geometry's n_u Gauss-Legendre nodes on [0, 1];
* intrinsic moments summed over the tracer Gaussians, A_r = sum P_k,
  A_theta = sum (1 - beta_k) P_k, A_phi = sum nu v_phi^2_k, tabulated on a
  polar grid of N_R radii log-spaced on [r_lo, r_hi] and N_TH angles evenly
  spaced on [0, pi/2], and interpolated bicubically (Catmull-Rom in ln r and
  in theta; at the ends of the radial range the missing radius is
  extrapolated linearly, and the moments are even about theta = 0 and
  theta = pi/2, so the missing angles are mirror images); below r_lo the
  first radius is used, beyond r_hi the moments are zero;
* line of sight: z' = a sinh(w), w on [-W, W] with sinh(W) a = Z, SEG_LOS
  segments of NODE_LOS Gauss-Legendre nodes, a = min_k sigma_k q_k / 4,
  Z = 12 max_k sigma_k.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import jam as ojam

SEG_TAU, NODE_TAU = 8, 8
SEG_LOS, NODE_LOS = 8, 8
N_R, N_TH = 128, 24


def _composite_gl(a: float, b: float, seg: int, nodes: int):
    x, w = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(a, b, seg + 1)
    xs, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        xs.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w)
    return np.concatenate(xs), np.concatenate(ws)


def model(geom, params):
    """FP64 numpy arrays of the deprojected tracer and mass Gaussians."""
    pt = ojam._param_tensors(geom, params)
    sk, qk, nu0, _ = ojam.tracer_gaussians(geom, pt)
    sj, qj, Mj = ojam.mass_gaussians(geom, pt)
    s = ojam.pc_per_arcsec(geom.distance_mpc)
    Kj = math.sqrt(2.0 / math.pi) * ojam.G_PC_KMS2 * Mj / (s * sj)
    u, wu = ojam.gauss_legendre_unit(geom.n_u)
    return dict(sk=sk.numpy(), qk=qk.numpy(), nu0=nu0.numpy(), beta=np.asarray(params.beta, np.float64),
                sj=sj.numpy(), e2=(1.0 - qj ** 2).numpy(), Kj=Kj.numpy(), u=u, wu=wu,
                inc=float(params.inc))


def _potential_terms(m, R, z):
    """G, G_theta, G_phi at the points (R, z) (any shape)."""
    R2 = (R * R)[..., None, None]
    z2 = (z * z)[..., None, None]
    sj = m["sj"][:, None]
    e2 = m["e2"][:, None]
    u2 = (m["u"] ** 2)[None, :]
    h = 1.0 - e2 * u2
    E = np.exp(-u2 * (R2 + z2 / h) / (2.0 * sj ** 2))
    wK = (m["wu"][None, :] * m["Kj"][:, None])
    G = np.sum(wK * u2 / (sj ** 2 * h ** 1.5) * E, axis=(-2, -1))
    Gt = np.sum(wK * e2 * u2 ** 3 / (sj ** 4 * h ** 2.5) * E, axis=(-2, -1))
    Gp = np.sum(wK * e2 * u2 ** 2 / (sj ** 2 * h ** 1.5) * E, axis=(-2, -1))
    return G, Gt, Gp


def _nu(m, k, R, z):
    return m["nu0"][k] * np.exp(-(R * R + z * z / m["qk"][k] ** 2) / (2.0 * m["sk"][k] ** 2))


def tracer_moments(m, k, r, theta):
    """(nu v_r^2, nu v_phi^2) of tracer Gaussian k at the points (r, theta)."""
    r = np.asarray(r, np.float64)
    theta = np.asarray(theta, np.float64)
    beta = m["beta"][k]
    sk, qk = m["sk"][k], m["qk"][k]
    P = np.zeros(r.shape)
    ID = np.zeros(r.shape)
    for idx in np.ndindex(r.shape):
        rr, th = float(r[idx]), float(theta[idx])
        rmax = math.sqrt(rr * rr + 50.0 * sk * sk)
        tau, wt = _composite_gl(0.0, math.log(rmax / rr), SEG_TAU, NODE_TAU)
        rp = rr * np.exp(tau)
        st = np.clip(math.sin(th) * (rr / rp) ** (1.0 - beta), 0.0, 1.0)
        ct = np.sqrt(1.0 - st * st)
        Rp, zp = rp * st, rp * ct
        G, Gt, _ = _potential_terms(m, Rp, zp)
        nu = _nu(m, k, Rp, zp)
        # dr' = r' dtau
        P[idx] = rr ** (-2.0 * beta) * np.sum(wt * rp ** (2.0 * beta + 2.0) * nu * G)
        ID[idx] = np.sum(wt * rp ** (3.0 * beta + 2.0) * Rp * nu *
                         (Gt + G * (1.0 / qk ** 2 - 1.0) / sk ** 2))
    R, z = r * np.sin(theta), r * np.cos(theta)
    _, _, Gp = _potential_terms(m, R, z)
    nu = _nu(m, k, R, z)
    phi = (1.0 - beta) * P + (1.0 - beta) * np.sin(theta) * r ** (1.0 - 3.0 * beta) * ID - nu * R * R * Gp
    return P, phi


def intrinsic_moments(m, r, theta):
    """A_r, A_theta, A_phi summed over the tracer Gaussians."""
    Ar = np.zeros(np.shape(r))
    At = np.zeros(np.shape(r))
    Ap = np.zeros(np.shape(r))
    for k in range(len(m["sk"])):
        P, ph = tracer_moments(m, k, r, theta)
        Ar += P
        At += (1.0 - m["beta"][k]) * P
        Ap += ph
    return Ar, At, Ap


def polar_grid(geom):
    """Radii and angles of the moment table: r on [r_lo, r_hi] (log), theta
    on [0, pi/2]; r_lo is half the smallest distance of a padded sub-pixel
    centre from the centre, r_hi = 12 max sigma_k / q'_min."""
    x, y, _ = ojam.padded_subgrid(geom)
    rs = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)
    r_lo = 0.5 * float(np.min(rs[rs > 0])) if np.any(rs > 0) else 1e-3
    r_hi = 12.0 * float(np.max(geom.lum_sigma)) / float(np.min(geom.lum_q))
    r = np.exp(np.linspace(math.log(r_lo), math.log(r_hi), N_R))
    th = np.linspace(0.0, 0.5 * math.pi, N_TH)
    return r, th


def moment_table(geom, params):
    m = model(geom, params)
    r, th = polar_grid(geom)
    RR, TT = np.meshgrid(r, th, indexing="ij")
    return m, r, th, intrinsic_moments(m, RR, TT)


def radial_weights(fx):
    """Catmull-Rom weights of the four radii i-1, i, i+1, i+2 around a point
    at fraction fx of cell [i, i+1] (cubic convolution, a = -1/2)."""
    f2, f3 = fx * fx, fx * fx * fx
    return ((-f3 + 2.0 * f2 - fx) / 2.0, (3.0 * f3 - 5.0 * f2 + 2.0) / 2.0,
            (-3.0 * f3 + 4.0 * f2 + fx) / 2.0, (f3 - f2) / 2.0)


def _interp(table, r, th, rq, tq):
    """Bicubic (Catmull-Rom in ln r and in theta).  In r the missing radius at
    either end is extrapolated linearly from the two nearest; in theta the
    moments are even about the axis (theta = 0) and about the equatorial plane
    (theta = pi/2), so the missing angles are mirror images.  The first radius
    stands for smaller ones; zero beyond the last."""
    lr = np.log(r)
    n, nt = len(r), len(th)
    x = (np.log(rq) - lr[0]) / (lr[1] - lr[0])
    y = tq / (th[1] - th[0])
    xi = np.clip(np.floor(x), 0, n - 2).astype(int)
    yi = np.clip(np.floor(y), 0, nt - 2).astype(int)
    fx = np.clip(x - xi, 0.0, 1.0)
    fy = np.clip(y - yi, 0.0, 1.0)
    wx = radial_weights(fx)
    wy = radial_weights(fy)
    out = []
    for T in table:
        def row(i):          # cubic in theta at radius index i (mirrored angles)
            v = 0.0
            for b in range(4):
                j = yi - 1 + b
                j = np.where(j < 0, -j, np.where(j > nt - 1, 2 * (nt - 1) - j, j))
                v = v + wy[b] * T[i, j]
            return v
        p0, p1 = row(xi), row(xi + 1)
        pm = np.where(xi >= 1, row(np.maximum(xi - 1, 0)), 2.0 * p0 - p1)
        p2 = np.where(xi + 2 <= n - 1, row(np.minimum(xi + 2, n - 1)), 2.0 * p1 - p0)
        v = wx[0] * pm + wx[1] * p0 + wx[2] * p1 + wx[3] * p2
        out.append(np.where(x > n - 1, 0.0, v))
    return out


def los_nodes(geom, params):
    m = model(geom, params)
    a = float(np.min(m["sk"] * m["qk"])) / 4.0
    Z = 12.0 * float(np.max(m["sk"]))
    W = math.asinh(Z / a)
    w, ww = _composite_gl(-W, W, SEG_LOS, NODE_LOS)
    return a * np.sinh(w), ww * a * np.cosh(w)


def _project(m, x, y, zp, moments_at):
    """nu v_los^2 at sky (x, y) and line-of-sight offsets zp."""
    si, ci = math.sin(m["inc"]), math.cos(m["inc"])
    X = np.broadcast_to(x, zp.shape)
    Y = zp * si - y * ci
    Z = y * si + zp * ci
    R = np.sqrt(X * X + Y * Y)
    r = np.sqrt(R * R + Z * Z)
    ct = Z / r
    st = R / r
    with np.errstate(invalid="ignore", divide="ignore"):
        sp = np.where(R > 0, Y / R, 0.0)
        cp = np.where(R > 0, X / R, 0.0)
    Ar, At, Ap = moments_at(r, np.arccos(np.abs(ct)))
    ner = si * st * sp + ci * ct
    net = si * ct * sp - ci * st
    nep = si * cp
    return ner ** 2 * Ar + net ** 2 * At + nep ** 2 * Ap


def numerator_direct(geom, params, x, y):
    """N(x', y') with the moments evaluated at every line-of-sight node (no
    table): the reference for the table's interpolation error."""
    m = model(geom, params)
    zp, wz = los_nodes(geom, params)
    out = []
    for xx, yy in zip(np.atleast_1d(x), np.atleast_1d(y)):
        f = _project(m, float(xx), float(yy), zp, lambda r, t: intrinsic_moments(m, r, t))
        out.append(np.sum(wz * f))
    return np.array(out)


def numerator_table(geom, params, x, y, table=None):
    """N(x', y') with the moments interpolated from the polar table."""
    if table is None:
        table = moment_table(geom, params)
    m, r, th, T = table
    zp, wz = los_nodes(geom, params)
    xs, ys = np.atleast_1d(x), np.atleast_1d(y)
    out = np.empty(len(xs))
    for i, (xx, yy) in enumerate(zip(xs, ys)):
        f = _project(m, float(xx), float(yy), zp, lambda rq, tq: _interp(T, r, th, rq, tq))
        out[i] = np.sum(wz * f)
    return out


def vrms2(geom, params):
    """v_rms^2 per bin of the spherically aligned model (table path)."""
    import torch
    table = moment_table(geom, params)
    x, y, h = ojam.padded_subgrid(geom)
    X, Y = np.meshgrid(x, y)
    N = numerator_table(geom, params, X.ravel(), Y.ravel(), table).reshape(X.shape)
    pt = ojam._param_tensors(geom, params)
    I = ojam.surface_brightness(geom, pt["lum_I0"], X.ravel(), Y.ravel()).reshape(X.shape)
    Nb = ojam.bin_sums(ojam.convolve_valid(torch.as_tensor(N), geom.psf, h), geom)
    Ib = ojam.bin_sums(ojam.convolve_valid(I, geom.psf, h), geom)
    return (Nb / Ib).numpy()

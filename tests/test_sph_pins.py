"""Pins of the spherically aligned JAM oracle (Sect. 2.4, eqs. J1, J2)
against things other than itself: the cylindrical closed form where the two
alignments coincide (isotropy), the textbook one-dimensional anisotropic
spherical Jeans solution and its projection, the Jeans equations themselves
by finite differences, and the size of the polar table's interpolation
error."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import jam as ojam
from oracle import jam_sph as S
from paper_2504_01302_amd import inputs

pytestmark = pytest.mark.slow


def _geom(seed, **kw):
    base = dict(n_lum=3, n_mass=2, nx=8, ny=7, psf_n=3, n_bins=3, n_u=48)
    base.update(kw)
    return inputs.small_geometry(seed=seed, **base)


def test_isotropic_equals_cylindrical_closed_form():
    """With beta = 0 both alignments describe the same isotropic meridional
    dispersion, so the spherical line-of-sight integral of the characteristic
    solution must reproduce the cylindrical closed form, flattened and
    inclined."""
    g = _geom(3)
    p = inputs.with_overrides(inputs.small_params(g, seed=3), beta=np.zeros(g.n_lum))
    xs = np.array([0.05, 0.3, 0.0, 0.25, 0.12])
    ys = np.array([0.1, 0.0, 0.2, 0.25, 0.05])
    Ns = S.numerator_direct(g, p, xs, ys)
    Nc = ojam.point_values(g, p, xs, ys)[0].numpy()
    assert np.all(np.abs(Ns - Nc) <= 2e-6 * np.abs(Nc) + 1e-9 * np.max(np.abs(Nc))), Ns / Nc - 1


def _spherical_geometry():
    g = _geom(6, n_lum=2, n_mass=2)
    return inputs.Geometry(g.lum_sigma, np.ones(g.n_lum), g.lum_I0, g.mass_sigma,
                           np.ones(g.n_mass), g.mass_S0, g.bh_sigma, g.distance_mpc, g.nx, g.ny,
                           g.pixsize, g.xc, g.yc, g.supersample, g.psf, g.n_bins, g.bin_index, 160)


def _textbook(g, p):
    """nu v_r^2(r) of each tracer Gaussian from the 1-D spherical Jeans
    equation with constant beta, with dPhi/dr = G M(<r) / r^2 of spherical
    Gaussians (enclosed mass erf(x) - sqrt(2/pi) x exp(-x^2/2), x = r/sigma)."""
    m = S.model(g, p)
    s = ojam.pc_per_arcsec(g.distance_mpc)
    Mj = m["Kj"] * s * m["sj"] / (math.sqrt(2.0 / math.pi) * ojam.G_PC_KMS2)

    def dphi(r):
        x = r / m["sj"]
        enc = special.erf(x / math.sqrt(2.0)) - math.sqrt(2.0 / math.pi) * x * np.exp(-x * x / 2)
        return ojam.G_PC_KMS2 * float(np.sum(Mj * enc)) / (s * r * r)

    def P(k, r):
        b = m["beta"][k]
        f = lambda rr: rr ** (2 * b) * m["nu0"][k] * math.exp(-rr * rr / (2 * m["sk"][k] ** 2)) * dphi(rr)
        return r ** (-2 * b) * integrate.quad(f, r, r + 40 * m["sk"][k], epsabs=0, epsrel=1e-12,
                                               limit=400)[0]
    return m, P


def test_spherical_anisotropic_matches_textbook():
    """q' = 1 everywhere: nu v_r^2 equals the textbook integral, nu v_phi^2 =
    (1 - beta) nu v_r^2, and the projection equals the textbook
    Sigma sigma_p^2(R) = 2 int_R^inf (1 - beta R^2/r^2) nu v_r^2 r dr / sqrt(r^2 - R^2)."""
    g = _spherical_geometry()
    p = inputs.Params(math.radians(60.0), np.array([0.35, -0.25]), 1.0, 1e8)
    m, P = _textbook(g, p)
    for k in range(2):
        for r, th in [(0.05, 0.3), (0.2, 1.1), (0.6, 0.7)]:
            Po, Fo = S.tracer_moments(m, k, np.array([r]), np.array([th]))
            ref = P(k, r)
            assert abs(Po[0] - ref) <= 2e-7 * abs(ref) + 1e-300, (k, r, Po[0], ref)
            assert abs(Fo[0] - (1 - m["beta"][k]) * Po[0]) <= 1e-12 * abs(Po[0])
    # projection, one sky radius, both tracers
    R = 0.15
    def integrand(rr):
        return sum((1 - m["beta"][k] * R * R / (rr * rr)) * P(k, rr) for k in range(2)) * rr
    u_max = 12 * max(m["sk"])
    # r = sqrt(R^2 + t^2) removes the endpoint singularity: dr r / sqrt(r^2-R^2) = dt
    ref = 2 * integrate.quad(lambda t: integrand(math.sqrt(R * R + t * t)) / math.sqrt(R * R + t * t),
                             0, u_max, epsabs=0, epsrel=1e-10, limit=400)[0]
    got = S.numerator_direct(g, p, np.array([R / math.sqrt(2)]), np.array([R / math.sqrt(2)]))[0]
    assert abs(got - ref) <= 1e-6 * abs(ref), (got, ref)


def test_jeans_equations_hold(monkeypatch):
    """Flattened, inclined, anisotropic (beta = 0.3 and -0.2): central finite
    differences of nu v_r^2 with nu v_phi^2 satisfy eqs. J1 and J2."""
    monkeypatch.setattr(S, "SEG_TAU", 16)
    monkeypatch.setattr(S, "NODE_TAU", 16)
    g = _geom(3, n_lum=2, n_mass=2)
    p = inputs.with_overrides(inputs.small_params(g, seed=3), beta=np.array([0.3, -0.2]))
    m = S.model(g, p)
    sj, e2 = m["sj"][:, None], m["e2"][:, None]
    u2 = (m["u"] ** 2)[None, :]
    hh = 1 - e2 * u2
    wK = m["wu"][None, :] * m["Kj"][:, None]
    for k in range(2):
        sk = m["sk"][k]
        for r, th in [(0.5 * sk, 0.4), (1.0 * sk, 1.2), (2.0 * sk, 0.9)]:
            PF = lambda rr, tt: S.tracer_moments(m, k, np.array([rr]), np.array([tt]))
            P0, F0 = PF(r, th)
            h = 1e-3
            Pr = (8 * (PF(r * (1 + h), th)[0] - PF(r * (1 - h), th)[0])
                  - (PF(r * (1 + 2 * h), th)[0] - PF(r * (1 - 2 * h), th)[0])) / (12 * h * r)
            Pt = (8 * (PF(r, th + h)[0] - PF(r, th - h)[0])
                  - (PF(r, th + 2 * h)[0] - PF(r, th - 2 * h)[0])) / (12 * h)
            b = m["beta"][k]
            R, z = r * math.sin(th), r * math.cos(th)
            E = np.exp(-u2 * (R * R + z * z / hh) / (2 * sj ** 2))
            PhR = np.sum(wK * u2 * R / (sj ** 2 * hh ** 0.5) * E)
            Phz = np.sum(wK * u2 * z / (sj ** 2 * hh ** 1.5) * E)
            nu = S._nu(m, k, np.array(R), np.array(z))
            dr = math.sin(th) * PhR + math.cos(th) * Phz
            dt = z * PhR - R * Phz
            J1 = Pr + ((1 + b) * P0 - F0) / r + nu * dr
            J2 = (1 - b) * Pt + ((1 - b) * P0 - F0) / math.tan(th) + nu * dt
            assert abs(J1) <= 1e-6 * (abs(Pr) + abs(nu * dr)), (k, r, th, J1)
            assert abs(J2) <= 1e-6 * (abs((1 - b) * Pt) + abs(nu * dt)), (k, r, th, J2)


def test_table_interpolation_error_is_small():
    """The polar table (128 x 24, bicubic in ln r and theta) stays
    within 1e-3 of the moments evaluated at every line-of-sight node."""
    g = _geom(4, n_u=32)
    p = inputs.small_params(g, seed=4)
    x, y, _ = ojam.padded_subgrid(g)
    X, Y = np.meshgrid(x, y)
    idx = np.random.default_rng(0).choice(X.size, 6, replace=False)
    Nd = S.numerator_direct(g, p, X.ravel()[idx], Y.ravel()[idx])
    Nt = S.numerator_table(g, p, X.ravel()[idx], Y.ravel()[idx])
    assert np.max(np.abs(Nt / Nd - 1)) <= 1e-3


def test_table_interpolation_reproduces_quadratics():
    """The bicubic (Catmull-Rom) interpolation reproduces any product of a
    quadratic in ln r and an even quadratic-plus-cos(2 theta) profile in
    theta exactly inside the table where the mirrored angles are exact, passes
    through the table's values, and its weights sum to one."""
    r = np.exp(np.linspace(np.log(0.01), np.log(50.0), 40))
    th = np.linspace(0.0, 0.5 * np.pi, 7)
    L, TH = np.meshgrid(np.log(r), th, indexing="ij")
    T = (0.3 + 1.7 * L - 0.45 * L ** 2) * (2.0 + 0.8 * (TH - 0.6) ** 2)
    rng = np.random.default_rng(3)
    rq = np.exp(rng.uniform(np.log(r[1]), np.log(r[-2]), 200))
    tq = rng.uniform(th[1], th[-2], 200)
    (v,) = S._interp([T], r, th, rq, tq)
    exact = (0.3 + 1.7 * np.log(rq) - 0.45 * np.log(rq) ** 2) * (2.0 + 0.8 * (tq - 0.6) ** 2)
    assert np.max(np.abs(v - exact)) <= 1e-11 * np.max(np.abs(exact))
    (vn,) = S._interp([T], r, th, r[[0, 5, 38]], th[[0, 3, 6]])
    assert np.allclose(vn, T[[0, 5, 38], [0, 3, 6]], rtol=1e-12, atol=0)
    for fx in np.linspace(0.0, 1.0, 11):
        assert abs(sum(S.radial_weights(fx)) - 1.0) < 1e-15


def test_table_interpolation_even_in_theta_at_the_ends():
    """With data even about theta = 0 and pi/2 (cos(2 theta) and cos(4
    theta) profiles) the mirrored end angles keep the interpolant close to
    the truth in the first and last angular cells."""
    r = np.exp(np.linspace(np.log(0.01), np.log(50.0), 20))
    th = np.linspace(0.0, 0.5 * np.pi, 24)
    L, TH = np.meshgrid(np.log(r), th, indexing="ij")
    T = 1.0 + 0.3 * np.cos(2 * TH) + 0.1 * np.cos(4 * TH)
    tq = np.concatenate([np.linspace(0.0, th[1], 9), np.linspace(th[-2], th[-1], 9)])
    rq = np.full_like(tq, r[7])
    (v,) = S._interp([T], r, th, rq, tq)
    exact = 1.0 + 0.3 * np.cos(2 * tq) + 0.1 * np.cos(4 * tq)
    assert np.max(np.abs(v - exact)) <= 2e-5

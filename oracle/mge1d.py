"""Plain FP64 CPU oracle of the one-dimensional multi-Gaussian expansion
(MGE) of a radial profile by an integral transform and the Euler algorithm.

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU library; only
the test suite may import it.  It shares no code with the GPU path.

What is computed (paper Sect. 3.2, eq. integral_transfer and the two
equations after it):

* A profile F(R) of the elliptical radius R is written as a continuous sum of
  Gaussians, F(R) = int f(sigma) / sqrt(2 pi) exp(-R^2 / (2 sigma^2)) dlog sigma.
  With s = 1 / (2 sigma^2) this is a Laplace transform in t = R^2, so the
  amplitude density is an inverse Laplace transform of F(sqrt(t)).
* The inversion uses the Euler algorithm: with P terms of the binomial
  (Euler) averaging, nodes beta_n = P ln(10) / 3 + i pi n and weights
  xi_0 = 1/2, xi_n = 1 (1 <= n <= P), xi_2P = 2^-P,
  xi_(2P-j) = xi_(2P-j+1) + 2^-P binom(P, j) (0 < j < P),
  the transform evaluates to f(sigma) = sum_n eta_n Re F(sigma chi_n) with
  chi_n = sqrt(2 beta_n) and eta_n = 2 sqrt(2 pi) 10^(P/3) (-1)^n xi_n.
* On N log-spaced sigma_n the integral over log sigma becomes a trapezoid
  sum: F(R) ~ sum_n A_n exp(-R^2 / (2 sigma_n^2)) with
  A_n = w_n f(sigma_n) dlog(sigma) / sqrt(2 pi), w = 1/2 at both ends and 1
  inside (natural logarithm).

Readings where the paper is silent: the Euler order P (the paper fixes only
that the eta_n, chi_n are precomputed), the weights w_n (trapezoid) and the
base of the logarithm (natural) are stated above.  Profiles are sums of cored
power-law components a (R^2 + c^2)^(-p), which cover the paper's Chameleon
and dPIE (p = 1/2 pairs), softened EPL (p = (gamma - 1) / 2) and the
core-steep-ellipsoid basis of its eNFW (p = 3/2); their inverse Laplace
transform is known in closed form, a s^(p-1) exp(-c^2 s) / Gamma(p), which
pins the inversion.
"""
from __future__ import annotations

import math

import numpy as np
import torch

DT = torch.float64
CT = torch.complex128


def euler_nodes(P: int):
    """Euler-algorithm nodes beta_n (complex) and weights (-1)^n xi_n, n = 0..2P."""
    xi = np.zeros(2 * P + 1)
    xi[0] = 0.5
    xi[1:P + 1] = 1.0
    xi[2 * P] = 2.0 ** -P
    for j in range(1, P):
        xi[2 * P - j] = xi[2 * P - j + 1] + 2.0 ** -P * math.comb(P, j)
    n = np.arange(2 * P + 1)
    beta = P * math.log(10.0) / 3.0 + 1j * math.pi * n
    return beta, ((-1.0) ** n) * xi


def inverse_laplace(Fhat, s, P: int):
    """Euler approximation of the inverse Laplace transform of Fhat at s > 0:
    (10^(P/3) / s) sum_n (-1)^n xi_n Re Fhat(beta_n / s)."""
    beta, w = euler_nodes(P)
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    for b, wn in zip(beta, w):
        out = out + wn * np.real(Fhat(b / s))
    return 10.0 ** (P / 3.0) / s * out


def transform_constants(P: int):
    """chi_n = sqrt(2 beta_n) and eta_n = 2 sqrt(2 pi) 10^(P/3) (-1)^n xi_n."""
    beta, w = euler_nodes(P)
    chi = np.sqrt(2.0 * beta)
    eta = 2.0 * math.sqrt(2.0 * math.pi) * 10.0 ** (P / 3.0) * w
    return chi, eta


def cored_power_law(comp):
    """F(R) = sum_c a_c (R^2 + c_c^2)^(-p_c) for components (a, c, p) given as
    a tensor [n_comp, 3]; returns a function of complex R."""
    comp = torch.as_tensor(comp, dtype=DT)

    def F(R):
        R2 = R * R
        out = torch.zeros_like(R2)
        for k in range(comp.shape[0]):
            a, c, p = comp[k, 0], comp[k, 1], comp[k, 2]
            out = out + a * torch.exp(-p * torch.log(R2 + c * c))
        return out
    return F


def sigma_grid(sigma_min: float, sigma_max: float, n: int) -> np.ndarray:
    """n log-spaced dispersions between sigma_min and sigma_max."""
    return np.exp(np.linspace(math.log(sigma_min), math.log(sigma_max), n))


def mge_amplitudes(comp, sigma, P: int = 10):
    """Peak amplitudes A_n of the Gaussians exp(-R^2 / (2 sigma_n^2)) that
    expand the cored power-law profile ``comp`` (autograd flows to comp)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    N = len(sigma)
    chi, eta = transform_constants(P)
    F = cored_power_law(comp)
    z = torch.as_tensor(np.outer(sigma, chi), dtype=CT)           # [N, 2P+1]
    f = torch.sum(torch.as_tensor(eta, dtype=DT) * torch.real(F(z)), dim=1)
    dlog = (math.log(sigma[-1]) - math.log(sigma[0])) / (N - 1) if N > 1 else 1.0
    w = torch.ones(N, dtype=DT)
    if N > 1:
        w[0] = w[-1] = 0.5
    return w * f * dlog / math.sqrt(2.0 * math.pi)


def reconstruct(amp, sigma, R):
    """sum_n A_n exp(-R^2 / (2 sigma_n^2)) at real radii R."""
    R = torch.as_tensor(np.asarray(R, dtype=np.float64))
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64))
    return torch.sum(torch.as_tensor(amp) * torch.exp(-R[:, None] ** 2 / (2.0 * s ** 2)), dim=1)

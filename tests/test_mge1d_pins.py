"""Pins of the one-dimensional MGE oracle (Sect. 3.2: integral transform and
Euler algorithm) against things other than itself: hand-computed Euler
weights, the closed-form inverse Laplace transform of cored power laws, the
paper's ~0.5 % reconstruction accuracy with 21 Gaussians, linearity, and
central differences of the gradient."""
import math

import numpy as np
import pytest
import torch

from oracle import mge1d as M


def test_euler_weights_by_hand():
    # P = 2: xi = (1/2, 1, 1, 1/4 + 2^-2 binom(2, 1), 2^-2) = (.5, 1, 1, .75, .25)
    beta, w = M.euler_nodes(2)
    assert np.allclose(w, [0.5, -1.0, 1.0, -0.75, 0.25], rtol=0, atol=1e-15)
    assert np.allclose(beta.real, 2 * math.log(10.0) / 3.0, rtol=1e-15)
    assert np.allclose(beta.imag, math.pi * np.arange(5), rtol=1e-15)


@pytest.mark.parametrize("c,p", [(1.0, 0.5), (0.3, 1.5), (0.01, 0.5), (2.0, 1.0), (0.5, 0.2)])
def test_euler_inversion_of_cored_power_laws(c, p):
    """L^-1[(t + c^2)^-p](s) = s^(p-1) exp(-c^2 s) / Gamma(p)."""
    s = np.logspace(-3, 3, 61)
    exact = s ** (p - 1) * np.exp(-c * c * s) / math.gamma(p)
    for P, tol in ((10, 1e-6), (12, 5e-8)):
        approx = M.inverse_laplace(lambda t: (t + c * c) ** (-p), s, P)
        assert np.max(np.abs(approx - exact)) <= tol * np.max(np.abs(exact)), (P, c, p)


def test_reconstruction_within_half_percent():
    """A Chameleon-type light profile (difference of two cored isothermals)
    from 21 log-spaced Gaussians reproduces the profile to < 0.5 % over the
    fitted range, the accuracy the paper quotes."""
    sig = M.sigma_grid(0.005, 50.0, 21)
    comp = [[1.0, 0.05, 0.5], [-1.0, 2.0, 0.5]]
    A = M.mge_amplitudes(comp, sig, 10)
    R = np.logspace(-2, 1, 60)
    F = M.cored_power_law(comp)(torch.as_tensor(R, dtype=torch.complex128)).real
    err = torch.max(torch.abs(M.reconstruct(A.numpy(), sig, R) / F - 1))
    assert float(err) < 5e-3


def test_amplitudes_linear_in_component_amplitudes():
    sig = M.sigma_grid(0.01, 20.0, 15)
    a = M.mge_amplitudes([[1.0, 0.1, 0.7]], sig)
    b = M.mge_amplitudes([[2.5, 0.1, 0.7]], sig)
    c = M.mge_amplitudes([[1.0, 0.1, 0.7], [2.5, 0.1, 0.7]], sig)
    # exact up to the rounding of the Euler sum, whose terms cancel strongly
    tol = 1e-10 * float(torch.max(torch.abs(a)))
    assert torch.allclose(b, 2.5 * a, rtol=1e-13, atol=2.5 * tol)
    assert torch.allclose(c, 3.5 * a, rtol=1e-13, atol=3.5 * tol)


def test_gradient_central_differences():
    sig = M.sigma_grid(0.01, 20.0, 21)
    comp0 = np.array([[1.3, 0.08, 0.5], [-0.7, 1.5, 0.5], [0.2, 0.02, 0.9]])
    cot = np.random.default_rng(2).standard_normal(len(sig))
    leaf = torch.tensor(comp0, dtype=torch.float64, requires_grad=True)
    L = torch.sum(M.mge_amplitudes(leaf, sig) * torch.as_tensor(cot))
    (g,) = torch.autograd.grad(L, [leaf])

    def Lf(c):
        return float(torch.sum(M.mge_amplitudes(c, sig) * torch.as_tensor(cot)))

    def d(i, j, h):
        cp, cm = comp0.copy(), comp0.copy()
        cp[i, j] += h
        cm[i, j] -= h
        return (Lf(cp) - Lf(cm)) / (2 * h)

    for i in range(comp0.shape[0]):
        for j in range(3):
            # Richardson-extrapolated central difference, O(h^4); the Euler sum
            # cancels strongly, so L carries ~1e-10 absolute rounding and the
            # step is kept large
            h = 1e-2 * max(abs(comp0[i, j]), 5e-2)
            fd = (4 * d(i, j, h / 2) - d(i, j, h)) / 3
            assert abs(float(g[i, j]) - fd) <= 1e-7 * abs(fd) + 2e-10 / h, (i, j, float(g[i, j]), fd)

"""Pins of the radial anisotropy profile oracle (Sect. 6, beta_ani(r)):
its limits, midpoint, constant case, step limit, monotonicity, and central
differences of its gradient; plus the identity that the JAM oracle fed the
sampled beta_k equals the JAM oracle fed the same numbers directly."""
import numpy as np
import torch

from oracle import anisotropy as A
from oracle import jam as ojam
from paper_2504_01302_amd import inputs


SIG = np.array([0.003, 0.02, 0.1, 0.5, 1.0, 2.0, 5.0, 30.0])


def test_midpoint_and_limits():
    b = A.beta_logistic(SIG, [-0.4, 0.3, 0.5, 2.0]).numpy()
    assert abs(b[3] - (-0.05)) < 1e-15                      # sigma = r_a: the mean
    assert abs(b[0] - (-0.4)) < 1e-4 and abs(b[-1] - 0.3) < 1e-3   # centre / outside
    assert np.all(np.diff(b) > 0)                            # monotone from beta_0 to beta_inf
    assert np.all((b > -0.4) & (b < 0.3))


def test_constant_when_limits_agree():
    b = A.beta_logistic(SIG, [0.17, 0.17, 0.8, 1.3]).numpy()
    assert np.all(b == 0.17)


def test_step_limit():
    b = A.beta_logistic(SIG, [-0.2, 0.4, 0.7, 200.0]).numpy()
    assert np.allclose(b, np.where(SIG < 0.7, -0.2, 0.4), rtol=0, atol=1e-15)


def test_closed_form_by_hand():
    # r_a = 1, alpha = 1: beta(sigma) = b0 + (binf - b0) sigma / (1 + sigma)
    b = A.beta_logistic([1.0, 3.0, 0.25], [0.1, 0.5, 1.0, 1.0]).numpy()
    assert np.allclose(b, [0.3, 0.1 + 0.4 * 0.75, 0.1 + 0.4 * 0.2], rtol=0, atol=1e-15)


def test_gradient_central_differences():
    p0 = np.array([-0.3, 0.35, 0.4, 1.7])
    cot = np.random.default_rng(4).standard_normal(len(SIG))
    leaf = torch.tensor(p0, requires_grad=True)
    (g,) = torch.autograd.grad(torch.sum(A.beta_logistic(SIG, leaf) * torch.as_tensor(cot)), [leaf])
    for i in range(4):
        h = 1e-5 * max(abs(p0[i]), 0.1)
        pp, pm = p0.copy(), p0.copy()
        pp[i] += h
        pm[i] -= h
        fd = float(torch.sum((A.beta_logistic(SIG, pp) - A.beta_logistic(SIG, pm)) * torch.as_tensor(cot))) / (2 * h)
        assert abs(float(g[i]) - fd) <= 1e-8 * max(1.0, abs(fd)), (i, float(g[i]), fd)


def test_sampled_profile_feeds_jam():
    g = inputs.small_geometry(seed=2, n_lum=4, n_mass=2, nx=6, ny=5, n_bins=3)
    p = inputs.small_params(g, seed=2)
    b = A.beta_logistic(g.lum_sigma, [-0.3, 0.4, float(np.median(g.lum_sigma)), 2.0]).numpy()
    V1 = ojam.vrms2(g, inputs.with_overrides(p, beta=b))
    V2 = ojam.vrms2(g, p, overrides=dict(beta=torch.as_tensor(b)))
    assert torch.equal(V1, V2)

"""Plain FP64 CPU oracle of a radially varying orbital anisotropy assigned to
the tracer Gaussians.

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU library; only
the test suite may import it.  It shares no code with the GPU path.

What is computed (paper Sect. 6: a radially varying beta_ani(r), tangential
near the black hole and radial further out, in place of the constant
anisotropy of its own code):

* The profile is a logistic function of log r,
      beta(r) = beta_0 + (beta_inf - beta_0) / (1 + (r_a / r)^alpha),
  with the central value beta_0, the outer value beta_inf, the transition
  radius r_a > 0 [arcsec] and the sharpness alpha > 0; beta(r_a) is the mean
  of the two limits.
* The Jeans solutions used here take a constant anisotropy per tracer
  Gaussian, so the profile is sampled once per Gaussian at its dispersion:
  beta_k = beta(sigma_k).  (Each Gaussian's light is concentrated around
  r ~ sigma_k; this is the standard way an MGE model carries a radial
  anisotropy profile.)

The paper names the profile's qualitative shape and its purpose only; the
functional form, its parameters and the sampling radius are the readings
stated above.
"""
from __future__ import annotations

import numpy as np
import torch

DT = torch.float64


def beta_logistic(sigma, prof):
    """beta_k = beta(sigma_k) for prof = (beta_0, beta_inf, r_a, alpha);
    torch float64 (autograd flows to prof)."""
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64))
    prof = torch.as_tensor(prof, dtype=DT)
    b0, binf, ra, alpha = prof[0], prof[1], prof[2], prof[3]
    x = torch.exp(alpha * torch.log(ra / s))          # (r_a / sigma)^alpha
    return b0 + (binf - b0) / (1.0 + x)

"""GPU adjoint against the FP64 oracle gradient (autograd of the oracle) and
against central differences of the GPU forward.

Tolerance (no gradient bar is fixed by the problem): per model the gradient
vector error ||g_gpu - g_ref|| <= 1e-4 ||g_ref||, and every component within
1e-3 relative or 1e-6 of the largest component.  The forward parity bar is
1e-5 per bin; one gradient component sums many signed forward terms, so it
keeps fewer significant digits.
"""
import numpy as np
import pytest
import torch

from oracle import jam as ojam
from paper_2504_01302_amd import binding, inputs

pytestmark = pytest.mark.gpu

KEYS = ("inc", "beta", "mass_scale", "m_bh", "lum_I0", "mass_S0")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _flat(d):
    return np.concatenate([np.atleast_1d(np.asarray(d[k], np.float64)) for k in KEYS])


def _check(gpu, ref, tag):
    a, b = _flat(gpu), _flat(ref)
    err = np.linalg.norm(a - b) / np.linalg.norm(b)
    comp = np.abs(a - b) <= np.maximum(1e-3 * np.abs(b), 1e-6 * np.max(np.abs(b)))
    print(f"{tag}: grad rel norm err {err:.3e}, components ok {comp.sum()}/{comp.size}")
    assert err <= 1e-4 and comp.all(), (tag, err, np.nonzero(~comp))


def _gpu_grads(ctx, w, cot, dev, with_forward=True):
    p = binding.pack_params(w, dev, amplitudes=True)
    V = None
    if with_forward:
        V, st = ctx.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"],
                               p["lum_I0"], p["mass_S0"])
    c = torch.as_tensor(np.concatenate(cot), device=dev)
    g = ctx.vjp(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"],
                p["mass_S0"], V, c)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}


def _split_grads(g, w):
    out = []
    lo = mo = 0
    for m, i in enumerate(w.geom_idx):
        G = w.geometries[i]
        out.append(dict(inc=g["inc"][m], mass_scale=g["mass_scale"][m], m_bh=g["m_bh"][m],
                        beta=g["beta"][lo:lo + G.n_lum], lum_I0=g["lum_I0"][lo:lo + G.n_lum],
                        mass_S0=g["mass_S0"][mo:mo + G.n_mass]))
        lo += G.n_lum
        mo += G.n_mass
    return out


@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("recompute", [False, True])
def test_vjp_small_vs_oracle(recompute, form):
    dev = _dev()
    g = inputs.small_geometry(seed=21, n_lum=4, n_mass=3, nx=8, ny=7, ss=2, psf_n=3, n_bins=4)
    p = inputs.small_params(g, seed=21)
    w = inputs.Workload("s", [g], np.zeros(1, np.int32), [p])
    cot = [np.random.default_rng(1).standard_normal(g.n_bins)]
    ctx = binding.Context([g], form=form)
    gg = _split_grads(_gpu_grads(ctx, w, cot, dev, with_forward=not recompute), w)[0]
    _, ref = ojam.vrms2_and_grad(g, p, cot[0])
    _check(gg, {k: v.numpy() for k, v in ref.items()}, f"small recompute={recompute} form={form}")
    ctx.close()


@pytest.mark.parametrize("form", [1, 2])
def test_vjp_cfg5_models_vs_oracle(form):
    dev = _dev()
    w = inputs.config5(n_models=8)
    cot = list(inputs.cotangent(w.geometries[0].n_bins, 8))
    ctx = binding.Context(w.geometries, form=form)
    gs = _split_grads(_gpu_grads(ctx, w, cot, dev), w)
    for m in (0, 3, 7):
        _, ref = ojam.vrms2_and_grad(w.geometries[0], w.params[m], cot[m])
        _check(gs[m], {k: v.numpy() for k, v in ref.items()}, f"cfg5 model {m} form={form}")
    ctx.close()


def test_vjp_larger_map_mfma_vs_oracle():
    """A map with several 32-row x tiles and y chunks of the MFMA adjoint."""
    dev = _dev()
    g = inputs.small_geometry(seed=22, n_lum=2, n_mass=2, nx=70, ny=45, ss=2, psf_n=3,
                              n_bins=5, n_u=12, pixsize=0.02)
    p = inputs.small_params(g, seed=22)
    w = inputs.Workload("L", [g], np.zeros(1, np.int32), [p])
    cot = [np.random.default_rng(2).standard_normal(g.n_bins)]
    ctx = binding.Context([g], form=2)
    gg = _split_grads(_gpu_grads(ctx, w, cot, dev), w)[0]
    _, ref = ojam.vrms2_and_grad(g, p, cot[0])
    _check(gg, {k: v.numpy() for k, v in ref.items()}, "larger map form=2")
    ctx.close()


def test_vjp_vs_gpu_central_differences():
    """Directional derivative of the GPU forward along a random direction in
    (inc, beta, mass_scale) vs the GPU adjoint's inner product."""
    dev = _dev()
    w = inputs.config1()
    g0 = w.geometries[0]
    p0 = w.params[0]
    cot = inputs.cotangent(g0.n_bins, 1)[0]
    ctx = binding.Context(w.geometries)
    gr = _split_grads(_gpu_grads(ctx, w, [cot], dev), w)[0]
    rng = np.random.default_rng(5)
    d_inc, d_ml = rng.standard_normal(2)
    d_beta = rng.standard_normal(g0.n_lum)

    def L(eps):
        pp = inputs.with_overrides(p0, inc=p0.inc + eps * d_inc * 1e-2,
                                   mass_scale=p0.mass_scale + eps * d_ml * 1e-2,
                                   beta=p0.beta + eps * d_beta * 1e-2)
        ww = inputs.Workload("fd", w.geometries, w.geom_idx, [pp])
        q = binding.pack_params(ww, dev)
        V, _ = ctx.eval_batch(ww.geom_idx, q["inc"], q["mass_scale"], q["m_bh"], q["beta"])
        return float(np.sum(V.cpu().numpy() * cot))

    h = 1e-2
    fd = (8 * (L(h) - L(-h)) - (L(2 * h) - L(-2 * h))) / (12 * h)
    ad = 1e-2 * (gr["inc"] * d_inc + gr["mass_scale"] * d_ml + np.dot(gr["beta"], d_beta))
    scale = float(np.sum(np.abs(cot) * 1e5))
    print(f"directional: adjoint {ad:.6e} fd {fd:.6e}")
    assert abs(ad - fd) <= 1e-3 * abs(fd) + 1e-7 * scale
    ctx.close()


def test_autograd_function_matches_vjp_and_oracle():
    from paper_2504_01302_amd.autograd import jam_vrms2
    dev = _dev()
    w = inputs.config5(n_models=3)
    cot = inputs.cotangent(w.geometries[0].n_bins, 3)
    ctx = binding.Context(w.geometries, form=2)
    p = binding.pack_params(w, dev, amplitudes=True)
    leaves = {k: p[k].clone().requires_grad_(True) for k in KEYS}
    V, st = jam_vrms2(ctx, w.geom_idx, leaves["inc"], leaves["mass_scale"], leaves["m_bh"],
                      leaves["beta"], leaves["lum_I0"], leaves["mass_S0"])
    L = torch.sum(V * torch.as_tensor(cot.reshape(-1), device=dev))
    L.backward()
    got = {k: leaves[k].grad.cpu().numpy() for k in KEYS}
    gs = _split_grads(got, w)
    _, ref = ojam.vrms2_and_grad(w.geometries[0], w.params[1], cot[1])
    _check(gs[1], {k: v.numpy() for k, v in ref.items()}, "autograd model 1")
    ctx.close()

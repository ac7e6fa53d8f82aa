"""GPU goodness of fit, eq. (chi2_dyn), against the FP64 oracle.

* The chi^2 kernel alone, fed the oracle's own binned moments: both sides are
  FP64 (a Cholesky inverse and matrix-vector product on the GPU, a general
  solve in the oracle), so they agree to 1e-11 relative.
* The fused forward + chi^2: the moments carry the forward's <= 1e-5 per-bin
  error, so v_pre = sqrt(V) carries <= 0.5e-5 relative and chi^2 moves by at
  most 2 sum_b |(cov^-1 r)_b| dv_b; the test allows that bound (first order)
  plus 1e-9 relative.
* The chi^2 adjoint against the oracle's autograd gradient, with the
  tolerance of the v_rms^2 adjoint (vector 1e-4, components 1e-3 relative or
  1e-6 of the largest).
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


def _near_fit_data(g, p, seed):
    """Observations within ~5 % of the model (oracle moments) and a
    covariance built like the synthetic kinematics' (5 % per bin, 2 % shared)."""
    V = ojam.vrms2(g, p).numpy()
    rng = np.random.default_rng(seed)
    vo = np.sqrt(V) * (1.0 + 0.05 * rng.standard_normal(g.n_bins))
    cov = np.diag((0.05 * vo) ** 2) + 0.02 ** 2 * np.outer(vo, vo)
    return V, vo, cov


def _oracle_s(V, vo, cov):
    r = vo - np.sqrt(V)
    return np.linalg.solve(cov, r), r


def test_chi2_kernel_on_oracle_moments():
    dev = _dev()
    w = inputs.config3(n_models=6)
    g = w.geometries[0]
    vo, cov = inputs.kinematic_data(g.n_bins, seed=1)
    ctx = binding.Context(w.geometries)
    ctx.set_kinematics(0, vo, cov)
    Vs = [ojam.vrms2(g, p).numpy() for p in w.params]
    V = torch.as_tensor(np.concatenate(Vs), device=dev)
    c2, d = ctx.chi2(w.geom_idx, V, want_grad=True)
    torch.cuda.synchronize()
    c2, d = c2.cpu().numpy(), d.cpu().numpy().reshape(len(Vs), -1)
    for m, Vm in enumerate(Vs):
        ref = float(ojam.chi2_dyn(Vm, vo, cov))
        Vt = torch.as_tensor(Vm, dtype=torch.float64).requires_grad_(True)
        (dref,) = torch.autograd.grad(ojam.chi2_dyn(Vt, vo, cov), [Vt])
        print(f"model {m}: chi2 {c2[m]:.10e} oracle {ref:.10e}")
        assert abs(c2[m] - ref) <= 1e-11 * abs(ref)
        assert np.allclose(d[m], dref.numpy(), rtol=1e-10, atol=1e-14 * np.max(np.abs(dref.numpy())))
    ctx.close()


def test_eval_chi2_vs_oracle_and_unfused():
    dev = _dev()
    w = inputs.config3(n_models=8)
    g = w.geometries[0]
    ctx = binding.Context(w.geometries)
    p0 = w.params[0]
    V0, vo, cov = _near_fit_data(g, p0, seed=2)
    ctx.set_kinematics(0, vo, cov)
    p = binding.pack_params(w, dev)
    c2, Vk, st = ctx.eval_chi2(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"],
                               keep_vrms2=True)
    V, st2 = ctx.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"])
    c2u, _ = ctx.chi2(w.geom_idx, V)
    torch.cuda.synchronize()
    assert torch.equal(Vk, V) and torch.equal(c2, c2u), "fused and unfused differ"
    assert torch.all(st == 0)
    c2 = c2.cpu().numpy()
    for m in (0, 3, 7):
        Vm = V0 if m == 0 else ojam.vrms2(g, w.params[m]).numpy()
        ref = float(ojam.chi2_dyn(Vm, vo, cov))
        s, _ = _oracle_s(Vm, vo, cov)
        tol = 1e-5 * float(np.sum(np.abs(s) * np.sqrt(Vm))) + 1e-9 * abs(ref)
        print(f"model {m}: chi2 {c2[m]:.8e} oracle {ref:.8e} |diff| {abs(c2[m]-ref):.2e} tol {tol:.2e}")
        assert abs(c2[m] - ref) <= tol
    ctx.close()


def _split(g, w):
    out, lo, mo = [], 0, 0
    for m, i in enumerate(w.geom_idx):
        G = w.geometries[i]
        out.append(dict(inc=g["inc"][m], mass_scale=g["mass_scale"][m], m_bh=g["m_bh"][m],
                        beta=g["beta"][lo:lo + G.n_lum], lum_I0=g["lum_I0"][lo:lo + G.n_lum],
                        mass_S0=g["mass_S0"][mo:mo + G.n_mass]))
        lo += G.n_lum
        mo += G.n_mass
    return out


def _check(gpu, ref, tag):
    a = np.concatenate([np.atleast_1d(np.asarray(gpu[k], np.float64)) for k in KEYS])
    b = np.concatenate([np.atleast_1d(np.asarray(ref[k], np.float64)) for k in KEYS])
    err = np.linalg.norm(a - b) / np.linalg.norm(b)
    comp = np.abs(a - b) <= np.maximum(1e-3 * np.abs(b), 1e-6 * np.max(np.abs(b)))
    print(f"{tag}: grad rel norm err {err:.3e}, components ok {comp.sum()}/{comp.size}")
    assert err <= 1e-4 and comp.all(), (tag, err, np.nonzero(~comp))


@pytest.mark.parametrize("form", [1, 2])
def test_vjp_chi2_vs_oracle(form):
    dev = _dev()
    w = inputs.config5(n_models=4)
    g = w.geometries[0]
    ctx = binding.Context(w.geometries, form=form)
    _, vo, cov = _near_fit_data(g, w.params[1], seed=3)
    ctx.set_kinematics(0, vo, cov)
    p = binding.pack_params(w, dev, amplitudes=True)
    cot = torch.as_tensor([1.0, -0.5, 2.0, 0.25], dtype=torch.float64, device=dev)
    gr = ctx.vjp_chi2(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"],
                      p["mass_S0"], cot)
    # the same with the forward output handed over instead of recomputed
    _, V, _ = ctx.eval_chi2(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"],
                            p["lum_I0"], p["mass_S0"], keep_vrms2=True)
    gv = ctx.vjp_chi2(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"],
                      p["mass_S0"], cot, vrms2=V)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(gr[k], gv[k]), k
    gs = _split({k: v.cpu().numpy() for k, v in gr.items()}, w)
    for m in (1, 2):
        _, ref = ojam.chi2_and_grad(g, w.params[m], vo, cov)
        ref = {k: float(cot[m]) * v.numpy() for k, v in ref.items()}
        _check(gs[m], ref, f"chi2 adjoint model {m} form {form}")
    ctx.close()


def test_autograd_chi2_matches_vjp():
    from paper_2504_01302_amd.autograd import jam_chi2
    dev = _dev()
    w = inputs.config5(n_models=3)
    g = w.geometries[0]
    ctx = binding.Context(w.geometries)
    _, vo, cov = _near_fit_data(g, w.params[0], seed=4)
    ctx.set_kinematics(0, vo, cov)
    p = binding.pack_params(w, dev, amplitudes=True)
    leaves = {k: p[k].clone().requires_grad_(True) for k in KEYS}
    c2, st = jam_chi2(ctx, w.geom_idx, leaves["inc"], leaves["mass_scale"], leaves["m_bh"],
                      leaves["beta"], leaves["lum_I0"], leaves["mass_S0"])
    torch.sum(c2).backward()
    ones = torch.ones(3, dtype=torch.float64, device=dev)
    gr = ctx.vjp_chi2(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"],
                      p["mass_S0"], ones)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(leaves[k].grad, gr[k]), k
    _, ref = ojam.chi2_and_grad(g, w.params[2], vo, cov)
    _check(_split({k: v.cpu().numpy() for k, v in gr.items()}, w)[2],
           {k: v.numpy() for k, v in ref.items()}, "autograd chi2 model 2")
    ctx.close()


def test_chi2_invalid_model_and_mixed_geometries():
    dev = _dev()
    ga = inputs.small_geometry(seed=31, n_lum=3, n_mass=2, nx=8, ny=6, psf_n=3, n_bins=4)
    gb = inputs.small_geometry(seed=32, n_lum=2, n_mass=3, nx=5, ny=9, psf_n=3, n_bins=6)
    pa, pb = inputs.small_params(ga, seed=31), inputs.small_params(gb, seed=32)
    bad = inputs.with_overrides(pa, inc=0.05)          # cannot be deprojected
    w = inputs.Workload("mix", [ga, gb], np.array([0, 1, 0], np.int32), [pa, pb, bad])
    ctx = binding.Context(w.geometries)
    kin = [inputs.kinematic_data(ga.n_bins, 5), inputs.kinematic_data(gb.n_bins, 6)]
    for i, (v, c) in enumerate(kin):
        ctx.set_kinematics(i, v, c)
    p = binding.pack_params(w, dev)
    c2, _, st = ctx.eval_chi2(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"])
    torch.cuda.synchronize()
    c2, st = c2.cpu().numpy(), st.cpu().numpy()
    assert st[0] == 0 and st[1] == 0 and st[2] != 0
    assert np.isnan(c2[2]) and np.isfinite(c2[:2]).all()
    for m, (G, P) in enumerate([(ga, pa), (gb, pb)]):
        ref = float(ojam.chi2_dyn(ojam.vrms2(G, P), *kin[m]))
        assert abs(c2[m] - ref) <= 1e-4 * abs(ref)
    ctx.close()


def test_chi2_argument_errors():
    _dev()
    g = inputs.small_geometry(seed=33, n_bins=3)
    ctx = binding.Context([g])
    v, cov = inputs.kinematic_data(3, 7)
    with pytest.raises(binding.JamError) as e:
        ctx.set_kinematics(0, v, -cov)                      # not positive definite
    assert e.value.status == 1
    asym = cov.copy()
    asym[0, 1] += 1.0
    with pytest.raises(binding.JamError):
        ctx.set_kinematics(0, v, asym)
    with pytest.raises(binding.JamError):
        ctx.set_kinematics(1, v, cov)                       # no such geometry
    p = binding.pack_params(inputs.Workload("e", [g], np.zeros(1, np.int32),
                                            [inputs.small_params(g, 33)]), "cuda")
    with pytest.raises(binding.JamError):                   # kinematics not set yet
        ctx.eval_chi2(np.zeros(1, np.int32), p["inc"], p["mass_scale"], p["m_bh"], p["beta"])
    ctx.set_kinematics(0, v, cov)
    c2, _, _ = ctx.eval_chi2(np.zeros(1, np.int32), p["inc"], p["mass_scale"], p["m_bh"],
                             p["beta"])
    torch.cuda.synchronize()
    assert np.isfinite(c2.cpu().numpy()).all()
    ctx.close()


def test_chi2_graph_replays_match_eager():
    dev = _dev()
    w = inputs.config3(n_models=16)
    g = w.geometries[0]
    vo, cov = inputs.kinematic_data(g.n_bins, seed=9)
    eager = binding.Context(w.geometries)
    graph = binding.Context(w.geometries, graph=1)
    for c in (eager, graph):
        c.set_kinematics(0, vo, cov)
    p = binding.pack_params(w, dev, amplitudes=True)
    args = (w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"], p["mass_S0"])
    ref, _, _ = eager.eval_chi2(*args)
    cot = torch.linspace(-1.0, 1.0, 16, dtype=torch.float64, device=dev)
    gref = eager.vjp_chi2(*args, cot)
    torch.cuda.synchronize()
    for rep in range(3):
        c2, _, _ = graph.eval_chi2(*args)
        gg = graph.vjp_chi2(*args, cot)
        torch.cuda.synchronize()
        assert torch.equal(c2, ref), rep
        for k in KEYS:
            assert torch.equal(gg[k], gref[k]), (rep, k)
        _ = eager.eval_batch(*args)                         # eager work between replays
        torch.cuda.synchronize()
    eager.close()
    graph.close()

"""GPU runtime features: persistent work-queue launches, HIP-graph replay and
the autotuner.  Each is checked against the plain eager evaluation (bitwise
where the arithmetic is the same) and against the FP64 oracle."""
import os

import numpy as np
import pytest
import torch

from oracle import jam as ojam
from paper_2504_01302_amd import binding, inputs

pytestmark = pytest.mark.gpu

RTOL = 1e-5


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _uneven(n=24, seed=0):
    """Small uneven batch: different MGE sizes, grids, node and bin counts."""
    rng = np.random.default_rng(seed)
    gs = []
    for i in range(6):
        gs.append(inputs.small_geometry(seed=40 + i, n_lum=int(rng.integers(2, 6)),
                                        n_mass=int(rng.integers(1, 6)),
                                        nx=int(rng.integers(5, 60)), ny=int(rng.integers(5, 60)),
                                        ss=int(rng.integers(1, 3)), psf_n=3,
                                        n_bins=int(rng.integers(2, 8)),
                                        n_u=int(rng.integers(8, 40)), pixsize=0.03))
    gi = rng.integers(0, len(gs), n).astype(np.int32)
    ps = [inputs.small_params(gs[i], seed=100 + m) for m, i in enumerate(gi)]
    return inputs.Workload("uneven", gs, gi, ps)


def _eval(ctx, w, p):
    V, st = ctx.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"],
                           p["lum_I0"], p["mass_S0"])
    torch.cuda.synchronize()
    return V.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("form", [1, 2])
def test_persistent_equals_one_workgroup_per_item(form):
    dev = _dev()
    w = _uneven()
    p = binding.pack_params(w, dev)
    a = binding.Context(w.geometries, form=form, launch=1)    # persistent queue
    b = binding.Context(w.geometries, form=form, launch=0)    # one worker per item
    Va, sa = _eval(a, w, p)
    Vb, sb = _eval(b, w, p)
    assert np.all(sa == 0) and np.array_equal(Va, Vb)
    ia, ib = a.plan_info(w.geom_idx), b.plan_info(w.geom_idx)
    # one workgroup per item, or a persistent grid of at most as many
    assert ia["num_grid"] <= ia["num_items"] and ib["num_grid"] == ib["num_items"]
    o = np.cumsum([0] + [w.geometries[i].n_bins for i in w.geom_idx])
    for m in (0, 7, 23):
        ref = ojam.vrms2(w.geometries[w.geom_idx[m]], w.params[m]).numpy()
        assert np.max(np.abs(Va[o[m]:o[m + 1]] / ref - 1)) <= RTOL
    a.close()
    b.close()


def test_graph_replay_matches_eager():
    dev = _dev()
    w = inputs.config3(n_models=64)
    p = binding.pack_params(w, dev)
    eager = binding.Context(w.geometries, form=2)
    Ve, _ = _eval(eager, w, p)
    g = binding.Context(w.geometries, form=2, graph=1)
    nb, _, _ = g.sizes(w.geom_idx)
    out = torch.empty(nb, dtype=torch.float64, device=dev)
    st = torch.empty(64, dtype=torch.int32, device=dev)
    for rep in range(4):
        out.fill_(-1.0)
        g.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], out=out,
                     status=st)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), Ve), rep
        # eager work of the program between replays
        _ = eager.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"])
        torch.cuda.synchronize()
    # new parameter values in the same buffers are picked up by the replay
    p["inc"].copy_(torch.as_tensor(np.full(64, np.deg2rad(80.0)), device=dev))
    g.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], out=out, status=st)
    torch.cuda.synchronize()
    pm = inputs.with_overrides(w.params[5], inc=np.deg2rad(80.0))
    ref = ojam.vrms2(w.geometries[0], pm).numpy()
    nb0 = w.geometries[0].n_bins
    assert np.max(np.abs(out.cpu().numpy()[5 * nb0:6 * nb0] / ref - 1)) <= RTOL
    eager.close()
    g.close()


def test_graph_replay_vjp_matches_eager():
    dev = _dev()
    w = inputs.config5(n_models=16)
    p = binding.pack_params(w, dev, amplitudes=True)
    cot = torch.as_tensor(inputs.cotangent(w.geometries[0].n_bins, 16).reshape(-1), device=dev)
    eager = binding.Context(w.geometries, form=2)
    V, _ = eager.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"],
                            p["lum_I0"], p["mass_S0"])
    ge = eager.vjp(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"],
                   p["mass_S0"], V, cot)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ge.items()}
    g = binding.Context(w.geometries, form=2, graph=1)
    for rep in range(3):
        gg = g.vjp(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"],
                   p["mass_S0"], V, cot)
        torch.cuda.synchronize()
        for k in ref:
            assert np.array_equal(gg[k].cpu().numpy(), ref[k]), (rep, k)
    eager.close()
    g.close()


def test_graph_replay_vjp_alternating_gradient_buffers():
    # The recorded adjoint writes into the gradient buffers it was recorded
    # with; calls that alternate between buffer sets, including a set with
    # two buffers swapped, must each fill exactly the buffers they pass.
    dev = _dev()
    n = 8
    w = inputs.config5(n_models=n)
    p = binding.pack_params(w, dev, amplitudes=True)
    cot = torch.as_tensor(inputs.cotangent(w.geometries[0].n_bins, n).reshape(-1), device=dev)
    eager = binding.Context(w.geometries, form=2)
    V, _ = eager.eval_batch(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"],
                            p["lum_I0"], p["mass_S0"])
    ge = eager.vjp(w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"], p["beta"], p["lum_I0"],
                   p["mass_S0"], V, cot)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ge.items()}
    keys = ("inc", "mass_scale", "m_bh", "beta", "lum_I0", "mass_S0")
    g = binding.Context(w.geometries, form=2, graph=1)
    ws = g.workspace(w.geom_idx, True, dev)
    s = torch.cuda.current_stream(dev).cuda_stream

    def bufs():
        return {k: torch.empty_like(ge[k]) for k in keys}

    A, B = bufs(), bufs()
    # set C: A's buffers with inc <-> mass_scale and beta <-> lum_I0 swapped
    C = dict(A, inc=A["mass_scale"], mass_scale=A["inc"], beta=A["lum_I0"], lum_I0=A["beta"])
    for rep in range(2):
        for name, S in (("A", A), ("B", B), ("C", C), ("A", A)):
            for t in list(A.values()) + list(B.values()):
                t.fill_(float("nan"))
            binding.jam_vjp(g.handle, w.geom_idx, p["inc"], p["mass_scale"], p["m_bh"],
                            p["beta"], p["lum_I0"], p["mass_S0"], V, cot, S["inc"],
                            S["mass_scale"], S["m_bh"], S["beta"], S["lum_I0"], S["mass_S0"],
                            ws, s)
            torch.cuda.synchronize()
            for k in keys:
                assert np.array_equal(S[k].cpu().numpy(), ref[k]), (rep, name, k)
            other = B if S is not B else A
            for k in keys:
                assert np.all(np.isnan(other[k].cpu().numpy())), (rep, name, k)
    eager.close()
    g.close()


def test_autotuner_and_cache_file(tmp_path):
    dev = _dev()
    w = _uneven(n=16, seed=3)
    p = binding.pack_params(w, dev)
    cache = str(tmp_path / "tune.txt")
    a = binding.Context(w.geometries, form=0, autotune=1, tune_cache=cache)
    Va, sa = _eval(a, w, p)
    info = a.plan_info(w.geom_idx)
    assert os.path.exists(cache)
    text = open(cache).read().split()
    assert len(text) == 5 and int(text[1]) == info["rule"] and int(text[3]) == info["gran"]
    o = np.cumsum([0] + [w.geometries[i].n_bins for i in w.geom_idx])
    for m in range(0, 16, 5):
        ref = ojam.vrms2(w.geometries[w.geom_idx[m]], w.params[m]).numpy()
        assert np.max(np.abs(Va[o[m]:o[m + 1]] / ref - 1)) <= RTOL
    # a second context reads the cached choice instead of tuning again
    mtime = os.path.getmtime(cache)
    b = binding.Context(w.geometries, form=0, autotune=1, tune_cache=cache)
    assert b.plan_info(w.geom_idx) == info
    assert os.path.getmtime(cache) == mtime
    a.close()
    b.close()

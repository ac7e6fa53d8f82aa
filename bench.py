"""Benchmark of the JAM-cyl hot path on one MI355X.

Workload: the IFU-scale model (40 luminous x 40 mass Gaussians + BH, 200x200
pixels at 0.025" with 2x supersampling, 128 u-nodes, 31x31 PSF, 60 bins),
synthetic and seeded.  A forward step is one jam_eval_batch of that model; a
fwd+bwd step adds one jam_vjp (the full adjoint).  By default the timed calls
replay HIP graphs the library recorded at their first call (the same kernels,
without per-launch gaps); per-kernel timings come from an eager loop.  Inputs
are resident in HBM before timing starts.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form 0|1|2]
                    [--batch N] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12     # MI355X published FP32 vector FLOP/s
FP32_MFMA_PEAK = 157.3e12       # MI355X published dense FP32 matrix FLOP/s
# FP32 flops per integrand of the per-pixel form: y^2 scale (1 mul), exponent
# argument (1 fma), polynomial (1 fma), accumulate (1 fma) = 7 flops, plus
# one exp2 counted separately.
PIX_FLOPS_PER_INTEGRAND = 7


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--form", type=int, default=2,
                    help="1 per-pixel VALU kernel, 2 matrix-core kernel (0 = library default)")
    ap.add_argument("--launch", type=int, default=0,
                    help="0 one worker per work item, 1 persistent work-queue grid")
    ap.add_argument("--graph", type=int, default=1,
                    help="1 (default) time the headline loops as replays of a recorded HIP "
                         "graph; the kernel timings behind the roofline always come from an "
                         "eager loop of the same model")
    ap.add_argument("--autotune", type=int, default=0, help="1 autotune the numerator schedule")
    ap.add_argument("--no-plain-baseline", action="store_true",
                    help="skip timing the plain per-model forward (per-pixel VALU kernel, "
                         "one workgroup per item, no graph)")
    ap.add_argument("--batch", type=int, default=1,
                    help="models per launch (copies of the IFU-scale model)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched workloads (4096 proposals on the small geometry, "
                         "1024 uneven models), reported under 'extra'")
    ap.add_argument("--extra", default="",
                    help="comma-separated names of the extra workloads to run (default all)")
    ap.add_argument("--only-extra", action="store_true",
                    help="run only the extra workloads (for profiling one of them); the "
                         "JSON line then carries no headline value")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy three times, the reference "
                         "kernel for scaling the HBM byte counters of a profile")
    ap.add_argument("--cpu-sample", type=int, default=16384,
                    help="padded sub-pixels the oracle evaluates for the CPU baseline")
    return ap.parse_args()


def cpu_baseline(g, p, n_sample):
    """The FP64 oracle, as it stands, on a bounded sample of the same model:
    the line-of-sight numerator at n_sample seeded padded sub-pixels, scaled
    to the full padded grid (the PSF and bin sums cost a negligible extra)."""
    import torch
    from oracle import jam as ojam
    x, y, _ = ojam.padded_subgrid(g)
    rng = np.random.default_rng(7)
    ix = rng.integers(0, len(x), n_sample)
    iy = rng.integers(0, len(y), n_sample)
    t0 = time.perf_counter()
    ojam.point_values(g, p, x[ix], y[iy])
    dt = time.perf_counter() - t0
    per_model = dt * (len(x) * len(y)) / n_sample
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f
                              if ln.startswith("model name")), None)
    except OSError:
        pass
    # a whole model end to end (every padded sub-pixel, PSF, all bins) on
    # the small geometry, beside the sampled IFU-scale figure
    from paper_2504_01302_amd import inputs
    w1 = inputs.config1()
    t0 = time.perf_counter()
    ojam.vrms2(w1.geometries[0], w1.params[0])
    dt1 = time.perf_counter() - t0
    return dict(value=1.0 / per_model, unit="models/s", cores=torch.get_num_threads(),
                kind="oracle", cpu_model=cpu_model, nproc=os.cpu_count(),
                affinity=len(os.sched_getaffinity(0)),
                sample=f"N and I at {n_sample} of {len(x) * len(y)} padded sub-pixels of the "
                       f"IFU-scale model ({dt:.1f} s), scaled to one model; the oracle evaluates "
                       f"every padded sub-pixel, i.e. all four mirror copies that the GPU "
                       f"evaluates once",
                whole_model_small_geometry={
                    "seconds": dt1, "models_per_s": 1.0 / dt1,
                    "workload": "oracle vrms2 end to end (30x30 px, 9x9 PSF, 20 bins, 10 x 12 "
                                "Gaussians + BH, 100 u-nodes), one model"})


def profiled_traffic(kernel):
    """HBM bytes per launch of the quadrature kernel on the IFU-scale model
    from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None
    when the kernel source has changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_ifu_scale_hbm.md")
    src = os.path.join(ROOT, "paper_2504_01302_amd", "csrc", "jam_kernels.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"Kernel source sha256: ([0-9a-f]{64})", text)
    b = re.search(kernel + r"_traffic_bytes_per_launch: ([0-9.]+)", text)
    if not h or not b:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != h.group(1):
        return None
    return float(b.group(1))


KERNEL_NAMES = {0: "k_num_pix", 1: "k_num_mfma", 2: "k_num_map", 3: "k_sph_moments"}


def unique_units(g):
    """Unique pixels (distinct |x'| x distinct |y'| of the padded sub-pixel
    grid, the map the kernels evaluate) times terms K (J + 1) n_u."""
    def distinct(n, c):
        v = (np.arange(n * g.supersample + g.psf_n - 1) - (n * g.supersample + g.psf_n - 2) / 2.0)
        return len(set(np.abs(c + v * (g.pixsize / g.supersample)).round(12)))
    n_pix = distinct(g.nx, g.xc) * distinct(g.ny, g.yc)
    return n_pix * g.n_lum * (g.n_mass + 1) * g.n_u


def roofline_fracs(w, ms_fwd, ms_fb, num_ms=None, sens_ms=None):
    """Fractions of the FP32 matrix-core peak at the algorithmic flop counts
    per (unique pixel, term): 2 for the forward quadrature (N = A B^T), 4 for
    the adjoint's two contractions, 6 for a forward + adjoint step."""
    units = float(sum(unique_units(w.geometries[i]) for i in w.geom_idx))
    out = {"units": units,
           "forward_frac": 2 * units / (ms_fwd * 1e-3) / FP32_MFMA_PEAK,
           "fwd_bwd_frac": 6 * units / (ms_fb * 1e-3) / FP32_MFMA_PEAK}
    if num_ms:
        out["numerator_kernel_ms"] = num_ms
        out["numerator_kernel_frac"] = 2 * units / (num_ms * 1e-3) / FP32_MFMA_PEAK
    if sens_ms:
        out["adjoint_kernel_ms"] = sens_ms
        out["adjoint_kernel_frac"] = 4 * units / (sens_ms * 1e-3) / FP32_MFMA_PEAK
    return out


def time_batch(torch, binding, w, dev, steps, form, launch, graph, autotune=0):
    """Forward and forward+adjoint throughput of one whole batch per launch
    (with autotune, the schedule search runs at the first call, untimed),
    and the quadrature and adjoint kernels' average durations from an eager
    loop of the same batch."""
    ctx = binding.Context(w.geometries, form=form, launch=launch, graph=graph, autotune=autotune)
    par = binding.pack_params(w, dev, amplitudes=True)
    nb, _, _ = ctx.sizes(w.geom_idx)
    V = torch.empty(nb, dtype=torch.float64, device=dev)
    st = torch.empty(len(w.geom_idx), dtype=torch.int32, device=dev)
    cot = torch.ones(nb, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def fwd():
        ctx.eval_batch(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                       par["lum_I0"], par["mass_S0"], out=V, status=st)

    def bwd():
        ctx.vjp(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                par["lum_I0"], par["mass_S0"], V, cot)

    fwd()
    bwd()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fwd()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(steps):
        fwd()
        bwd()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fb = e0.elapsed_time(e1) / steps
    n = len(w.geom_idx)
    ok = bool((st == 0).all().item())
    sched = ctx.plan_info(w.geom_idx)
    ctx.close()
    # kernel durations from eager launches (graph replays are not bracketed)
    ek = binding.Context(w.geometries, form=form, launch=launch, graph=0, autotune=autotune)

    def efwd():
        ek.eval_batch(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                      par["lum_I0"], par["mass_S0"], out=V, status=st)

    efwd()
    ek.vjp(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
           par["lum_I0"], par["mass_S0"], V, cot)
    torch.cuda.synchronize()
    binding.jam_timing(ek.handle, True)
    for _ in range(max(2, steps // 2)):
        efwd()
        ek.vjp(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
               par["lum_I0"], par["mass_S0"], V, cot)
    num_ms, num_n, sens_ms, sens_n = binding.jam_timing(ek.handle, False)
    ek.close()
    rec = {"models": n, "ms_forward": ms_f, "models_per_s": n * 1000.0 / ms_f,
           "ms_fwd_bwd": ms_fb, "fwd_bwd_per_s": n * 1000.0 / ms_fb, "all_status_ok": ok,
           "schedule": sched, "numerator_kernel": KERNEL_NAMES.get(sched.get("num_kernel"))}
    rec["roofline"] = roofline_fracs(w, ms_f, ms_fb, num_ms / max(1, num_n),
                                     sens_ms / max(1, sens_n))
    return rec


def time_spherical(torch, binding, w, dev, steps, backward=True, form=0, values=None):
    """Forward and forward+adjoint throughput of the spherically aligned
    model (eqs. J1, J2) on one whole batch per launch; form 0: the forward
    interpolates the potential sums from their grid, form 1: it sums the
    terms at every characteristic node.  With a list `values`, the forward's
    v_rms^2 is appended to it."""
    ctx = binding.Context(w.geometries, alignment=1, form=form)
    par = binding.pack_params(w, dev, amplitudes=True)
    nb, _, _ = ctx.sizes(w.geom_idx)
    V = torch.empty(nb, dtype=torch.float64, device=dev)
    st = torch.empty(len(w.geom_idx), dtype=torch.int32, device=dev)
    cot = torch.ones(nb, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def fwd():
        ctx.eval_batch(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                       par["lum_I0"], par["mass_S0"], out=V, status=st)

    def bwd():
        return ctx.vjp(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                       par["lum_I0"], par["mass_S0"], V, cot)

    fwd()
    if backward:
        g = bwd()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fwd()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1) / steps
    n = len(w.geom_idx)
    rec = {"models": n, "ms_forward": ms_f, "models_per_s": n * 1000.0 / ms_f}
    if backward:
        e0.record(stream)
        for _ in range(steps):
            fwd()
            g = bwd()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_fb = e0.elapsed_time(e1) / steps
        rec.update(ms_fwd_bwd=ms_fb, fwd_bwd_per_s=n * 1000.0 / ms_fb,
                   grads_finite=bool(torch.isfinite(g["inc"]).all().item()))
    rec["all_status_ok"] = bool((st == 0).all().item())
    if values is not None:
        values.append(V.cpu().numpy())
    ctx.close()
    return rec


def time_spherical_both(torch, binding, w, dev, steps, backward=True):
    """time_spherical with the potential grid, plus the direct-sum forward's
    time and the largest relative difference of the two forwards."""
    vals = []
    rec = time_spherical(torch, binding, w, dev, steps, backward, 0, vals)
    d = time_spherical(torch, binding, w, dev, steps, False, 1, vals)
    rec["direct_sums"] = {"ms_forward": d["ms_forward"], "models_per_s": d["models_per_s"],
                          "max_rel_diff_grid_vs_direct":
                              float(np.max(np.abs(vals[0] / vals[1] - 1.0)))}
    return rec


def time_chi2(torch, binding, w, dev, steps, form, launch, graph):
    """chi^2 per proposal (eq. chi2_dyn) fused after the forward, and its
    adjoint, for a whole batch per launch (one scalar and one gradient per
    proposal for a gradient sampler)."""
    from paper_2504_01302_amd import inputs
    ctx = binding.Context(w.geometries, form=form, launch=launch, graph=graph)
    for gi, g in enumerate(w.geometries):
        ctx.set_kinematics(gi, *inputs.kinematic_data(g.n_bins, seed=gi))
    par = binding.pack_params(w, dev, amplitudes=True)
    n = len(w.geom_idx)
    cot = torch.ones(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    args = (w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"], par["lum_I0"],
            par["mass_S0"])

    state = {}

    def fwd():
        state["out"] = ctx.eval_chi2(*args, keep_vrms2=True)
        return state["out"]

    def bwd():
        ctx.vjp_chi2(*args, cot, vrms2=state["out"][1])

    c2, _, st = fwd()
    bwd()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fwd()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(steps):
        fwd()
        bwd()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fb = e0.elapsed_time(e1) / steps
    ok = bool((st == 0).all().item()) and bool(torch.isfinite(c2).all().item())
    ctx.close()
    return {"models": n, "ms_chi2": ms_f, "chi2_per_s": n * 1000.0 / ms_f,
            "ms_chi2_and_grad": ms_fb, "chi2_and_grad_per_s": n * 1000.0 / ms_fb,
            "all_finite": ok}


def time_beta_profile(torch, binding, w, dev, steps):
    """Radial anisotropy profile per proposal (4 numbers) sampled into the
    per-Gaussian beta_k, chi^2 and its gradient back to the profile, for a
    whole batch per launch."""
    from paper_2504_01302_amd import inputs
    ctx = binding.Context(w.geometries)
    for gi, g in enumerate(w.geometries):
        ctx.set_kinematics(gi, *inputs.kinematic_data(g.n_bins, seed=gi))
    par = binding.pack_params(w, dev, amplitudes=True)
    n = len(w.geom_idx)
    rng = np.random.default_rng(7)
    prof = torch.as_tensor(np.stack([rng.uniform(-0.4, 0.0, n), rng.uniform(0.0, 0.4, n),
                                     10.0 ** rng.uniform(-1.5, 0.5, n), rng.uniform(1.0, 3.0, n)],
                                    axis=1), device=dev)
    cot = torch.ones(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    state = {}

    def step():
        beta = ctx.beta_logistic(w.geom_idx, prof)
        args = (w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], beta, par["lum_I0"],
                par["mass_S0"])
        c2, V, st = ctx.eval_chi2(*args, keep_vrms2=True)
        g = ctx.vjp_chi2(*args, cot, vrms2=V)
        state["gp"] = ctx.beta_logistic_vjp(w.geom_idx, prof, g["beta"])
        state["ok"] = (st, c2)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st, c2 = state["ok"]
    ok = bool((st == 0).all().item()) and bool(torch.isfinite(state["gp"]).all().item())
    ctx.close()
    return {"models": n, "ms_profile_to_chi2_and_grad": ms, "per_s": n * 1000.0 / ms,
            "all_finite": ok}


def time_mge_pipeline(torch, binding, dev, steps, n=4096):
    """Per-proposal pipeline from profile parameters to chi^2 and its
    gradient: 1-D MGE of a Chameleon light profile (21 Gaussians, Euler
    order 10) -> lum_I0 of a small geometry -> v_rms^2 and chi^2 -> adjoint
    -> gradient with respect to the profile components; n proposals per
    launch.  Also the MGE kernels alone."""
    import numpy as np
    from paper_2504_01302_amd import inputs
    sig = np.exp(np.linspace(np.log(0.02), np.log(20.0), 21))
    base = inputs.config3(n).geometries[0]
    K = len(sig)
    g = inputs.Geometry(sig, np.full(K, 0.8), np.ones(K), base.mass_sigma, base.mass_q,
                        base.mass_S0, base.bh_sigma, base.distance_mpc, base.nx, base.ny,
                        base.pixsize, base.xc, base.yc, base.supersample, base.psf, base.n_bins,
                        base.bin_index, base.n_u)
    w = inputs.config3(n)
    params = [inputs.Params(p.inc, np.full(K, float(np.mean(p.beta))), p.mass_scale, p.m_bh)
              for p in w.params]
    w = inputs.Workload("mge", [g], np.zeros(n, np.int32), params)
    ctx = binding.Context([g])
    ctx.set_kinematics(0, *inputs.kinematic_data(g.n_bins, seed=0))
    par = binding.pack_params(w, dev, amplitudes=True)
    rng = np.random.default_rng(7)
    comp = np.zeros((n, 2, 3))
    comp[:, 0] = np.c_[np.full(n, 1.0), rng.uniform(0.03, 0.08, n), np.full(n, 0.5)]
    comp[:, 1] = np.c_[np.full(n, -1.0), rng.uniform(1.5, 3.0, n), np.full(n, 0.5)]
    comp = torch.as_tensor(comp, device=dev)
    ones = torch.ones(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    args = lambda amp: (w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                        amp.reshape(-1), par["mass_S0"])

    def mge_only():
        amp = binding.jam_mge1d(comp, sig, 10)
        binding.jam_mge1d_vjp(comp, sig, amp, 10)

    def pipeline():
        amp = binding.jam_mge1d(comp, sig, 10)
        c2, V, st = ctx.eval_chi2(*args(amp), keep_vrms2=True)
        gr = ctx.vjp_chi2(*args(amp), ones, vrms2=V)
        return c2, st, binding.jam_mge1d_vjp(comp, sig, gr["lum_I0"].reshape(n, K), 10)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms_mge = timed(mge_only, steps)
    ms_pipe = timed(pipeline, steps)
    c2, st, gcomp = pipeline()
    torch.cuda.synchronize()
    ok = bool((st == 0).all().item()) and bool(torch.isfinite(c2).all().item()) and \
        bool(torch.isfinite(gcomp).all().item())
    ctx.close()
    return {"proposals": n, "gaussians": K, "ms_mge_fwd_bwd": ms_mge,
            "ms_profile_to_chi2_and_grad": ms_pipe,
            "proposals_per_s": n * 1000.0 / ms_pipe, "all_finite": ok}


def run_extras(a, torch, binding, inputs, dev, w1):
    """The extra workloads named by --extra (default all), each timed on its own."""
    g, p = w1.geometries[0], w1.params[0]
    k = max(3, a.steps // 4)
    extras = {
        "batched_4096_small": lambda: time_batch(torch, binding, inputs.config3(4096), dev,
                                                 k, a.form, a.launch, a.graph),
        "ifu_scale_batch_8": lambda: time_batch(
            torch, binding, inputs.Workload("cfg2x8", [g], np.zeros(8, np.int32), [p] * 8),
            dev, k, a.form, a.launch, a.graph),
        "uneven_1024": lambda: time_batch(torch, binding, inputs.config4(1024), dev, 2,
                                          a.form, a.launch, a.graph),
        "uneven_1024_autotuned_graph": lambda: time_batch(
            torch, binding, inputs.config4(1024), dev, 2, 0, 0, 1, autotune=1),
        "chi2_4096_small": lambda: time_chi2(torch, binding, inputs.config3(4096), dev, k,
                                             a.form, a.launch, a.graph),
        "mge_chi2_4096_small": lambda: time_mge_pipeline(torch, binding, dev, k),
        "beta_profile_chi2_4096_small": lambda: time_beta_profile(
            torch, binding, inputs.config3(4096), dev, k),
        "spherical_ifu_scale": lambda: time_spherical_both(torch, binding, w1, dev, k),
        "cylindrical_composite_42x95": lambda: time_batch(
            torch, binding, inputs.config_composite(), dev, k, a.form, a.launch, a.graph),
        "spherical_composite_42x95": lambda: time_spherical_both(
            torch, binding, inputs.config_composite(), dev, max(2, k // 2)),
        "spherical_1024_small": lambda: time_spherical_both(torch, binding, inputs.config3(1024),
                                                            dev, max(2, k // 2)),
    }
    names = [x for x in a.extra.split(",") if x] or list(extras)
    unknown = [x for x in names if x not in extras]
    if unknown:
        sys.exit(f"unknown extra workload(s) {unknown}; known: {list(extras)}")
    return {x: extras[x]() for x in names}


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                          "(the path shards by model or by pixel rows across GPUs, "
                          "which is documented but not built)"}))
        sys.exit(2)
    import torch
    from paper_2504_01302_amd import binding, inputs

    dev = torch.device("cuda:0")
    w1 = inputs.config2(seed=0)
    g, p = w1.geometries[0], w1.params[0]
    if a.only_extra:
        rec = {"extra": run_extras(a, torch, binding, inputs, dev, w1)}
        print(json.dumps(rec), flush=True)
        return
    n = a.batch
    w = inputs.Workload("cfg2", [g], np.zeros(n, np.int32), [p] * n)
    ctx = binding.Context([g], form=a.form, launch=a.launch, graph=a.graph, autotune=a.autotune)
    par = binding.pack_params(w, dev, amplitudes=True)
    cot = torch.as_tensor(np.tile(inputs.cotangent(g.n_bins, 1)[0], n), device=dev)
    nb, _, _ = ctx.sizes(w.geom_idx)
    V = torch.empty(nb, dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def fwd(c):
        c.eval_batch(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                     par["lum_I0"], par["mass_S0"], out=V, status=st)

    def bwd(c):
        return c.vjp(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                     par["lum_I0"], par["mass_S0"], V, cot)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(c, steps, with_bwd):
        """Event-timed loop of `steps` forward (+ backward) calls of context c,
        with the library's kernel timer running: (ms per step, wall s,
        numerator ms, numerator launches, sensitivity ms, its launches)."""
        binding.jam_timing(c.handle, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            fwd(c)
            if with_bwd:
                bwd(c)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return (e0.elapsed_time(e1) / steps, wall) + tuple(binding.jam_timing(c.handle, False))

    # eager loops: per-kernel timings (graph replays are not bracketed by the
    # kernel timer), and the eager throughput
    ek = ctx if not a.graph else binding.Context([g], form=a.form, launch=a.launch, graph=0,
                                                 autotune=a.autotune)
    for _ in range(a.warmup):
        fwd(ek)
        bwd(ek)
    torch.cuda.synchronize()
    ms_f, wall_f, num_ms, num_n, _, _ = timed(ek, a.steps, False)
    ms_fb, _, _, _, sens_ms, sens_n = timed(ek, a.steps, True)
    eager = {"models_per_s": n * 1000.0 / ms_f, "fwd_bwd_per_s": n * 1000.0 / ms_fb}
    if a.graph:
        # headline loops: the same calls replayed from recorded HIP graphs
        for _ in range(a.warmup):
            fwd(ctx)
            bwd(ctx)
        torch.cuda.synchronize()
        ms_f, wall_f, _, _, _, _ = timed(ctx, a.steps, False)
        ms_fb, _, _, _, _, _ = timed(ctx, a.steps, True)
        ek.close()

    # plain per-model forward on the same GPU: the per-pixel VALU kernel, one
    # workgroup per work item, no graph, one model per launch
    plain = None
    if not a.no_plain_baseline:
        w_one = inputs.Workload("cfg2", [g], np.zeros(1, np.int32), [p])
        pc = binding.Context([g], form=1, launch=0)
        p1 = binding.pack_params(w_one, dev, amplitudes=True)
        V1 = torch.empty(g.n_bins, dtype=torch.float64, device=dev)
        s1 = torch.empty(1, dtype=torch.int32, device=dev)
        run1 = lambda: pc.eval_batch(w_one.geom_idx, p1["inc"], p1["mass_scale"], p1["m_bh"],
                                     p1["beta"], p1["lum_I0"], p1["mass_S0"], out=V1, status=s1)
        run1()
        torch.cuda.synchronize()
        k1 = max(3, a.steps // 4)
        e0.record(stream)
        for _ in range(k1):
            run1()
        e1.record(stream)
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1) / k1
        plain = {"ms_per_model": ms1, "models_per_s": 1000.0 / ms1,
                 "speedup_of_value": (n * 1000.0 / ms_f) / (1000.0 / ms1)}
        pc.close()

    # parity of the timed configuration against the stored oracle values
    max_rel = None
    gpath = os.path.join(ROOT, "tests", "golden", "cfg2_seed0.json")
    if os.path.exists(gpath):
        ref = np.array(json.load(open(gpath))["vrms2"])
        out = V.cpu().numpy().reshape(n, -1)
        max_rel = float(np.max(np.abs(out / ref[None, :] - 1.0)))

    # roofline of the dominant kernel (the quadrature kernel)
    xs = {abs(v) for v in ((np.arange(g.nx * g.supersample + g.psf_n - 1)
                            - (g.nx * g.supersample + g.psf_n - 2) / 2.0))}
    ys = {abs(v) for v in ((np.arange(g.ny * g.supersample + g.psf_n - 1)
                            - (g.ny * g.supersample + g.psf_n - 2) / 2.0))}
    n_pix = len(xs) * len(ys)
    T = g.n_lum * (g.n_mass + 1) * g.n_u
    # (graph replays are not bracketed by the kernel timer)
    avg_num_s = (num_ms / num_n) * 1e-3 if num_n else None
    form_used = 1 if a.form == 1 else 2
    if form_used == 2:
        flops = 2.0 * n_pix * T * n
        roof = dict(bound="mfma", peak=FP32_MFMA_PEAK / 1e12)
    else:
        flops = PIX_FLOPS_PER_INTEGRAND * n_pix * T * n
        roof = dict(bound="alu", peak=FP32_VECTOR_PEAK / 1e12)
    achieved = flops / avg_num_s / 1e12 if avg_num_s else None
    kname = KERNEL_NAMES.get(ctx.plan_info(w.geom_idx).get("num_kernel"), "k_num_pix")
    traffic = profiled_traffic(kname) if (form_used == 2 and n == 1 and a.launch == 0
                                          and not a.autotune) else None
    roof.update(achieved=achieved, unit="TFLOP/s",
                frac=achieved / roof["peak"] if achieved else None, traffic=traffic,
                kernel=kname, avg_launch_ms=avg_num_s * 1e3 if avg_num_s else None,
                launches=num_n, flops_per_launch=flops)

    rec = {
        "metric": "JAM models/sec and fwd+bwd/sec (200² px, 40×40 MGE) at ≤1e-5 rel err vs FP64",
        "value": n * 1000.0 / ms_f,
        "unit": "models/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_f,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 set-up, SB, bins)",
        "data": "synthetic",
        "config": {"workload": "IFU-scale JAM-cyl forward: 40 lum x 40 mass Gaussians + BH, "
                               "200x200 px at 0.025\" with 2x supersampling, 128 u-nodes, "
                               "31x31 PSF, 60 bins",
                   "models_per_launch": n, "form": form_used, "launch": a.launch,
                   "graph": a.graph, "autotune": a.autotune,
                   "schedule": ctx.plan_info(w.geom_idx)},
        "fwd_bwd_per_s": n * 1000.0 / ms_fb,
        "ms_per_fwd_bwd": ms_fb,
        "integrand_evals_per_s": float(n_pix) * T * n * 1000.0 / ms_f,
        "max_rel_err_vs_oracle": max_rel,
        "wall_s_forward_loop": wall_f,
        "roofline": roof,
        "eager_launches": eager,
        "sens_kernel_avg_ms": sens_ms / max(1, sens_n),
        "plain_per_model_forward": plain,
    }
    if not a.no_extra:
        rec["extra"] = run_extras(a, torch, binding, inputs, dev, w1)
    if a.copy_calibration:
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)     # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = src.numel() * 8
    if not a.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(g, p, a.cpu_sample)
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

"""Benchmark of the JAM-cyl hot path on one MI355X.

Workload: the IFU-scale model (40 luminous x 40 mass Gaussians + BH, 200x200
pixels at 0.025" with 2x supersampling, 128 u-nodes, 31x31 PSF, 60 bins),
synthetic and seeded.  A forward step is one jam_eval_batch of that model; a
fwd+bwd step adds one jam_vjp (the full adjoint).  Inputs are resident in HBM
before timing starts.  Prints one JSON line.

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
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", type=int, default=2,
                    help="1 per-pixel VALU kernel, 2 matrix-core kernel (0 = library default)")
    ap.add_argument("--batch", type=int, default=1,
                    help="models per launch (copies of the IFU-scale model)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy three times, the reference "
                         "kernel for scaling the HBM byte counters of a profile")
    ap.add_argument("--cpu-sample", type=int, default=256,
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
    return dict(value=1.0 / per_model, unit="models/s", cores=torch.get_num_threads(),
                kind="oracle",
                sample=f"N and I at {n_sample} of {len(x) * len(y)} padded sub-pixels of the "
                       f"IFU-scale model ({dt:.1f} s), scaled to one model")


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(the path shards by model or by pixel rows across GPUs, "
                          "which is documented but not built)"}))
        sys.exit(2)
    import torch
    from paper_2504_01302_amd import binding, inputs

    dev = torch.device("cuda:0")
    w1 = inputs.config2(seed=0)
    g, p = w1.geometries[0], w1.params[0]
    n = a.batch
    w = inputs.Workload("cfg2", [g], np.zeros(n, np.int32), [p] * n)
    ctx = binding.Context([g], form=a.form)
    par = binding.pack_params(w, dev, amplitudes=True)
    cot = torch.as_tensor(np.tile(inputs.cotangent(g.n_bins, 1)[0], n), device=dev)
    nb, _, _ = ctx.sizes(w.geom_idx)
    V = torch.empty(nb, dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def fwd():
        ctx.eval_batch(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                       par["lum_I0"], par["mass_S0"], out=V, status=st)

    def bwd():
        return ctx.vjp(w.geom_idx, par["inc"], par["mass_scale"], par["m_bh"], par["beta"],
                       par["lum_I0"], par["mass_S0"], V, cot)

    for _ in range(a.warmup):
        fwd()
        bwd()
    torch.cuda.synchronize()

    # forward
    binding.jam_timing(ctx.handle, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(a.steps):
        fwd()
    e1.record(stream)
    torch.cuda.synchronize()
    wall_f = time.perf_counter() - t0
    ms_f = e0.elapsed_time(e1) / a.steps
    num_ms, num_n, _, _ = binding.jam_timing(ctx.handle, False)

    # forward + backward
    binding.jam_timing(ctx.handle, True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(a.steps):
        fwd()
        bwd()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fb = e0.elapsed_time(e1) / a.steps
    _, _, sens_ms, sens_n = binding.jam_timing(ctx.handle, False)

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
    avg_num_s = (num_ms / max(1, num_n)) * 1e-3
    form_used = 1 if a.form == 1 else 2
    if form_used == 2:
        flops = 2.0 * n_pix * T * n
        roof = dict(bound="mfma", peak=FP32_MFMA_PEAK / 1e12)
    else:
        flops = PIX_FLOPS_PER_INTEGRAND * n_pix * T * n
        roof = dict(bound="alu", peak=FP32_VECTOR_PEAK / 1e12)
    achieved = flops / avg_num_s / 1e12
    roof.update(achieved=achieved, unit="TFLOP/s", frac=achieved / roof["peak"], traffic=None,
                kernel="k_num_pix" if form_used == 1 else "k_num_mfma",
                avg_launch_ms=avg_num_s * 1e3, launches=num_n)

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
                   "models_per_launch": n, "form": form_used},
        "fwd_bwd_per_s": n * 1000.0 / ms_fb,
        "ms_per_fwd_bwd": ms_fb,
        "max_rel_err_vs_oracle": max_rel,
        "wall_s_forward_loop": wall_f,
        "roofline": roof,
        "sens_kernel_avg_ms": sens_ms / max(1, sens_n),
    }
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

#!/usr/bin/env python3
"""Benchmark of the tensor-tomography hot path on one MI355X.

One step = one L-BFGS iteration of the plain method (search direction from
the history, forward projection of the direction, exact line search,
coefficient/residual update, adjoint for the new gradient, history update)
on the 100^3, ell_max 8, 240-projection, 100x100 x 8-segment workload with a
seeded twisted-fibre phantom and 1% noise.  Inputs are resident on the
device before the timed region.

value = algorithmic bytes of one forward plus one adjoint (per projection
4 C V + 4 nj nk n_seg each way) per step, divided by the step time.

Also reported: the dominant kernel against the HBM roofline (HIP-event
timing of every launch inside the timed region), the plain method's
time-to-residual, and the float64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def algorithmic_bytes(w):
    """Per projection, one direction: read/accumulate the volume and the image."""
    return 4.0 * w.n_coeff * w.n_vox + 4.0 * w.nj * w.nk * w.n_seg


def kernel_bytes(kind, w, n_unique, launches_per_call, S):
    """Algorithmic bytes of one launch of a kernel class (per-projection figures x projections per launch)."""
    V, C = w.n_vox, w.n_coeff
    img = 4.0 * w.nj * w.nk * w.n_seg
    if kind == "backproject":  # the whole adjoint of all S projections
        return S * (4.0 * C * V + img)
    if kind == "march":        # np projections per launch: read the mapped volume, write the image
        np_ = S / launches_per_call
        return np_ * (4.0 * n_unique * V + img)
    if kind == "map":          # read the volume once, write np mapped volumes
        np_ = S / launches_per_call
        return 4.0 * C * V + np_ * 4.0 * n_unique * V
    return None


def _source_sha():
    h = hashlib.sha256()
    for f in ("tt_proj.hip", "tt_internal.h", "tt_device.h"):
        with open(os.path.join(ROOT, "paper_2504_16446_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel, workload):
    """Measured HBM bytes per launch from committed rocprofv3 counter runs, if current."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != _source_sha():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, n_sample, c_np, y_np):
    """FP64 oracle forward + adjoint on n_sample evenly spaced projections."""
    import numpy as np
    import oracle
    import tt_inputs as synth

    inner, outer = synth.angles(w)
    sel = np.linspace(0, len(inner) - 1, n_sample).round().astype(int)
    g = oracle.Geometry(w.n, w.ell_max, inner[sel], outer[sel], w.nj, w.nk, w.n_seg,
                        synth.lab_frame(), n_sub=w.n_sub, step=w.step)
    g.B()
    c64 = c_np.astype(np.float64)
    y64 = y_np[sel].astype(np.float64)
    t0 = time.perf_counter()
    oracle.project(g, c64)
    oracle.adjoint(g, y64)
    dt = time.perf_counter() - t0
    bytes_ = 2 * n_sample * algorithmic_bytes(w)
    threads = oracle.max_threads()
    per_vol = 8.0 * w.n_vox * w.n_coeff
    adj_threads = max(1, min(threads, int(oracle.MEM_BUDGET // per_vol)))
    return {
        "value": bytes_ / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
        "sample": (f"float64 C oracle, forward + adjoint of {n_sample} of {w.n_proj} projections "
                   f"({w.name} geometry, same algorithmic-byte count per projection), {dt:.2f} s wall; "
                   f"forward on {threads} OpenMP threads, adjoint on {adj_threads}; host '{_cpu_model()}', "
                   f"os.cpu_count()={os.cpu_count()}"),
    }


def warm_vs_plain_heldout(dev, n=4, plain_iters=30):
    """Learned warm start vs zero start on held-out 48^3 phantoms: wall time to the
    residual the zero start reaches after plain_iters iterations (medians)."""
    import numpy as np
    import torch
    import tt_inputs as synth
    from paper_2504_16446_amd import warmstart
    from paper_2504_16446_amd.projector import LBFGS, Projector

    if not os.path.exists(warmstart.DEFAULT_WEIGHTS):
        return None
    model = warmstart.load(warmstart.DEFAULT_WEIGHTS, dev)
    w = synth.WORKLOADS["c4"]
    P = Projector.from_workload(w, device=dev)
    kap = warmstart.kappa(P, w.radius)
    rows = []
    for seed in 1_000_000 + np.arange(n):
        c_true = warmstart.bundle_phantom(w, int(seed), dev)
        data = P.forward(c_true)
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(seed) + 100000)
        data.add_(torch.randn(data.shape, generator=gen, device=dev), alpha=w.noise * float(data.abs().max()))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = torch.zeros(P.vol_shape, device=dev)
        it_p, _, rel_p, s1 = warmstart.lbfgs_to(P, data, w.mu, c, 0.0, plain_iters, log_every=0)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        del s1
        t0 = time.perf_counter()
        c0, _, fb = warmstart.warm_start(model, P, data, kap=kap)
        c = torch.zeros(P.vol_shape, device=dev)
        it_w, _, rel_w, s2 = warmstart.lbfgs_to(P, data, w.mu, c, rel_p, 4 * plain_iters, log_every=0,
                                                first_direction=c0)
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        del s2
        rows.append((t_plain, it_p, t_warm, it_w, rel_p))
    a = np.array(rows)
    return {"workload": "c4 held-out phantoms (seeds 1e6..), 48^3, ell_max 6, 120 projections, 1% noise",
            "phantoms": n, "target": f"zero-start residual after {plain_iters} iterations",
            "plain_seconds_median": float(np.median(a[:, 0])), "plain_iterations": plain_iters,
            "warm_seconds_median": float(np.median(a[:, 2])), "warm_iterations_median": float(np.median(a[:, 3])),
            "speedup_median": float(np.median(a[:, 0] / a[:, 2])),
            "note": "warm time includes the scale kappa, backprojection, inference and blending"}


def precision_report(dev, n_rays=128, n_vox=16):
    """Errors of the fp32 and bf16 map tiers against the float64 oracle on the
    128^3 / ell_max 8 / 300-projection / 16-segment workload (sampled outputs)."""
    import numpy as np
    import torch
    import oracle
    import tt_inputs as synth
    from paper_2504_16446_amd import phantom
    from paper_2504_16446_amd.projector import Projector

    w = synth.WORKLOADS["c3"]
    og = oracle.Geometry.from_workload(w)
    rng = np.random.default_rng(5)
    c = phantom.coefficients(w)
    y = rng.standard_normal((w.n_proj, w.nj, w.nk, w.n_seg), dtype=np.float32)
    sjk = np.stack([rng.integers(0, w.n_proj, n_rays), rng.integers(0, w.nj, n_rays),
                    rng.integers(0, w.nk, n_rays)], 1)
    xyz = np.stack([rng.integers(0, m, n_vox) for m in w.n], 1)
    ref_f = oracle.project_rays(og, c, sjk)
    ref_a = oracle.adjoint_voxels(og, y, xyz)
    out = {"workload": "c3", "inputs": "phantom coefficients; Gaussian data",
           "sampled": f"{n_rays} rays x {w.n_seg} segments, {n_vox} voxels x {w.n_coeff} coefficients"}
    P = Projector.from_workload(w, device=dev)
    ct, yt = torch.from_numpy(c).to(dev), torch.from_numpy(y).to(dev)
    for tier in ("fp32", "bf16"):
        P.set_precision(tier)
        I = P.forward(ct)
        g = P.adjoint(yt)
        got_f = I[sjk[:, 0], sjk[:, 1], sjk[:, 2]].cpu().numpy().astype(np.float64)
        got_a = g[xyz[:, 0], xyz[:, 1], xyz[:, 2]].cpu().numpy().astype(np.float64)
        out[tier] = {"forward_rel_l2": float(np.linalg.norm(got_f - ref_f) / np.linalg.norm(ref_f)),
                     "adjoint_rel_l2": float(np.linalg.norm(got_a - ref_a) / np.linalg.norm(ref_a))}
    return out


def properties_bench(dev, reps=5):
    """Derived per-voxel quantities on a 256^3 / ell_max 8 coefficient volume:
    HBM throughput (read C floats, write 22 floats per voxel) of one launch."""
    import torch
    import tt_inputs as synth
    from paper_2504_16446_amd.projector import PROPERTY_FIELDS, tensor_properties

    w = synth.WORKLOADS["c5"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(4321)
    c = torch.randn((w.n_vox, w.n_coeff), device=dev, generator=gen)
    out = tensor_properties(c, w.ell_max)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        tensor_properties(c, w.ell_max, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 4.0 * w.n_vox * (w.n_coeff + len(PROPERTY_FIELDS))
    del c, out
    torch.cuda.empty_cache()
    return {"workload": f"{w.n[0]}^3 voxels x {w.n_coeff} coefficients (ell_max {w.ell_max})",
            "ms": ms, "algorithmic_bytes": nbytes, "achieved": nbytes / (ms * 1e-3) / 1e9,
            "unit": "GB/s", "peak": HBM_PEAK_GBPS, "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def regulariser_bench(dev, reps=5):
    """Laplacian / Huber regularisers and the gradient-descent update on a
    256^3 x 45 coefficient volume: HBM throughput of each (algorithmic bytes:
    Laplacian 20 n, Huber 12 n, update 20 n for n floats)."""
    import ctypes as C
    import torch
    import tt_inputs as synth
    from paper_2504_16446_amd._lib import call
    from paper_2504_16446_amd.projector import huber_reg, laplacian_reg

    w = synth.WORKLOADS["c5"]
    shape = w.n + (w.n_coeff,)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    c = torch.randn(shape, device=dev, generator=gen)
    g = torch.zeros_like(c)
    work = torch.empty_like(c)
    y = c.clone()
    val = torch.zeros(1, dtype=torch.float64, device=dev)
    n = c.numel()
    stream = torch.cuda.current_stream(dev)
    out = {"workload": f"{w.n[0]}^3 x {w.n_coeff} coefficients"}
    cases = (("laplacian", 20.0, lambda: laplacian_reg(c, 1e-2, g, val, work)),
             ("huber", 12.0, lambda: huber_reg(c, 0.05, 1e-2, g, val)),
             ("gd_step", 20.0, lambda: call("tt_gd_step", C.c_void_p(c.data_ptr()), C.c_void_p(y.data_ptr()),
                                            C.c_void_p(g.data_ptr()), None, n, 1e-6, 0.5,
                                            C.c_void_p(stream.cuda_stream))))
    for name, per, fn in cases:
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "GBps": per * n / (ms * 1e-3) / 1e9, "frac": per * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    del c, g, work, y
    torch.cuda.empty_cache()
    return out


def joseph_bench(w, dev, reps=3):
    """Forward + adjoint with Joseph's method on the same workload: kernel times
    and algorithmic GB/s (same per-projection bytes as the trilinear model)."""
    import torch
    from paper_2504_16446_amd.projector import Projector

    P = Projector.from_workload(w, device=dev, model="joseph")
    gen = torch.Generator(device=dev)
    gen.manual_seed(99)
    c = torch.randn(P.vol_shape, device=dev, generator=gen)
    y = torch.randn(P.data_shape, device=dev, generator=gen)
    I = P.forward(c)
    g = P.adjoint(y)
    torch.cuda.synchronize()
    P.timing(True)
    for _ in range(reps):
        P.forward(c, out=I)
        P.adjoint(y, out=g)
    kt = P.timing_read()
    P.timing(False)
    ms = {k: v[0] / reps for k, v in kt.items() if v[1]}
    total = sum(ms.values())
    bytes_ = 2 * w.n_proj * algorithmic_bytes(w)
    del P, c, y, I, g
    torch.cuda.empty_cache()
    return {"workload": w.name, "ms_fwd_adj": total, "kernels_ms": ms,
            "algorithmic_GBps": bytes_ / (total * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--ttr-iters", type=int, default=None,
                    help="plain L-BFGS iterations for time-to-residual (default: the workload's)")
    ap.add_argument("--cpu-sample", type=int, default=24, help="projections in the CPU-oracle sample")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--ttr-c5", action="store_true",
                    help="also run the 256^3 plain-vs-warm comparison to relative residual 1e-3 (minutes)")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision report")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the derived-quantity, Joseph and regulariser measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import tt_inputs as synth
    from paper_2504_16446_amd import phantom
    from paper_2504_16446_amd.projector import LBFGS, Projector

    w = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] workload {w.name}: {w.n} ell_max {w.ell_max} S={w.n_proj} "
          f"detector {w.nj}x{w.nk}x{w.n_seg}", file=sys.stderr, flush=True)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    P = Projector.from_workload(w, device=dev)
    c_true_np = phantom.coefficients(w)
    c_true = torch.from_numpy(c_true_np).to(dev)
    clean = P.forward(c_true)
    sigma = w.noise * float(clean.abs().max())
    noise = torch.from_numpy(synth.noise(P.data_shape, w.seed_noise).astype(np.float32)).to(dev)
    data = (clean + sigma * noise).contiguous()
    del clean, noise
    torch.cuda.synchronize()

    # ---- timed region: K L-BFGS iterations -------------------------------
    solver = LBFGS(P, m=10)
    c = torch.zeros(P.vol_shape, device=dev)
    solver.init(c, data, None, w.mu)
    for _ in range(args.warmup):
        solver.step()
    torch.cuda.synchronize()
    P.timing(True)
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        solver.step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t_wall
    step_ms = ev0.elapsed_time(ev1) / args.steps
    kt = P.timing_read()
    P.timing(False)
    print(f"[bench] {args.steps} steps: {step_ms:.3f} ms/step (wall {wall_s:.3f} s)", file=sys.stderr, flush=True)

    per_dir = w.n_proj * algorithmic_bytes(w)
    value = 2 * per_dir / (step_ms * 1e-3) / 1e9

    kernels = {}
    for k, (ms, n) in kt.items():
        if n:
            kernels[k] = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps,
                          "avg_launch_ms": ms / n}
    dom = max(((k, v) for k, v in kernels.items() if k in ("map", "march", "backproject")),
              key=lambda kv: kv[1]["ms_per_step"])[0]
    per_call = kernels[dom]["launches_per_step"]
    kb = kernel_bytes(dom, w, P.n_unique, per_call, w.n_proj)
    avg_s = kernels[dom]["avg_launch_ms"] * 1e-3
    achieved = kb / avg_s / 1e9
    traffic = _traffic(dom, w.name)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                "traffic": traffic, "algorithmic_bytes_per_launch": kb}

    # ---- plain method: time to residual ----------------------------------
    iters = args.ttr_iters if args.ttr_iters is not None else (50 if w.name == "c2" else 10)
    solver2 = LBFGS(P, m=10)
    c2 = torch.zeros(P.vol_shape, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver2.init(c2, data, None, w.mu)
    n_done, hist = solver2.run(iters)
    torch.cuda.synchronize()
    ttr_s = time.perf_counter() - t0
    r = P.forward(c2) - data
    final_rel = float(r.double().norm() / data.double().norm())
    del solver2, r
    ttr = {"plain": {"workload": w.name, "iterations": n_done, "seconds": ttr_s, "final_rel_residual": final_rel,
                     "loss_first_last": [float(hist[0, 0]), float(hist[-1, 0])] if n_done else None},
           "warm_start": None}
    del solver
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu oracle sample ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, args.cpu_sample, c_true_np, data.cpu().numpy())
    if not args.no_warm:
        print("[bench] warm start vs plain ...", file=sys.stderr, flush=True)
        ttr["warm_start"] = warm_vs_plain_heldout(dev)
        if args.ttr_c5:
            from paper_2504_16446_amd import warmstart
            del P, data, c, c2
            torch.cuda.empty_cache()
            model = warmstart.load(warmstart.DEFAULT_WEIGHTS, dev)
            ttr["warm_start_c5"] = warmstart.compare(model, synth.WORKLOADS["c5"], 1e-3, 1500)
    print("[bench] precision report ...", file=sys.stderr, flush=True)
    precision = None if args.no_precision else precision_report(dev)
    print("[bench] derived quantities ...", file=sys.stderr, flush=True)
    props = None if args.no_extras else properties_bench(dev)
    print("[bench] Joseph's method ...", file=sys.stderr, flush=True)
    joseph = None if args.no_extras else joseph_bench(w, dev)
    print("[bench] regularisers ...", file=sys.stderr, flush=True)
    regs = None if args.no_extras else regulariser_bench(dev)

    line = {
        "metric": "fwd+adj projector GB/s & % HBM roof; time-to-residual warm-start vs plain",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n[0]}^3 voxels, ell_max {w.ell_max} ({w.n_coeff} coeffs), "
                               f"{w.n_proj} projections, {w.nj}x{w.nk} px x {w.n_seg} segments; "
                               f"step = one L-BFGS iteration (m=10, mu={w.mu})",
                   "fwd_adj_algorithmic_bytes_per_step": 2 * per_dir},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "time_to_residual": ttr,
        "precision": precision,
        "tensor_properties": props,
        "joseph": joseph,
        "regularisers": regs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

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
    """Algorithmic bytes of one launch of a kernel class."""
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
    from paper_2504_16446_amd import synth

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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--ttr-iters", type=int, default=None,
                    help="plain L-BFGS iterations for time-to-residual (default: the workload's)")
    ap.add_argument("--cpu-sample", type=int, default=12, help="projections in the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2504_16446_amd import phantom, synth
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
    ttr = {"plain": {"iterations": n_done, "seconds": ttr_s, "final_rel_residual": final_rel,
                     "loss_first_last": [float(hist[0, 0]), float(hist[-1, 0])] if n_done else None},
           "warm_start": None}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu oracle sample ...", file=sys.stderr, flush=True)
        y_np = data.cpu().numpy()
        cpu = cpu_baseline(w, args.cpu_sample, c_true_np, y_np)

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
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

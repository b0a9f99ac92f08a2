#!/usr/bin/env python3
"""Benchmark of the tensor-tomography hot path on one MI355X.

One step = one L-BFGS iteration of the plain method (search direction from
the history, forward projection of the direction, exact line search,
coefficient/residual update, adjoint for the new gradient, history update).
Default workload: 256^3 voxels, ell_max 8 (45 coefficients), 400 projections,
256x256 px x 16 segments, seeded multi-bundle phantom, no noise (the largest
single-GPU configuration).  Inputs are resident on the device before the
timed region.

value = algorithmic bytes of one forward plus one adjoint (per projection
4 C V + 4 nj nk n_seg each way) per step, divided by the step time (an
effective rate: the kernels keep data on chip across projections).

roofline: the dominant kernel against the roof that binds it -- the adjoint
(voxel-driven gather + MFMA transpose map) against the fp32 compute peak with
its algorithmic flops (16 U flops per ray sample touching the volume: 8
voxels x U segment values x multiply-add; 2 U C flops per voxel and
projection for the transpose map), the map against the fp32 MFMA peak, the
march against HBM with its algorithmic bytes; HIP-event timing of every
launch inside the timed region, measured HBM traffic from committed
rocprofv3 counter runs.  Also reported: time to residual (at 256^3 the plain
zero start against the learned warm start, both to relative residual 1e-3),
the float64 CPU oracle on a bounded projection subset, precision tiers and
secondary kernels.
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
FP32_PEAK_TFLOPS = 157.3  # MI355X fp32 vector (and fp32 dense MFMA)


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


def kernel_roof(kind, w, n_unique, samples, launches_per_step, avg_s):
    """Roofline entry of one kernel class: (bound, algorithmic quantity per launch, unit, peak)."""
    V, C, S = w.n_vox, w.n_coeff, w.n_proj
    img = 4.0 * w.nj * w.nk * w.n_seg
    per_launch_proj = S / launches_per_step
    if kind == "backproject":  # the whole adjoint of all S projections per launch
        flops = 16.0 * n_unique * samples + 2.0 * n_unique * C * V * S
        return {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "algorithmic_flops_per_launch": flops,
                "count": "16 U per ray sample touching the volume + 2 U C per voxel and projection"}
    if kind == "map":  # read c once, M_s = B_s c for the batch's projections on MFMA
        flops = 2.0 * n_unique * C * V * per_launch_proj
        return {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "algorithmic_flops_per_launch": flops, "count": "2 U C per voxel and projection"}
    if kind == "fused":  # sparse fused forward: read the volume per projection, write the images
        nbytes = per_launch_proj * (4.0 * C * V + img)
        return {"bound": "hbm", "achieved": nbytes / avg_s / 1e9, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "algorithmic_bytes_per_launch": nbytes, "count": "4 C V + 4 nj nk n_seg per projection"}
    if kind == "march":  # read the batch's mapped volumes, write its images
        nbytes = per_launch_proj * (4.0 * n_unique * V + img)
        return {"bound": "hbm", "achieved": nbytes / avg_s / 1e9, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "algorithmic_bytes_per_launch": nbytes, "count": "4 U V + 4 nj nk n_seg per projection"}
    return None


WORKLOAD_LABEL = {"c1": "32cubed", "c2": "100cubed", "c3": "128cubed", "c4": "48cubed", "c5": "256cubed"}


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
        path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{WORKLOAD_LABEL.get(workload, workload)}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != _source_sha():
        return None
    return rec.get("bytes_per_launch")


def _compute_counters(kernel, workload):
    """Issue-side counters per launch of one kernel class (VALU busy, active
    lanes per VALU instruction, MFMA busy) from committed rocprofv3 runs, if current."""
    path = os.path.join(ROOT, "profiles", f"pmc_compute_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != _source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    return {"valu_busy": k["valu_busy"], "active_lanes": k["active_lanes"], "mfma_busy": k["mfma_busy"],
            "source": f"profiles/pmc_compute_{workload}.json"}


def cpu_sample_index(w, n_sample):
    import numpy as np
    return np.linspace(0, w.n_proj - 1, n_sample).round().astype(int)


def cpu_baseline(w, n_sample, c_np, y_sel):
    """FP64 oracle forward + adjoint on n_sample evenly spaced projections
    (y_sel: the data of those projections); the rate extrapolates linearly in
    the number of projections (projector cost is linear in S)."""
    import numpy as np
    import oracle
    import tt_inputs as synth

    inner, outer = synth.angles(w)
    sel = cpu_sample_index(w, n_sample)
    g = oracle.Geometry(w.n, w.ell_max, inner[sel], outer[sel], w.nj, w.nk, w.n_seg,
                        synth.lab_frame(), n_sub=w.n_sub, step=w.step)
    g.B()
    c64 = c_np.astype(np.float64)
    y64 = np.asarray(y_sel, dtype=np.float64)
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
                   f"({w.name} geometry, same algorithmic-byte count per projection; the rate extrapolates "
                   f"linearly to all {w.n_proj}), {dt:.2f} s wall; "
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


def precision_report(dev, n_rays=128, n_vox=16, reps=3):
    """Errors of the fp32 and bf16 map tiers against the float64 oracle on the
    128^3 / ell_max 8 / 300-projection / 16-segment workload (sampled outputs),
    and each tier's kernel times per forward + adjoint."""
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
        # per-kernel times of the tier (event-timed, 3 forward + adjoint passes)
        torch.cuda.synchronize()
        P.timing(True)
        P.timing_read()
        for _ in range(reps):
            P.forward(ct, out=I)
            P.adjoint(yt, out=g)
        kt = P.timing_read()
        P.timing(False)
        out[tier]["kernels_ms"] = {k: ms / reps for k, (ms, n) in kt.items() if n}
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


def sparse_bench(w, dev, ks=(1, 2, 4, 0), reps=2):
    """Sparse fused forward (sect. "Pipelines"): the forward with the k
    largest basis constants per projection and segment in one fused kernel
    (no mapped volumes), against the two-pass map + march with the exact
    constants on the same workload.  k = 0 stands for k = C (the exact map
    evaluated by the fused kernel)."""
    import torch
    from paper_2504_16446_amd.projector import Projector

    out = {"workload": w.name}
    gen = torch.Generator(device=dev)
    gen.manual_seed(98)
    c = None
    for k in ks:
        kk = k if k > 0 else w.n_coeff
        P = Projector.from_workload(w, device=dev, sparse_k=kk)
        if c is None:
            c = torch.randn(P.vol_shape, device=dev, generator=gen)
        I = P.forward(c)
        torch.cuda.synchronize()
        P.timing(True)
        for _ in range(reps):
            P.forward(c, out=I)
        kt = P.timing_read()
        P.timing(False)
        ms = kt["fused"][0] / max(kt["fused"][1], 1)
        out[f"k{kk}"] = {"ms_forward": ms, "workspace_bytes": P.work_bytes,
                         "algorithmic_GBps": w.n_proj * algorithmic_bytes(w) / (ms * 1e-3) / 1e9}
        del P, I
        torch.cuda.empty_cache()
    del c
    torch.cuda.empty_cache()
    return out


def measured_hbm(dev, gib=4, reps=5):
    """What the HBM sustains for plain streams under torch's own kernels (lower
    bounds of the hardware's rates): a device copy (read + write bytes), a fill
    (writes) and a dot product of two buffers (reads; the best of torch's
    reductions, sum and max read ~10% slower) over gib GiB each, averaged over
    reps launches timed with events on the current stream."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    nbytes = 4 * n
    out = {"bytes": nbytes,
           "copy_GBps": 2 * nbytes / timed(lambda: b.copy_(a)) / 1e9,
           "fill_GBps": nbytes / timed(lambda: b.fill_(0.5)) / 1e9,
           "read_GBps": 2 * nbytes / timed(lambda: torch.dot(a, b)) / 1e9,
           "kernels": "torch copy_, fill_ and dot over float32 buffers"}
    del a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--ttr-iters", type=int, default=None,
                    help="plain L-BFGS iterations for time-to-residual on workloads other than c5 (default 50)")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="projections in the CPU-oracle sample (default 4 at 256^3, 24 otherwise)")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision report")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the derived-quantity, Joseph and regulariser measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sparse-k", type=int, default=0,
                    help="time the steps with the sparse fused forward keeping k basis constants per segment")
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
    if args.sparse_k > 0:  # data from the exact operator, steps with the sparse fused forward
        P_exact, P = P, Projector.from_workload(w, device=dev, sparse_k=args.sparse_k)
    samples = P.ray_samples()
    forward_batch = P.batch
    work_bytes = P.work_bytes
    c_true_np = phantom.coefficients(w)
    c_true = torch.from_numpy(c_true_np).to(dev)
    data = (P_exact if args.sparse_k > 0 else P).forward(c_true)
    if args.sparse_k > 0:
        del P_exact
        torch.cuda.empty_cache()
    if w.noise > 0:
        sigma = w.noise * float(data.abs().max())
        noise = torch.from_numpy(synth.noise(P.data_shape, w.seed_noise).astype(np.float32)).to(dev)
        data.add_(noise, alpha=sigma)
        del noise
    del c_true
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
    roofs = {}
    for k in ("map", "march", "fused", "backproject"):
        if k in kernels:
            r = kernel_roof(k, w, P.n_unique, samples, kernels[k]["launches_per_step"],
                            kernels[k]["avg_launch_ms"] * 1e-3)
            r["frac"] = r["achieved"] / r["peak"]
            r["avg_launch_ms"] = kernels[k]["avg_launch_ms"]
            r["traffic"] = _traffic(k, w.name)
            r["counters"] = _compute_counters(k, w.name)
            roofs[k] = r
    dom = max(roofs, key=lambda k: kernels[k]["ms_per_step"])
    roofline = dict(kernel=dom, **roofs[dom])

    # ---- time to residual ---------------------------------------------------
    ttr = {}
    del solver
    n_sample = args.cpu_sample if args.cpu_sample is not None else (4 if w.name == "c5" else 24)
    y_sel = data[torch.from_numpy(cpu_sample_index(w, n_sample)).to(dev)].cpu().numpy()
    torch.cuda.empty_cache()
    if w.name == "c5":
        if not args.no_warm:
            from paper_2504_16446_amd import warmstart
            P = data = c = None
            torch.cuda.empty_cache()
            print("[bench] 256^3 plain vs warm start to relative residual 1e-3 ...", file=sys.stderr, flush=True)
            model = warmstart.load(warmstart.DEFAULT_WEIGHTS, dev)
            ttr["c5_plain_vs_warm"] = warmstart.compare(model, w, 1e-3, 1500)
    else:
        iters = args.ttr_iters if args.ttr_iters is not None else 50
        solver2 = LBFGS(P, m=10)
        c2 = torch.zeros(P.vol_shape, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver2.init(c2, data, None, w.mu)
        n_done, hist = solver2.run(iters)
        torch.cuda.synchronize()
        ttr_s = time.perf_counter() - t0
        solver2.refresh()
        _, rn, In, _ = solver2.query()
        ttr["plain"] = {"workload": w.name, "iterations": n_done, "seconds": ttr_s, "final_rel_residual": rn / In,
                        "loss_first_last": [float(hist[0, 0]), float(hist[-1, 0])] if n_done else None}
        del solver2, c2
        if not args.no_warm:
            print("[bench] warm start vs plain on held-out 48^3 phantoms ...", file=sys.stderr, flush=True)
            ttr["c4_heldout"] = warm_vs_plain_heldout(dev)
    P = data = c = None
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu oracle sample ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, n_sample, c_true_np, y_sel)
    print("[bench] precision report ...", file=sys.stderr, flush=True)
    precision = None if args.no_precision else precision_report(dev)
    print("[bench] derived quantities ...", file=sys.stderr, flush=True)
    props = None if args.no_extras else properties_bench(dev)
    print("[bench] Joseph's method ...", file=sys.stderr, flush=True)
    joseph = None if args.no_extras else joseph_bench(w, dev)
    print("[bench] regularisers ...", file=sys.stderr, flush=True)
    regs = None if args.no_extras else regulariser_bench(dev)
    print("[bench] sparse fused forward ...", file=sys.stderr, flush=True)
    sparse = None if args.no_extras else sparse_bench(w, dev)
    print("[bench] measured HBM streams ...", file=sys.stderr, flush=True)
    hbm = None if args.no_extras else measured_hbm(dev)
    print("[bench] warm-start network layers ...", file=sys.stderr, flush=True)
    if args.no_extras:
        netb = None
    else:
        from paper_2504_16446_amd import net as _net
        netb = _net.bench(dev)
    if sparse is not None:
        sparse["two_pass_ms_forward"] = sum(kernels[k]["ms_per_step"] for k in ("map", "march") if k in kernels)
        sparse["two_pass_workspace_bytes"] = work_bytes

    line = {
        "metric": "fwd+adj projector GB/s & % HBM roof; time-to-residual warm-start vs plain",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n[0]}^3 voxels, ell_max {w.ell_max} ({w.n_coeff} coeffs), "
                               + (f"sparse fused map k={args.sparse_k}, " if args.sparse_k > 0 else "") +
                               f"{w.n_proj} projections, {w.nj}x{w.nk} px x {w.n_seg} segments, "
                               f"{w.phantom} phantom, noise {w.noise}; "
                               f"step = one L-BFGS iteration (m=10, mu={w.mu})",
                   "fwd_adj_algorithmic_bytes_per_step": 2 * per_dir, "ray_samples_per_direction": samples,
                   "forward_batch": forward_batch},
        "roofline": roofline,
        "roofline_kernels": roofs,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "time_to_residual": ttr,
        "precision": precision,
        "tensor_properties": props,
        "joseph": joseph,
        "regularisers": regs,
        "sparse_fused": sparse,
        "network": netb,
        "measured_hbm": hbm,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

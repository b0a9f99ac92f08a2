"""Learned warm start for L-BFGS: training-set synthesis, training, patchwise
inference and the plain-versus-warm comparison.

The paper's outlook (section 4) names simulated data for training
machine-learning models; here such data trains a small 3-D convolutional
network that maps the normalised backprojection of the measured data to
initial SH coefficients, which L-BFGS then refines.  Zero-initialised L-BFGS
is the fallback (taken when the prediction is zero or not finite; a poor but
finite prediction costs at most the one iteration whose exact line search
scales it), and the final data residual, recomputed with an explicit forward
projection, decides whether it helped.

Pipeline (the projections, the scale kappa, the statistics, the network and
the tiling run in libtt_hip.so; torch supplies memory, the seeded phantoms'
rasterisation and the noise draws, which are inputs):
  1. x = A^T I / kappa, with kappa the median over the support of
     (A^T A u)_{v,00} for the unit isotropic field u: one scale per geometry,
     insensitive to the number of projections and segments;
  2. per-channel standardisation with training-set statistics (ell <= 6: the
     first 28 coefficient channels);
  3. the network on 48^3 tiles with an 8-voxel overlap, blended with linear
     ramps; coefficients of order 8 start at 0.
Training: seeded multi-bundle phantoms at 48^3 / ell_max 6, forward-projected
on 120 projections, 1% noise, backprojected; MSE against the true
coefficients; Adam (constant lr 1e-3), 20 epochs, batch 8.
The prediction enters L-BFGS as the first search direction from zero, so the
exact line search fixes its scale (the geometry normalisation of 48^3
training volumes and large volumes differs) and adds a curvature pair along it.

Command line:
  python -m paper_2504_16446_amd.warmstart train   --out W.npz [--phantoms 4096 --epochs 20]
  python -m paper_2504_16446_amd.warmstart holdout --weights W.npz
  python -m paper_2504_16446_amd.warmstart compare --weights W.npz [--workload c5]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np
import torch

import tt_inputs as synth

from . import net
from ._lib import call
from .projector import LBFGS, Projector, sh_eval, sumsq

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_c4.npz")
TILE, OVERLAP, NET_CH = 48, 8, 28


def _log(msg, **kw):
    """Progress record (one JSON object per line) on stderr: stdout carries results only."""
    print(json.dumps({"t": round(time.time(), 3), "msg": msg, **kw}), file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# phantoms on the device
# ---------------------------------------------------------------------------
def _ell_of_index(ell_max):
    return np.concatenate([np.full(2 * l + 1, l) for l in range(0, ell_max + 1, 2)])


def lobe_coeffs(ell_max, axis, degree):
    """SH coefficients of the fibre lobe (1-d) + 5 d (n.q)^4 about `axis`."""
    Y = sh_eval(ell_max, np.asarray(axis, np.float64)[None])[0]
    g = synth.zh_lobe_weights(np.array([degree]))[0]
    ells = _ell_of_index(ell_max)
    out = np.zeros_like(Y)
    for slot, l in enumerate((0, 2, 4)):
        if l <= ell_max:
            out[ells == l] = g[slot] * 4.0 * np.pi / (2 * l + 1) * Y[ells == l]
    return out


def bundle_phantom(w: synth.Workload, seed: int, device, background=0.1):
    """Multi-bundle phantom coefficients [nx, ny, nz, C] (float32, on device)."""
    ax = [torch.arange(m, device=device, dtype=torch.float32) - (m - 1) / 2.0 for m in w.n]
    X, Y, Z = torch.meshgrid(*ax, indexing="ij")
    ball = (X * X + Y * Y + Z * Z) <= w.radius ** 2
    c = torch.zeros(w.n + (w.n_coeff,), device=device)
    c[..., 0] = background * math.sqrt(4.0 * math.pi) * ball
    for axis, centre, radius, degree in synth.bundle_params(w, seed):
        rx, ry, rz = X - float(centre[0]), Y - float(centre[1]), Z - float(centre[2])
        along = rx * float(axis[0]) + ry * float(axis[1]) + rz * float(axis[2])
        perp2 = rx * rx + ry * ry + rz * rz - along * along
        mask = ((perp2 <= radius * radius) & ball).to(torch.float32)
        lobe = torch.tensor(lobe_coeffs(w.ell_max, axis, degree), dtype=torch.float32, device=device)
        c += mask[..., None] * lobe
    return c.contiguous()


def kappa(P: Projector, radius: float) -> float:
    """Lower median over the support ball of (A^T A u)_{v,00} for u_{v,00} = 1 (library)."""
    return P.kappa(radius)


# ---------------------------------------------------------------------------
# training set and training
# ---------------------------------------------------------------------------
def synthesize(w: synth.Workload, seeds, device, log_every=256):
    """(backprojections [n, X, Y, Z, 28] float32, targets [n, X, Y, Z, 28] float32, kappa).

    The network input is the backprojection scaled by 1 / kappa; the scale is
    applied by the statistics and packing kernels, so the stored arrays are
    copies of the library's outputs."""
    P = Projector.from_workload(w, device=device)
    kap = kappa(P, w.radius)
    n = len(seeds)
    Xs = torch.empty((n,) + w.n + (NET_CH,), device=device)
    Ts = torch.empty((n,) + w.n + (NET_CH,), device=device)
    I = torch.empty(P.data_shape, device=device)
    g = torch.empty(P.vol_shape, device=device)
    for i, seed in enumerate(seeds):
        c = bundle_phantom(w, int(seed), device)
        P.forward(c, out=I)
        if w.noise > 0:
            gen = torch.Generator(device=device)
            gen.manual_seed(int(seed) + 100000)
            sigma = w.noise * float(I.abs().max())
            I.add_(torch.randn(I.shape, generator=gen, device=device), alpha=sigma)
        P.adjoint(I, out=g)
        Xs[i].copy_(g[..., :NET_CH])
        Ts[i].copy_(c[..., :NET_CH])
        if log_every and (i + 1) % log_every == 0:
            _log("synthesised", n=i + 1, of=n)
    return Xs, Ts, kap


def tiles_meeting_ball(n, radius, T=TILE, overlap=OVERLAP):
    """Origins of the inference tiles whose box meets the support ball
    (radius about the volume centre, voxel-centre coordinates)."""
    orig = [tile_origins(m, T, overlap) for m in n]
    keep = []
    for ox in orig[0]:
        for oy in orig[1]:
            for oz in orig[2]:
                d2 = 0.0
                for o, m in zip((ox, oy, oz), n):
                    lo, hi = o - (m - 1) / 2.0, o + T - 1 - (m - 1) / 2.0
                    d2 += max(lo, 0.0, -hi) ** 2
                if d2 <= radius * radius:
                    keep.append((ox, oy, oz))
    return keep


def synthesize_tiles(w: synth.Workload, seeds, tiles_per_phantom, device, seed=0):
    """Training tiles cut from whole phantoms of a large workload, as inference sees them.

    Each seeded multi-bundle phantom of workload w is projected with w's
    geometry (noise as w states) and backprojected; tiles_per_phantom of the
    48^3 inference tiles that meet the support ball are drawn at random, and
    the raw backprojection (first 28 channels) and the true coefficients are
    copied out of them.  Returns (inputs, targets, kappa) like synthesize."""
    dev = torch.device(device)
    P = Projector.from_workload(w, device=dev)
    kap = kappa(P, w.radius)
    keep = tiles_meeting_ball(w.n, w.radius)
    rng = np.random.default_rng(seed)
    n = len(seeds) * tiles_per_phantom
    Xs = torch.empty((n, TILE, TILE, TILE, NET_CH), device=dev)
    Ts = torch.empty((n, TILE, TILE, TILE, NET_CH), device=dev)
    I = torch.empty(P.data_shape, device=dev)
    g = torch.empty(P.vol_shape, device=dev)
    k = 0
    for i, sd in enumerate(seeds):
        c = bundle_phantom(w, int(sd), dev)
        P.forward(c, out=I)
        if w.noise > 0:
            gen = torch.Generator(device=dev)
            gen.manual_seed(int(sd) + 100000)
            I.add_(torch.randn(I.shape, generator=gen, device=dev), alpha=w.noise * float(I.abs().max()))
        P.adjoint(I, out=g)
        for t in rng.choice(len(keep), tiles_per_phantom, replace=False):
            ox, oy, oz = keep[t]
            Xs[k].copy_(g[ox:ox + TILE, oy:oy + TILE, oz:oz + TILE, :NET_CH])
            Ts[k].copy_(c[ox:ox + TILE, oy:oy + TILE, oz:oz + TILE, :NET_CH])
            k += 1
        del c
        _log("synthesised tiles", phantoms=i + 1, of=len(seeds), tiles=k)
    del P, I, g
    torch.cuda.empty_cache()
    return Xs, Ts, kap


def train(w: synth.Workload, n_phantoms=4096, epochs=20, batch=8, lr=1e-3, device="cuda:0", seed=0,
          tiles_per_phantom=0, seed0=0):
    """Train on whole 48^3 phantoms of w (tiles_per_phantom = 0, seeds 0..n-1) or on
    tiles of larger phantoms of w (seeds seed0..seed0+n-1, see synthesize_tiles)."""
    dev = torch.device(device)
    t0 = time.time()
    if tiles_per_phantom > 0:
        Xs, Ts, kap = synthesize_tiles(w, seed0 + np.arange(n_phantoms), tiles_per_phantom, dev, seed=seed)
    else:
        Xs, Ts, kap = synthesize(w, seed0 + np.arange(n_phantoms), dev)
    n_phantoms = Xs.shape[0]
    _log("training set ready", seconds=round(time.time() - t0, 2), kappa=kap, samples=n_phantoms)
    model = net.WarmStartNet(dev, seed=seed)
    model.set_input_statistics(Xs, pre=1.0 / kap)
    Xb = model.prepare_input(Xs, pre=1.0 / kap)  # bf16 [n, X, Y, Z, 32]
    del Xs
    torch.cuda.empty_cache()
    rng = np.random.default_rng(seed + 1)
    nvox = batch * int(np.prod(Ts.shape[1:4]))
    history = []
    for ep in range(epochs):
        perm = rng.permutation(n_phantoms)
        tot, nb = 0.0, 0
        for b0 in range(0, n_phantoms - batch + 1, batch):
            idx = torch.from_numpy(perm[b0:b0 + batch]).to(dev)
            loss = model.train_step(Xb.index_select(0, idx).contiguous(), Ts.index_select(0, idx).contiguous(), lr)
            tot += float(loss.item()) if (nb % 64 == 0) else 0.0
            nb += 1
        mse = tot / (len(range(0, nb, 64)) * nvox * NET_CH)
        history.append(mse)
        _log("epoch", epoch=ep + 1, sampled_mse=mse, seconds=round(time.time() - t0, 2))
    return model, history, kap


def save(model: net.WarmStartNet, path, meta):
    d = {k: v.numpy() for k, v in model.state_dict().items()}
    d["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, **d)


def load(path, device) -> net.WarmStartNet:
    """Load weights (numpy .npz of float arrays, no pickles)."""
    with np.load(path, allow_pickle=False) as f:
        d = {k: torch.from_numpy(f[k]) for k in f.files if k != "meta"}
    model = net.WarmStartNet(torch.device(device))
    model.load_state_dict(d)
    return model


# ---------------------------------------------------------------------------
# inference
# ---------------------------------------------------------------------------
def tile_origins(n, T=TILE, overlap=OVERLAP):
    if n == T:
        return [0]
    if n < T:
        raise ValueError("volume axis shorter than a tile")
    o = list(range(0, n - T + 1, T - overlap))
    if o[-1] + T < n:
        o.append(n - T)
    return o


def predict(model: net.WarmStartNet, P: Projector, data: torch.Tensor, kap: float, batch=8):
    """Warm-start coefficients [nx, ny, nz, C]: network on the normalised backprojection."""
    dev = P.device
    x = P.adjoint(data)  # scaled by 1 / kap inside the tile gather
    C_out = P.n_coeff
    orig = [tile_origins(m) for m in P.n]
    ot = [torch.tensor(o, dtype=torch.int32, device=dev) for o in orig]
    ntiles = len(orig[0]) * len(orig[1]) * len(orig[2])
    ytiles = torch.empty((ntiles, TILE, TILE, TILE, 32), device=dev)
    s = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    p = lambda t: C.c_void_p(t.data_ptr())
    xb = net.bf16_empty((batch, TILE, TILE, TILE, 32), dev)
    for t0 in range(0, ntiles, batch):
        nt = min(batch, ntiles - t0)
        call("tt_tile_gather", p(x), *P.n, C_out, NET_CH, 32, p(ot[0]), len(orig[0]), p(ot[1]), len(orig[1]),
             p(ot[2]), len(orig[2]), TILE, float(1.0 / kap), p(model.in_shift), p(model.in_scale), t0, nt, p(xb), s)
        y = model.forward(xb[:nt])
        ytiles[t0:t0 + nt].copy_(y)
    c0 = torch.empty(P.vol_shape, device=dev)
    call("tt_tile_blend", p(ytiles), 32, NET_CH, *P.n, p(ot[0]), len(orig[0]), p(ot[1]), len(orig[1]), p(ot[2]),
         len(orig[2]), TILE, OVERLAP, C_out, p(c0), s)
    return c0


def lbfgs_to(P: Projector, data, mu, c, target_rel, max_iter, log_every=10, label="", first_direction=None):
    """Run L-BFGS from c (in place) until ||Ac - I|| / ||I|| <= target_rel.

    The stop test reads the solver's running residual; the returned final
    residual is recomputed from an explicit forward projection of c.  With
    first_direction, the first iteration searches along that direction (exact
    line search) instead of the steepest-descent direction."""
    solver = LBFGS(P, m=10)
    solver.init(c, data, None, mu)
    loss, rn, In, _ = solver.query()
    rel0 = rn / In
    it, rel = 0, rel0
    if first_direction is not None and rel > target_rel and max_iter > 0:
        solver.step_direction(first_direction)
        loss, rn, In, _ = solver.query()
        rel = rn / In
        it = 1
    while rel > target_rel and it < max_iter:
        solver.step()
        loss, rn, In, _ = solver.query()
        rel = rn / In
        it += 1
        if log_every and it % log_every == 0:
            _log(f"{label} iteration", it=it, rel_resid=rel)
    solver.refresh()
    _, rn, In, _ = solver.query()
    return it, rel0, rn / In, solver


def warm_start(model, P, data, kap=None, radius=None):
    """(prediction, kappa, fallback): the network's coefficients, or None when the
    prediction is not finite (then the solver starts from zero as usual).

    The prediction is used as the first search direction from zero, so the
    exact line search picks its scale and a poor prediction costs at most one
    iteration; the loss can never rise above the zero start's."""
    if kap is None:
        kap = kappa(P, radius)
    c0 = predict(model, P, data, kap)
    ss = torch.zeros(1, dtype=torch.float64, device=P.device)
    sumsq(c0, ss)
    n2 = float(ss.item())
    if not math.isfinite(n2) or n2 == 0.0:
        return None, kap, True
    return c0, kap, False


def compare(model, w: synth.Workload, tol=1e-3, max_iter=2000, device="cuda:0", seed=None):
    """Plain (zero-start) L-BFGS to rel. residual tol, then the warm start to the same residual."""
    dev = torch.device(device)
    P = Projector.from_workload(w, device=dev)
    c_true = bundle_phantom(w, w.seed_phantom if seed is None else seed, dev)
    data = P.forward(c_true)
    if w.noise > 0:
        gen = torch.Generator(device=dev)
        gen.manual_seed(w.seed_noise)
        data.add_(torch.randn(data.shape, generator=gen, device=dev), alpha=w.noise * float(data.abs().max()))
    del c_true
    torch.cuda.synchronize()
    _log("compare: data ready", workload=w.name)
    c = torch.zeros(P.vol_shape, device=dev)
    t0 = time.perf_counter()
    it_p, rel0_p, rel_p, solver = lbfgs_to(P, data, w.mu, c, tol, max_iter, label="plain")
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    del solver
    _log("plain done", iterations=it_p, rel_resid=rel_p, seconds=t_plain)
    target = max(rel_p, tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c0, kap, fell_back = warm_start(model, P, data, radius=w.radius)
    torch.cuda.synchronize()
    t_ws = time.perf_counter() - t0
    c = torch.zeros(P.vol_shape, device=dev)
    it_w, rel0_w, rel_w, solver = lbfgs_to(P, data, w.mu, c, target, max_iter, label="warm", first_direction=c0)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    del solver
    res = {"workload": w.name, "target_rel_resid": target,
           "plain": {"iterations": it_p, "seconds": t_plain, "initial_rel_resid": rel0_p, "final_rel_resid": rel_p},
           "warm": {"iterations": it_w, "seconds": t_warm, "warm_start_seconds": t_ws,
                    "final_rel_resid": rel_w, "fallback": fell_back},
           "speedup": t_plain / t_warm if t_warm > 0 else None}
    _log("compare done", **res)
    return res


def holdout(model, w: synth.Workload, seeds, plain_iters=30, device="cuda:0"):
    """Per held-out phantom: zero-start residual after plain_iters iterations, and the
    iterations the warm start needs to reach it."""
    dev = torch.device(device)
    P = Projector.from_workload(w, device=dev)
    kap = kappa(P, w.radius)
    rows = []
    for seed in seeds:
        c_true = bundle_phantom(w, int(seed), dev)
        data = P.forward(c_true)
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(seed) + 100000)
        data.add_(torch.randn(data.shape, generator=gen, device=dev), alpha=w.noise * float(data.abs().max()))
        c = torch.zeros(P.vol_shape, device=dev)
        s = LBFGS(P, m=10)
        s.init(c, data, None, w.mu)
        _, rn, In, _ = s.query()
        rel_zero0 = rn / In
        for _ in range(plain_iters):
            s.step()
        _, rn, In, _ = s.query()
        target = rn / In
        c0, _, fb = warm_start(model, P, data, kap=kap)
        c = torch.zeros(P.vol_shape, device=dev)
        it_w, _, rel_w, s2 = lbfgs_to(P, data, w.mu, c, target, 4 * plain_iters, log_every=0, first_direction=c0)
        # relative residual right after the step along the prediction
        c1 = torch.zeros(P.vol_shape, device=dev)
        _, _, rel1, _ = lbfgs_to(P, data, w.mu, c1, 0.0, 1, log_every=0, first_direction=c0)
        rows.append({"seed": int(seed), "target": target, "zero_init_rel_resid": rel_zero0,
                     "warm_rel_resid_after_first_step": rel1, "warm_iterations": it_w,
                     "plain_iterations": plain_iters, "fallback": fb})
        _log("holdout", **rows[-1])
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned warm start for L-BFGS")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("train")
    a.add_argument("--out", required=True)
    a.add_argument("--phantoms", type=int, default=4096)
    a.add_argument("--epochs", type=int, default=20)
    a.add_argument("--batch", type=int, default=8)
    a.add_argument("--lr", type=float, default=1e-3)
    a.add_argument("--workload", default="c4",
                   help="geometry and phantom generator of the training data (c4: whole 48^3 phantoms)")
    a.add_argument("--tiles-per-phantom", type=int, default=0,
                   help="> 0: train on this many random inference tiles of each (larger) phantom")
    a.add_argument("--seed0", type=int, default=0, help="first phantom seed")
    b = sub.add_parser("holdout")
    b.add_argument("--weights", default=DEFAULT_WEIGHTS)
    b.add_argument("--count", type=int, default=16)
    b.add_argument("--plain-iters", type=int, default=30)
    c = sub.add_parser("compare")
    c.add_argument("--weights", default=DEFAULT_WEIGHTS)
    c.add_argument("--workload", default="c5")
    c.add_argument("--tol", type=float, default=1e-3)
    c.add_argument("--max-iter", type=int, default=2000)
    args = ap.parse_args(argv)
    if args.cmd == "train":
        w = synth.WORKLOADS[args.workload]
        model, hist, kap = train(w, args.phantoms, args.epochs, args.batch, args.lr,
                                 tiles_per_phantom=args.tiles_per_phantom, seed0=args.seed0)
        save(model, args.out, {"workload": args.workload, "phantoms": args.phantoms, "epochs": args.epochs,
                               "tiles_per_phantom": args.tiles_per_phantom, "seed0": args.seed0,
                               "batch": args.batch, "lr": args.lr, f"kappa_{args.workload}": kap,
                               "sampled_mse": hist})
        _log("saved", path=args.out)
    elif args.cmd == "holdout":
        model = load(args.weights, "cuda:0")
        rows = holdout(model, synth.WORKLOADS["c4"], 1_000_000 + np.arange(args.count), args.plain_iters)
        its = [r["warm_iterations"] for r in rows]
        _log("holdout summary", median_warm_iterations=float(np.median(its)), plain_iterations=args.plain_iters)
    else:
        model = load(args.weights, "cuda:0")
        compare(model, synth.WORKLOADS[args.workload], args.tol, args.max_iter)


if __name__ == "__main__":
    main()

"""Learned warm start: training data from the GPU solver, training with the
library's own network kernels, and evaluation at equal accuracy.

The network only proposes where a solve starts (phi0); the FAS V-cycle then
finishes every solve, so the fixed point it reaches is the solver's, and the
comparison with the marker-based phi0 is made at the same absolute residual:
a solve from any start stops once its finest-grid residual is at most
tol times the residual of the marker-based phi0 of that image.

Everything numeric runs in the HIP library (solves, features, forward,
backward, Adam); this module draws seeded instances on the host, moves
tensors and keeps the bookkeeping.
"""
from __future__ import annotations

import multiprocessing as mp
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import mgseg, synth

TRAIN_SEEDS = range(500000, 520000)
HELDOUT_SEEDS = range(600000, 601000)


def gpu_runtime_loaded() -> bool:
    """True when this process has the HIP / HSA runtime mapped (the library or
    torch initialised the GPU, or a profiler preloaded its runtime): such a
    process must not fork workers."""
    if torch.cuda.is_initialized():
        return True
    try:
        with open("/proc/self/maps") as fh:
            maps = fh.read()
    except OSError:
        return True
    return "libhsa-runtime64" in maps or "libamdhip64" in maps


def generate(seeds, n=512, workers=16, log=None):
    """Seeded 4-20-shape instances (images, markers, seeds).  Drawn on `workers`
    forked host processes that never touch the GPU, but only while this process
    has no GPU runtime loaded; otherwise (or for few seeds) in this process,
    calling log(done) every 50 instances if given.
    The pool is closed and joined, never terminated."""
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 4 or gpu_runtime_loaded():
        out = []
        for s in seeds:
            out.append(synth.config5_arrays((s, n)))
            if log is not None and len(out) % 50 == 0:
                log(len(out))
        return out
    pool = mp.get_context("fork").Pool(min(workers, len(seeds)))
    try:
        out = pool.map(synth.config5_arrays, [(s, n) for s in seeds],
                       chunksize=max(1, len(seeds) // (4 * workers)))
    finally:
        pool.close()
        pool.join()
    return out


@dataclass
class Dataset:
    feats: torch.Tensor          # [N, 3, n, m] FP32 on the device
    phi: torch.Tensor            # [N, n, m] converged level sets, FP32 on the device
    seeds: list
    cycles: list
    dropped: list = field(default_factory=list)   # seeds whose solve did not converge


def solve_targets(instances, params: mgseg.Params, tol=1e-6, max_cycles=80, chunk=64, log=None) -> Dataset:
    """Solve every instance on the GPU (batches of `chunk` images on the
    library's internal streams) and keep (features, converged phi) pairs;
    instances that do not reach tol are dropped."""
    feats, phis, seeds, cycles, dropped = [], [], [], [], []
    for c0 in range(0, len(instances), chunk):
        part = instances[c0:c0 + chunk]
        b = mgseg.Batch([p[0] for p in part], [p[1] for p in part], params)
        b.set_streams(8)
        cyc, rel, _ = b.solve(tol, max_cycles)
        for i, (img, mk, seed) in enumerate(part):
            if not rel[i] <= tol:
                dropped.append(seed)
                continue
            v = b.image(i)
            feats.append(v.features())
            phis.append(v.phi().float())
            seeds.append(seed)
            cycles.append(cyc[i])
        b.close()
        if log:
            log(f"targets {min(c0 + chunk, len(instances))}/{len(instances)} kept {len(seeds)}")
    return Dataset(torch.stack(feats), torch.stack(phis), seeds, cycles, dropped)


def object_weight(data: Dataset) -> float:
    """sqrt(background / object) pixel ratio of the targets: the loss weight of
    object pixels, so that the few object pixels (a few percent of an image)
    are not outweighed into the empty level set."""
    f = float((data.phi > 0).float().mean())
    f = min(max(f, 1e-6), 1 - 1e-6)
    return float(np.sqrt((1 - f) / f))


def train(net: mgseg.Net, data: Dataset, M: float, epochs=10, batch=8, lr=1e-3, lr_final=None, seed=0,
          pos_weight=None, log=None):
    """Adam on the network's weighted cross-entropy against phi / M (object
    weight pos_weight, default object_weight(data)) over shuffled
    mini-batches, the step size falling from lr to lr_final (default lr / 20)
    along a half cosine; returns the mean loss of every epoch."""
    g = torch.Generator().manual_seed(seed)
    N = data.feats.shape[0]
    pw = object_weight(data) if pos_weight is None else pos_weight
    lr_final = lr / 20 if lr_final is None else lr_final
    steps = max(1, epochs * (N // batch))
    hist, k = [], 0
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g)
        tot, cnt = 0.0, 0
        for s in range(0, N - batch + 1, batch):
            idx = perm[s:s + batch].to(data.feats.device)
            x = data.feats.index_select(0, idx)
            t = data.phi.index_select(0, idx)
            net.forward(x, M)
            tot += net.backward(t, M, pw)
            net.adam_step(lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * k / steps)))
            k += 1
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.5f}")
    return hist


def _timed_solve(s: mgseg.Solver, tol_abs, max_cycles, prep=None):
    """Wall time (ms) of prep() plus a solve to absolute residual tol_abs."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if prep is not None:
        prep()
    res0 = s.scalars()["res0"]
    cyc, rel, ok = s.solve(max(tol_abs / res0, 1e-300), max_cycles) if res0 > tol_abs else (0, res0, True)
    torch.cuda.synchronize()
    return dict(ms=1e3 * (time.perf_counter() - t0), cycles=cyc, res0=res0, res=rel * res0 if cyc else res0,
                converged=bool(ok))


def evaluate(net: mgseg.Net | None, instances, params: mgseg.Params, tol=1e-6, max_cycles=80, zero=True, scale=1.0):
    """Per instance: the marker-based phi0 (the method without the network),
    the network's phi0 times `scale` (taken only if it holds every marker,
    else the marker start) and (if `zero`) phi0 = 0, each solved to the same absolute
    residual; also the share of pixels whose final masks differ from the
    marker-based solve's (a start that reaches the residual at another fixed
    point, e.g. the empty level set, has not reached equal accuracy)."""
    out = []
    for img, mk, seed in instances:
        s = mgseg.Solver(img, mk, params)
        r0 = s.scalars()["res0"]
        tol_abs = tol * r0
        row = dict(seed=seed, res0_marker=r0)
        row["marker"] = _timed_solve(s, tol_abs, max_cycles)
        ref_mask = s.mask()
        if net is not None:
            acc = []
            row["learned"] = _timed_solve(s, tol_abs, max_cycles, prep=lambda: acc.append(s.predict_phi0(net, scale)))
            row["learned"]["accepted"] = acc[0]
            row["learned"]["mask_diff"] = float((s.mask() != ref_mask).float().mean())
        if zero:
            z = torch.zeros((s.n, s.m), dtype=torch.float32, device="cuda")
            row["zero"] = _timed_solve(s, tol_abs, max_cycles, prep=lambda: s.set_phi0(z))
            row["zero"]["mask_diff"] = float((s.mask() != ref_mask).float().mean())
        s.close()
        out.append(row)
    return out


def summarize(rows):
    """Means over instances of cycles and milliseconds for every start."""
    summ = {}
    for key in ("marker", "learned", "zero"):
        rs = [r[key] for r in rows if key in r]
        if not rs:
            continue
        summ[key] = dict(cycles=float(np.mean([r["cycles"] for r in rs])),
                         ms=float(np.mean([r["ms"] for r in rs])),
                         converged=int(sum(r["converged"] for r in rs)), count=len(rs))
        if "mask_diff" in rs[0]:
            summ[key]["mask_diff"] = float(np.mean([r["mask_diff"] for r in rs]))
            summ[key]["same_fixed_point"] = int(sum(r["mask_diff"] <= 1e-4 for r in rs))
        if "accepted" in rs[0]:
            summ[key]["accepted"] = int(sum(r["accepted"] for r in rs))
    return summ


def choose_scale(net: mgseg.Net, instances, params: mgseg.Params, scales=(1.0, 0.5, 0.25), log=None):
    """The amplitude of the network's phi0 with the fewest mean cycles among
    those that reach the marker start's fixed point on at least as many of
    `instances` (a validation split, never the held-out set) as scale 1."""
    stats = {}
    for sc in scales:
        summ = summarize(evaluate(net, instances, params, zero=False, scale=sc))["learned"]
        stats[sc] = summ
        if log:
            log(f"scale {sc}: {summ['cycles']:.1f} cycles, {summ['same_fixed_point']}/{summ['count']} at the "
                f"marker start's fixed point")
    floor = stats[scales[0]]["same_fixed_point"]
    ok = [sc for sc in scales if stats[sc]["same_fixed_point"] >= floor]
    return min(ok, key=lambda sc: stats[sc]["cycles"])


def save(net: mgseg.Net, path, scale=1.0, optimizer=True):
    """The network's parameters (library order), its shape and the amplitude
    of its phi0, as .npz; with optimizer, also Adam's moments and step count,
    so that training can resume where it stopped."""
    p, _ = net.params()
    extra = {}
    if optimizer:
        m, v, t = net.adam_state()
        extra = dict(adam_m=m, adam_v=v, adam_steps=t)
    np.savez(path, params=p, base=net.base, depth=net.depth, scale=scale, **extra)


def load(path):
    """(network, amplitude) saved by save(), with Adam's state where saved."""
    d = np.load(path)
    net = mgseg.Net(int(d["base"]), int(d["depth"]))
    net.set_params(d["params"])
    if "adam_m" in d:
        net.set_adam_state(d["adam_m"], d["adam_v"], int(d["adam_steps"]))
    return net, float(d["scale"]) if "scale" in d else 1.0


def main(argv=None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description="train / evaluate the warm-start network on 4-20-shape images")
    ap.add_argument("--train", type=int, default=0, help="training instances (0: load --weights)")
    ap.add_argument("--eval", type=int, default=16, help="held-out instances")
    ap.add_argument("--n", type=int, default=512, help="image side")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--depth", type=int, default=4)
    ap.add_argument("--weights", default=None, help="where to save (with --train) or load the parameters")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--json", default=None, help="write the evaluation summary here")
    ap.add_argument("--val", type=int, default=0, help="validation instances for the amplitude (0: keep it)")
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, flush=True)

    t0 = time.perf_counter()
    tr = generate(TRAIN_SEEDS[:a.train], a.n, a.workers) if a.train else []
    he = generate(HELDOUT_SEEDS[:a.eval], a.n, a.workers) if a.eval else []
    log(f"drew {len(tr)} training and {len(he)} held-out instances in {time.perf_counter() - t0:.1f} s")
    params = mgseg.Params(levels=synth.levels_for(a.n, a.n))
    if a.train:
        t0 = time.perf_counter()
        data = solve_targets(tr, params, log=log)
        log(f"targets: {len(data.seeds)} kept, {len(data.dropped)} not converged, "
            f"{np.mean(data.cycles):.1f} cycles on average, {time.perf_counter() - t0:.1f} s")
        net = mgseg.Net(a.base, a.depth, 1)
        t0 = time.perf_counter()
        train(net, data, params.M, a.epochs, a.batch, a.lr, log=log)
        torch.cuda.synchronize()
        log(f"trained {a.epochs} epochs in {time.perf_counter() - t0:.1f} s")
        del data
        scale = 1.0
    else:
        net, scale = load(a.weights)
    if a.val:
        va = generate(TRAIN_SEEDS[len(TRAIN_SEEDS) - a.val:], a.n, a.workers)
        scale = choose_scale(net, va, params, log=log)
        log(f"amplitude {scale}")
    if a.weights and (a.train or a.val):
        save(net, a.weights, scale)
    if he:
        rows = evaluate(net, he, params, scale=scale)
        summ = summarize(rows)
        log(json.dumps(summ))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(dict(summary=summ, rows=rows), f, indent=1)


if __name__ == "__main__":
    main()

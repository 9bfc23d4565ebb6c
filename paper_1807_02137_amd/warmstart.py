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


def generate(seeds, n=512, workers=16):
    """Seeded 4-20-shape instances (images, markers, seeds), drawn on `workers`
    host processes that never touch the GPU: forked while this process has
    not initialised the GPU yet, else spawned (which re-imports the caller's
    main module, so that module must guard its script code)."""
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 4:
        return [synth.config5_arrays((s, n)) for s in seeds]
    method = "spawn" if torch.cuda.is_initialized() else "fork"
    with mp.get_context(method).Pool(min(workers, len(seeds))) as pool:
        return pool.map(synth.config5_arrays, [(s, n) for s in seeds],
                        chunksize=max(1, len(seeds) // (4 * workers)))


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


def train(net: mgseg.Net, data: Dataset, M: float, epochs=10, batch=8, lr=1e-3, seed=0, pos_weight=None,
          log=None):
    """Adam on mean(w (tanh(o) - phi / M)^2) (w = pos_weight on object
    pixels, default object_weight(data)) over shuffled mini-batches; returns
    the mean loss of every epoch."""
    g = torch.Generator().manual_seed(seed)
    N = data.feats.shape[0]
    pw = object_weight(data) if pos_weight is None else pos_weight
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g)
        tot, cnt = 0.0, 0
        for s in range(0, N - batch + 1, batch):
            idx = perm[s:s + batch].to(data.feats.device)
            x = data.feats.index_select(0, idx)
            t = data.phi.index_select(0, idx)
            net.forward(x, M)
            tot += net.backward(t, M, pw)
            net.adam_step(lr)
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
    res0 = s.stats()["res0"]
    cyc, rel, ok = s.solve(max(tol_abs / res0, 1e-300), max_cycles) if res0 > tol_abs else (0, res0, True)
    torch.cuda.synchronize()
    return dict(ms=1e3 * (time.perf_counter() - t0), cycles=cyc, res0=res0, res=rel * res0 if cyc else res0,
                converged=bool(ok))


def evaluate(net: mgseg.Net | None, instances, params: mgseg.Params, tol=1e-6, max_cycles=80, zero=True):
    """Per instance: the marker-based phi0 (the method without the network),
    the network's phi0 (taken only if it holds every marker, else the marker
    start) and (if `zero`) phi0 = 0, each solved to the same absolute
    residual; also the share of pixels whose final masks differ from the
    marker-based solve's (a start that reaches the residual at another fixed
    point, e.g. the empty level set, has not reached equal accuracy)."""
    out = []
    for img, mk, seed in instances:
        s = mgseg.Solver(img, mk, params)
        r0 = s.stats()["res0"]
        tol_abs = tol * r0
        row = dict(seed=seed, res0_marker=r0)
        row["marker"] = _timed_solve(s, tol_abs, max_cycles)
        ref_mask = s.mask()
        if net is not None:
            acc = []
            row["learned"] = _timed_solve(s, tol_abs, max_cycles, prep=lambda: acc.append(s.predict_phi0(net)))
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

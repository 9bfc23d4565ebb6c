"""Benchmark: time to a relative residual of 1e-6 and grid points per second
per V-cycle of the FAS V(2,2) cycle with Hybrid Smoother 2 on one GPU.

Default (the largest single-GPU configuration): one 8192 x 8192 image of 200
star polygons (seed 4000), 14 grids down to 1 x 1, FP32 cycles with the FP64
finest-grid defect correction.  One step = setup (edge detector, distance
map, initial level set, coarse maps) + V-cycles until the projected residual
of the paper's rows is at most 1e-6 of its initial value; the image is
resident in HBM before the timed region.  --workload c2 runs the 1024 x 1024
twelve-ellipse image (seed 2000, 9 grids) the same way; c3 the batch of 64
uneven images; c5 the learned warm start.

Prints one JSON line: value = grid points per second per V-cycle (finest
points x cycles / wall time), the time to tolerance, the roofline of the
finest-grid sweep kernel and the CPU oracle timed on a bounded sample.

Roofline: one directional sweep must move at least 21 B per cell (read the
state, psi, w, the fit map and F, 4 B each, and the label byte; write the
state, 4 B): algorithmic bytes = 21 x cells per launch, over the average
launch time from HIP events on the solver's stream.  (The design's own
traffic, with stored face coefficients and bounds, is 37 B per cell; it is
reported beside as design_bytes_per_launch.)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0          # dense bf16 matrix-core peak
WEIGHTS = os.path.join(ROOT, "paper_1807_02137_amd", "weights", "warmstart_512_b32_d4.npz")
TRAFFIC_FILES = {"c2": os.path.join(ROOT, "profiles", "k_sweep_1024x1024_traffic.json"),
                 "c4": os.path.join(ROOT, "profiles", "k_sweep_long_8192x8192_traffic.json")}
MODEL_NAMES = {"sc": "Spencer-Chen", "rc": "Rada-Chen", "cv": "global Chan-Vese (w = 1, no selection term)"}
# the source of the directional sweep kernels (the roofline's kernel): a counter record
# taken on other sources is not reported
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1807_02137_amd", "csrc", "mgseg_device.h")]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload="c2"):
    """HBM bytes per finest-grid sweep launch from the recorded FETCH_SIZE /
    WRITE_SIZE counters (scaled by a plain copy of known size), or None when
    the kernel sources have changed since they were taken."""
    try:
        with open(TRAFFIC_FILES[workload]) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


def calibrate_copy(mib: int = 1024):
    """One plain device-to-device copy of `mib` MiB (read + write of that many
    bytes): the reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 4}))


def copy_bandwidth(mib: int = 1024, reps: int = 5) -> float:
    """GB/s of a plain device-to-device copy of `mib` MiB (read + write counted),
    best of `reps`: the bandwidth a streaming kernel reaches on this GPU."""
    import torch
    a = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    return best


SEED = 2000
N = 1024
SMOOTHERS = {"hs2": (0, "Hybrid Smoother 2"), "gslex": (1, "GSLEX-I"), "hs1": (2, "Hybrid Smoother 1"),
             "gsline": (3, "GSLINE-I"), "newt": (4, "NEWT-I"), "gslex2": (5, "GSLEX-II"),
             "gsline2": (6, "GSLINE-II"), "newt2": (7, "NEWT-II")}
LEVELS = 9
TOL = 1e-6
MAX_CYCLES = 80
BATCH_MAX_CYCLES = 150      # the batch's slowest images need about 100 cycles (the oracle: 93 and 99)


def batch_bench(count: int):
    """64 images, sides 32 round(exp(U[ln 256, ln 2048]) / 32), each solved to
    1e-6: throughput of the tuned multi-stream batch and of one stream."""
    import torch
    from paper_1807_02137_amd import build, mgseg, synth
    if not os.path.exists(build.LIB):
        build.build()
    torch.cuda.set_device(0)
    insts = [synth.config3(k) for k in range(count)]
    print(f"batch: {count} images generated", file=sys.stderr, flush=True)
    px = [i.image.shape[0] * i.image.shape[1] for i in insts]
    out = {}
    for mode in ("tuned", "one_stream"):
        b = mgseg.Batch([i.image for i in insts], [i.markers for i in insts], mgseg.Params(levels=0))
        torch.cuda.synchronize()
        if mode == "tuned":
            S, ms = b.tune(1)
        else:
            b.set_streams(1)
            S, ms = 1, None
        before = [b.image(k).stats()["cycles"] for k in range(count)]
        t0 = time.perf_counter()
        cyc, rel, ok = b.solve(1e-6, BATCH_MAX_CYCLES)
        wall = time.perf_counter() - t0
        done = [c - c0 for c, c0 in zip(cyc, before)]
        out[mode] = {"streams": S, "tune_ms_per_round": ms, "wall_s": wall, "converged": ok,
                     "value": sum(p * d for p, d in zip(px, done)) / wall, "cycles": cyc}
        print(f"batch {mode}: {S} streams, {wall:.2f} s", file=sys.stderr, flush=True)
        b.close()
    print(json.dumps({
        "metric": "grid-pts/s per V-cycle, batch of uneven images (solve to rel. residual 1e-6)",
        "value": out["tuned"]["value"], "unit": "grid-pts/s per V-cycle", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{count} images, sides 256-2048 (multiples of 32), 3 shapes each, "
                               f"Spencer-Chen, FAS V(2,2), Hybrid Smoother 2, tol 1e-6, at most {BATCH_MAX_CYCLES} cycles",
                   "total_px": sum(px), "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
        "tuned": out["tuned"], "one_stream": out["one_stream"],
        "speedup_vs_one_stream": out["tuned"]["value"] / out["one_stream"]["value"]}))


def warmstart_bench(steps: int, warmup: int, count: int):
    """Learned warm start on 512x512 images of 4-20 shapes (held-out seeds).

    One step = for each of `count` held-out images: setup, the network's
    phi0 (features + forward pass + marker check), and V-cycles until the
    finest residual is at most 1e-6 times that of the marker-based phi0 (the
    same absolute accuracy as the plain solve).  The plain (marker phi0) and
    phi0 = 0 starts are timed the same way for comparison, and the share of
    images whose final segmentation equals the plain solve's is reported.
    The roofline is that of the convolution kernel (k_conv) over a forward
    and a training step of 8 images, timed with HIP events per launch."""
    import numpy as np
    import torch
    from paper_1807_02137_amd import build, mgseg, synth, warmstart
    if not os.path.exists(build.LIB):
        build.build()
    inst = warmstart.generate(warmstart.HELDOUT_SEEDS[:count], 512, workers=1,   # no fork from this process
                              log=lambda k: print(f"c5: {k} held-out images drawn", file=sys.stderr, flush=True))
    print(f"c5: {count} held-out images drawn", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    net, scale = warmstart.load(WEIGHTS)
    params = mgseg.Params(levels=synth.levels_for(512, 512))
    stream = torch.cuda.current_stream()
    zeros = torch.zeros((512, 512), dtype=torch.float32, device="cuda")
    imgs = [(torch.from_numpy(i).to("cuda"), mk) for i, mk, _ in inst]

    def solve_one(img, mk, start):
        s = mgseg.Solver(img, mk, params, stream=stream)
        r0 = s.scalars()["res0"]
        taken = None
        if start == "learned":
            taken = s.predict_phi0(net, scale)
        elif start == "zero":
            s.set_phi0(zeros)
        res0 = s.scalars()["res0"]
        cyc, ok = 0, True
        if res0 > TOL * r0:
            cyc, _, ok = s.solve(TOL * r0 / res0, MAX_CYCLES)
        mask = s.mask()
        s.close()
        return cyc, ok, mask, taken

    res = {}
    for start in ("marker", "learned", "zero"):
        for _ in range(warmup):
            for img, mk in imgs:
                solve_one(img, mk, start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = []
        for _ in range(steps):
            runs = [solve_one(img, mk, start) for img, mk in imgs]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[start] = dict(wall=wall, runs=runs)
        print(f"c5 {start}: {wall / steps * 1e3:.1f} ms per pass", file=sys.stderr, flush=True)
    ref = [r[2] for r in res["marker"]["runs"]]

    def summary(start):
        runs = res[start]["runs"]
        same = [bool((r[2] == m).all()) for r, m in zip(runs, ref)]
        out = {"ms_per_image": res[start]["wall"] / (steps * count) * 1e3,
               "cycles": [r[0] for r in runs], "mean_cycles": float(np.mean([r[0] for r in runs])),
               "converged": int(sum(r[1] for r in runs)), "same_segmentation_as_plain": int(sum(same))}
        if start == "learned":
            out["network_phi0_taken"] = int(sum(bool(r[3]) for r in runs))
        return out

    # convolution roofline: forward and training step on 8 held-out images
    feats = []
    for img, mk in imgs[:8]:
        s = mgseg.Solver(img, mk, params, stream=stream)
        feats.append(s.features())
        s.close()
    x = torch.stack(feats)
    net.forward(x, params.M)
    torch.cuda.synchronize()
    net.profile(True)
    net.forward(x, params.M)
    f_ms, f_n, f_fl = net.profile_read()
    tgt = torch.zeros((x.shape[0], 512, 512), dtype=torch.float32, device="cuda")
    net.backward(tgt, params.M)                     # warm the backward buffers
    net.profile(True)
    net.forward(x, params.M)
    net.backward(tgt, params.M)
    b_ms, b_n, b_fl = net.profile_read()
    net.profile(False)
    achieved = f_fl / (f_ms * 1e-3) / 1e12
    plain, learned = summary("marker"), summary("learned")
    print(json.dumps({
        "metric": "time to the plain solve's residual (1e-6 of the marker start's), learned warm start",
        "value": learned["ms_per_image"], "unit": "ms per 512x512 image", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": learned["ms_per_image"] * count, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 network + f32/f64 solve", "data": "synthetic",
        "config": {"workload": f"{count} held-out 512x512 images of 4-20 shapes (seeds "
                               f"{warmstart.HELDOUT_SEEDS.start}..{warmstart.HELDOUT_SEEDS.start + count - 1}), "
                               "8 grids, network base 32 depth 4, amplitude %.2f" % scale},
        "learned": learned, "plain": plain, "zero": summary("zero"),
        "speedup_vs_plain": plain["ms_per_image"] / learned["ms_per_image"],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_conv (bf16 implicit-GEMM 3x3 convolution), forward pass of 8 images",
                     "launches": f_n, "avg_us": f_ms / max(f_n, 1) * 1e3, "flops_per_launch": f_fl / max(f_n, 1)},
        "training_step": {"conv_launches": b_n, "conv_ms": b_ms, "conv_tflops": b_fl / (b_ms * 1e-3) / 1e12},
    }))


SWEEP_BYTES_PER_PX = 21.0      # compulsory FP32 bytes per cell of one directional sweep (see module doc)
C4_SEED, C4_N, C4_LEVELS, C4_MAX_CYCLES = 4000, 8192, 14, 300


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            return next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown CPU"


def oracle_sample(image, markers, levels, seconds, **kw):
    """The FP64 oracle (single-threaded C) timed on the host: setup, then whole
    V-cycles until `seconds` have passed.  Returns grid-pts/s per V-cycle (setup
    included in the time) and a description."""
    from oracle import Oracle, OracleParams
    from oracle.core import OPT_FLAGS
    t0 = time.perf_counter()
    o = Oracle(image, markers, OracleParams(levels=levels, **kw))
    k = 0
    while True:
        o.vcycle()
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    tc = time.perf_counter() - t0
    n, m = image.shape
    return n * m * k / tc, k, tc, f"single-threaded FP64 C, gcc {' '.join(OPT_FLAGS)}, {host_cpu()}"


def large_bench(steps: int, warmup: int, max_cycles: int, cpu_seconds: float, no_cpu: bool):
    """The 8192 x 8192 solve (the largest single-GPU configuration): 200 star
    polygons (seed 4000), 8 markers, 14 grids down to 1 x 1, FP32 cycles with
    the FP64 finest residual, to a relative residual of 1e-6 of the paper's
    rows.  One step = setup + solve, the image resident in HBM."""
    import torch
    from paper_1807_02137_amd import build, mgseg, synth
    if not os.path.exists(build.LIB):
        build.build()
    t0 = time.perf_counter()
    inst = synth.config4(C4_SEED, C4_N)
    print(f"c4: image drawn in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    n = inst.image.shape[0]
    img = torch.from_numpy(inst.image).to("cuda")
    params = mgseg.Params(levels=C4_LEVELS)
    stream = torch.cuda.current_stream()

    def step():
        s = mgseg.Solver(img, inst.markers, params, stream=stream)
        cyc, rel, ok = s.solve(TOL, max_cycles)
        st = s.stats()
        s.close()
        return cyc, rel, ok, st

    for _ in range(warmup):
        step()
    cycles, rels, oks, sts = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cyc, rel, ok, st = step()
        cycles.append(cyc); rels.append(rel); oks.append(ok); sts.append(st)
        print(f"c4: solve {len(cycles)}: {cyc} cycles, rel {rel:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # finest-sweep timing: HIP events around every finest-grid sweep launch on
    # the solver's stream over one more whole solve (eager launches, outside the
    # timed region), so that the average covers the same launches as a kernel
    # trace of one solve
    s = mgseg.Solver(img, inst.markers, params, stream=stream)
    s.profile(True)
    s.solve(TOL, max_cycles)
    prof_ms, prof_n, design_bytes = s.profile_read()
    s.close()
    avg_ms = prof_ms / max(prof_n, 1)
    alg_bytes = SWEEP_BYTES_PER_PX * n * n
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9 if prof_n else 0.0
    copy = copy_bandwidth()
    cpu = None
    if not no_cpu:
        sample = synth.config4(C4_SEED, 2048)
        v, k, tc, how = oracle_sample(sample.image, sample.markers, 12, cpu_seconds)
        cpu = {"value": v, "unit": "grid-pts/s per V-cycle", "cores": 1, "kind": "oracle",
               "sample": f"oracle setup + {k} V-cycles ({tc:.1f} s) of the same recipe drawn at 2048 x 2048 "
                         f"(12 grids), {how}"}
    st = sts[-1]
    print(json.dumps({
        "metric": "time to rel. residual 1e-6 + grid-pts/s per V-cycle (%HBM peak)",
        "value": n * n * sum(cycles) / wall, "unit": "grid-pts/s per V-cycle", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "8192x8192 image of 200 star polygons (blur 1.5, noise 0.05), 8 markers, "
                               "Spencer-Chen, FAS V(2,2), 14 grids (1x1 coarsest), Hybrid Smoother 2, "
                               "FP32 cycles + FP64 finest residual, tol 1e-6", "seed": C4_SEED},
        "time_to_tol_ms": wall / steps * 1e3,
        "cycles_per_solve": cycles, "rel_res": rels, "rel_res_rows": st["rel_res_rows"], "converged": all(oks),
        "ms_per_cycle": wall / max(sum(cycles), 1) * 1e3,
        "segmentation": {"foreground_share": st["frac_fg"], "jump_set_share": st["frac_D"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("c4"),
                     "copy_gbs": copy, "frac_of_copy": achieved / copy,
                     "kernel": "k_sweep_long (finest-grid directional sweep, 8192-cell lines; one sweep is two "
                               "launches, and a reverse sweep's output one tiled transpose more)",
                     "launches": prof_n, "unit_of_launch": "one sweep", "avg_us": avg_ms * 1e3,
                     "bytes_per_launch": alg_bytes,
                     "bytes_per_px": SWEEP_BYTES_PER_PX, "design_bytes_per_launch": design_bytes},
        "cpu_baseline": cpu,
    }))


# compulsory bytes of one AOS step per pixel: read phi (FP64), w and d (FP64), the
# image (FP32); write phi (FP64)
AOS_BYTES_PER_PX = 8 + 16 + 4 + 8


def aos_bench(args, img, inst, params, stream):
    """The AOS time stepper on the 1024x1024 image, run to the paper's relative-change
    stop; its segmentation is compared with the multigrid solve of the same image."""
    import torch

    from paper_1807_02137_amd import mgseg
    s = mgseg.Solver(img, inst.markers, params, stream=stream)
    s.solve(TOL, MAX_CYCLES)
    ref = s.get("phi64") > 0
    s.close()

    def step():
        s = mgseg.Solver(img, inst.markers, params, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, eta, rel, ok = s.aos(args.aos_tau, args.aos_eta, 5000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        seg = s.get("phi64") > 0
        s.close()
        return it, eta, rel, ok, t1 - t0, seg

    for _ in range(args.warmup):
        step()
    runs = [step() for _ in range(args.steps)]
    wall = sum(r[4] for r in runs)
    iters = [r[0] for r in runs]
    seg = runs[-1][5]
    iou = float((seg & ref).sum() / max((seg | ref).sum(), 1))
    npts = N * N
    ms_step = wall / max(sum(iters), 1) * 1e3
    achieved = AOS_BYTES_PER_PX * npts / (ms_step * 1e-3) / 1e9
    out = {
        "metric": "time to relative change 1e-4 (AOS) + grid-pts/s per AOS step",
        "value": npts * sum(iters) / wall,
        "unit": "grid-pts/s per AOS step",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"1024x1024 12-ellipse image, 6 markers, {MODEL_NAMES[args.model]}, AOS "
                               f"tau {args.aos_tau} h/mu, stop at relative change {args.aos_eta}",
                   "seed": SEED, "parallelism": "single GPU"},
        "aos_steps": iters, "eta": [r[1] for r in runs], "rel_res_paper": [r[2] for r in runs],
        "converged": all(r[3] for r in runs),
        "iou_vs_multigrid": iou,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "one whole AOS step (coefficients, column and row Thomas solves, combine, "
                               "region means, change)",
                     "bytes_per_px": AOS_BYTES_PER_PX, "avg_us": ms_step * 1e3},
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain copy of known size (counter calibration) and exit")
    ap.add_argument("--workload", default="c4", choices=("c2", "c3", "c4", "c5"),
                    help="c4: the 8192x8192 solve (default, the largest single-GPU configuration); c2: the "
                         "1024x1024 solve; c3: the 64-image batch of uneven sizes; c5: the learned warm start "
                         "on 512x512 held-out images")
    ap.add_argument("--model", default="sc", choices=("sc", "rc", "cv"),
                    help="c2 only: Spencer-Chen (default), Rada-Chen or the global Chan-Vese workload")
    ap.add_argument("--smoother", default="hs2", choices=tuple(SMOOTHERS),
                    help="c2 only: Hybrid Smoother 2 (default, the paper's Algorithm 3), Hybrid Smoother 1 "
                         "(its Algorithm 2) or a standard smoother of its Algorithm 1 (gslex, gsline, newt: "
                         "the -I variants; gslex2, gsline2, newt2: the local -II variants)")
    ap.add_argument("--solver", default="mg", choices=("mg", "aos"),
                    help="c2 only: the FAS multigrid (default) or the AOS time stepper the paper compares "
                         "against (Sec. 5), run to the relative change --aos-eta")
    ap.add_argument("--aos-tau", type=float, default=200.0, help="AOS time step in units of h/mu")
    ap.add_argument("--aos-eta", type=float, default=1e-4, help="AOS stop: relative change of phi")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--c5-images", type=int, default=16)
    ap.add_argument("--max-cycles", type=int, default=C4_MAX_CYCLES, help="c4 only: cycle cap of a solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: libmgseg runs on one GPU (asked for --gpus {args.gpus}); "
              "sharding a solve or a batch over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "c3":
        # the batch's streams run side by side only on as many hardware queues as the HIP
        # runtime opens (read when it starts, before any device call; HIP's default is 4)
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 16:
            os.environ["GPU_MAX_HW_QUEUES"] = "16"
        batch_bench(args.batch_count)
        return
    if args.workload == "c5":
        warmstart_bench(args.steps, args.warmup, args.c5_images)
        return
    if args.workload == "c4":
        large_bench(args.steps, args.warmup, args.max_cycles, args.cpu_seconds, args.no_cpu_baseline)
        return
    import torch

    from paper_1807_02137_amd import build, mgseg, synth
    if not os.path.exists(build.LIB):
        build.build()
    torch.cuda.set_device(0)
    inst = synth.config2(SEED, N)
    img = torch.from_numpy(inst.image).to("cuda")
    model = 1 if args.model == "rc" else 0
    smoother = SMOOTHERS[args.smoother][0]
    params = (mgseg.chan_vese_params(levels=LEVELS, smoother=smoother) if args.model == "cv"
              else mgseg.Params(levels=LEVELS, model=model, smoother=smoother))
    stream = torch.cuda.current_stream()

    if args.solver == "aos":
        aos_bench(args, img, inst, params, stream)
        return

    def step(profile=False):
        s = mgseg.Solver(img, inst.markers, params, stream=stream)
        if profile:
            s.profile(True)
        cyc, rel, ok = s.solve(TOL, MAX_CYCLES)
        prof = s.profile_read() if profile else None
        s.close()
        return cyc, rel, ok, prof

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles, rels, oks = [], [], []
    for _ in range(args.steps):
        cyc, rel, ok, _ = step()
        cycles.append(cyc); rels.append(rel); oks.append(ok)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    # kernel timing: one more solve outside the timed region, launched eagerly
    # with HIP events around every finest-grid sweep on the solver's stream
    _, _, _, prof = step(profile=True)
    prof_ms, prof_n, design_bytes = prof
    npts = N * N
    value = npts * sum(cycles) / wall
    avg_ms = prof_ms / max(prof_n, 1)
    prof_bytes = SWEEP_BYTES_PER_PX * npts
    achieved = prof_bytes / (avg_ms * 1e-3) / 1e9 if prof_n else 0.0
    copy = copy_bandwidth()
    rates = smoothing_rate_table(img, inst, params, stream) if args.model != "cv" else None

    cpu = None
    if not args.no_cpu_baseline:
        okw = dict(mgseg.CHAN_VESE) if args.model == "cv" else {"model": model}
        okw["smoother"] = smoother
        v, k, tc, how = oracle_sample(inst.image, inst.markers, LEVELS, args.cpu_seconds, **okw)
        cpu = {"value": v, "unit": "grid-pts/s per V-cycle", "cores": 1, "kind": "oracle",
               "sample": f"oracle setup + {k} V-cycles of the same 1024x1024 image ({tc:.1f} s), {how}"}

    out = {
        "metric": "time to rel. residual 1e-6 + grid-pts/s per V-cycle (%HBM peak)",
        "value": value,
        "unit": "grid-pts/s per V-cycle",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "1024x1024 12-ellipse image, 6 markers, "
                               f"{MODEL_NAMES[args.model]}, FAS V(2,2), "
                               f"9 grids, {SMOOTHERS[args.smoother][1]}, tol 1e-6",
                   "seed": SEED,
                   "parallelism": "single GPU"},
        "cycles_per_solve": cycles,
        "rel_res": rels,
        "converged": all(oks),
        "time_to_tol_ms": wall / args.steps * 1e3,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("c2") if args.model == "sc" and not smoother else None,
                     "copy_gbs": copy, "frac_of_copy": achieved / copy,
                     "kernel": "k_sweep (finest-grid directional sweep; a forward sweep is two launches)",
                     "launches": prof_n, "unit_of_launch": "one sweep", "avg_us": avg_ms * 1e3,
                     "bytes_per_launch": prof_bytes,
                     "bytes_per_px": SWEEP_BYTES_PER_PX, "design_bytes_per_launch": design_bytes},
        "cpu_baseline": cpu,
        "smoothing_rates": rates,
    }
    print(json.dumps(out))


def smoothing_rate_table(img, inst, params, stream):
    """Table 1's measurement on this image: the local Fourier analysis of each
    smoother over every pixel at the solved phi (mu~_max, mu~_avg, and the same
    over the jump set), with the analysis kernel's time."""
    import torch

    from paper_1807_02137_amd import mgseg
    s = mgseg.Solver(img, inst.markers, params, stream=stream)
    s.solve(TOL, MAX_CYCLES)
    out = {}
    for name, k in (("GSLEX-I", 1), ("GSLINE-I", 3), ("NEWT-I", 4), ("Hybrid Smoother 2", 0)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        agg, _ = s.smoothing_rates(k)
        torch.cuda.synchronize()
        agg["ms"] = (time.perf_counter() - t0) * 1e3
        out[name] = agg
    s.close()
    return out


if __name__ == "__main__":
    main()

"""Throughput of the damped-acoustic forward propagator on one MI355X.

One bench step = one full forward modelling run of the workload (every time
step: stencil + leapfrog + damping, fused source injection and receiver
sampling), inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workloads (seeded synthetic layered models, sponge, Ricker source):
  3d-256-o8   256^3, space order 8, 1000 steps, 128x128 receivers (default;
              `value` is this one)
  3d-512-o16  512^3, space order 16, 2000 steps, 256x256 receivers (the
              roofline benchmark; also reported as its own leg of the default
              run, with its own roofline block)
Further legs of the default run: the FWI gradient (200^3, checkpointed,
FP32/BF16/FP16 snapshots) against the plain forward, 48 batched 2D shots
against the single-shot path (with the batch kernel's own roofline block),
the paper's diffusion example, and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpts/s (grid-point updates/sec) + % HBM roofline; FWI gradient sec/shot vs plain"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 20     # read u^n, u^{n-1}, alpha, beta; write u^{n+1} (FP32)


def make_workload(name):
    from paper_1609_03361_amd import synth
    if name == "3d-256-o8":
        return synth.config_3d_o8()
    if name == "3d-512-o16":
        return synth.config_3d_o16()
    raise SystemExit(f"unknown workload {name}")


STEP_SOURCES = ("wave_step.h", "wave_internal.h")


def step_kernel_sha():
    """Hash of the step kernel's sources (the templates and the argument layout)."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1609_03361_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, tile):
    """HBM bytes per step launch from the committed rocprofv3 --pmc summary
    (FETCH_SIZE and WRITE_SIZE scaled by the plain-copy calibration), or None
    when the step kernel's source has changed since the counters were taken
    or the launch runs another tile than the one they were taken on."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != step_kernel_sha() or rec.get("tile") != tile:
        return None
    return rec["hbm_bytes_per_launch"]


def forward_leg(dev, p, steps, warmup, tile=0):
    """Time `steps` forward runs of problem p (after `warmup`): whole-job
    Gpts/s from torch events around the runs, and the step kernel's average
    launch time from the library's HIP events around each time loop (on the
    stream the kernel runs on)."""
    import torch
    from paper_1609_03361_amd import api, _lib
    geom = api.Geometry(p.shape, p.spacing, p.order, p.dt, p.nt, p.src, p.rec)
    m = torch.from_numpy(p.m).to(dev)
    eta = torch.from_numpy(p.eta).to(dev)
    q = torch.from_numpy(p.q).to(dev)
    for _ in range(warmup):
        api.forward(geom, m, eta, q, tile=tile)
    torch.cuda.synchronize()
    _lib.set_profiling(True)
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    loop_ms, launches = 0.0, 0
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        api.forward(geom, m, eta, q, tile=tile)
        ms, n = _lib.last_loop()          # waits for this run's loop to end
        loop_ms += ms
        launches += n
    e1.record(stream)
    torch.cuda.synchronize()
    _lib.set_profiling(False)
    total_ms = e0.elapsed_time(e1)
    per_launch_ms = loop_ms / launches
    alg_bytes = BYTES_PER_UPDATE * p.npoints
    achieved = alg_bytes / (per_launch_ms * 1e-3) / 1e9
    resolved = api.resolve_tile(geom, tile)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(p.name, resolved),
            "kernel": "leapfrog step", "launch_ms": round(per_launch_ms, 5),
            "alg_bytes_per_launch": alg_bytes, "tile": resolved}
    return total_ms, roof


def cpu_baseline(p, steps):
    """The FP64 oracle on the host cores, on the first `steps` time steps of
    the same workload (full grid)."""
    import oracle
    t0 = time.perf_counter()
    oracle.forward(p.shape, p.spacing, p.order, p.dt, steps, p.m, p.eta, p.src,
                   p.q[:steps], p.rec, want_final=False)
    el = time.perf_counter() - t0
    return {"value": p.npoints * steps / el / 1e9, "unit": "Gpts/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{'x'.join(map(str, p.shape))} grid, order {p.order}, first {steps} of "
                      f"{p.nt} time steps, FP64, {el:.1f} s"}


def copy_calibration():
    """A plain device-to-device copy of 256 MiB, ten times: reads and writes
    exactly 256 MiB each per launch, the reference for the HBM byte counters."""
    import torch
    n = 64 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 4, "launches": 10}), flush=True)


def gradient_bench(dev, reps=2):
    """FWI gradient on the 200^3 order-8 workload (1500 steps, 4 shots,
    checkpoints every 20 steps): seconds per shot of the checkpointed
    gradient (FP32 / BF16 / FP16 snapshots) against the plain forward."""
    import torch
    from paper_1609_03361_amd import api, synth
    m0, m_true, eta, shots = synth.config_gradient_3d()
    m = torch.from_numpy(m0).to(dev)
    mt = torch.from_numpy(m_true).to(dev)
    e = torch.from_numpy(eta).to(dev)
    geoms = [api.Geometry(p.shape, p.spacing, p.order, p.dt, p.nt, p.src, p.rec) for p in shots]
    qs = [torch.from_numpy(p.q).to(dev) for p in shots]
    dobs = [api.forward(g, mt, e, q) for g, q in zip(geoms, qs)]
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best / len(shots)

    fwd = timed(lambda: [api.forward(g, m, e, q) for g, q in zip(geoms, qs)])
    out = {"workload": f"3d-{shots[0].shape[0]}-o{shots[0].order}, {shots[0].nt} steps, "
                       f"{len(shots)} shots, {shots[0].rec.shape[0]} receivers, checkpoint every 20",
           "forward_s_per_shot": round(fwd, 5)}
    for dt in ("fp32", "bf16", "fp16"):
        s = timed(lambda: [api.gradient(g, m, e, q, d, ckpt_every=20, ckpt_dtype=dt)
                           for g, q, d in zip(geoms, qs, dobs)])
        out[f"gradient_{dt}_s_per_shot"] = round(s, 5)
        out[f"gradient_{dt}_vs_forward"] = round(s / fwd, 3)
    return out


BYTES_PER_PASS = 24       # two-step pass: read u^n, u^{n-1}, alpha, beta; write two levels


def batched_bench(dev, reps=2, nt=0, full=True, tile=0):
    """48 2D shots of uneven aperture on a 2001 x 801 layered model, order 8,
    2000 steps, launches over all shots replayed from a hipGraph, tile chosen
    by the autotuner (the two-step body advances two levels per launch);
    against the single-shot order-8 2D kernel on the full 2001 x 801 model.
    The roofline block prices the batch kernel's average launch (HIP events
    around the time loop inside the library) at its algorithmic bytes."""
    import torch
    from paper_1609_03361_amd import api, synth, _lib
    probs = synth.config_batched_2d(nt=nt) if nt > 0 else synth.config_batched_2d()
    shots = []
    for p in probs:
        geom = api.Geometry(p.shape, p.spacing, p.order, p.dt, p.nt, p.src, p.rec)
        shots.append((geom, torch.from_numpy(p.m).to(dev), torch.from_numpy(p.eta).to(dev),
                      torch.from_numpy(p.q).to(dev)))
    tune_us = None
    if tile == 0:
        tile, tune_us = api.tune_batch(shots, steps=10)
    pts = sum(p.npoints for p in probs) * probs[0].nt

    def timed(fn, reps=reps):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    tb = timed(lambda: api.forward_batch(shots, tile=tile))
    # one more run with the library's loop events: the average launch
    _lib.set_profiling(True)
    api.forward_batch(shots, tile=tile)
    loop_ms, launches = _lib.last_loop()
    _lib.set_profiling(False)
    two = (tile >> 16) == 4
    npts = sum(p.npoints for p in probs)
    passes = probs[0].nt // 2 if two else probs[0].nt
    per_launch_ms = loop_ms / passes     # two-step: the launches that advance two levels
    alg = (BYTES_PER_PASS if two else BYTES_PER_UPDATE) * npts
    achieved = alg / (per_launch_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            # counters were taken on the two-step body with columns of 64 rows
            "traffic": measured_traffic("batch2d-o8", tile) if nt == 0 else None,
            "kernel": "two-step pass (levels n+1, n+2)" if two else "leapfrog step",
            "launch_ms": round(per_launch_ms, 5), "alg_bytes_per_launch": alg,
            "launches_in_loop": launches}
    if not full:
        return {"batched_gpts": round(pts / tb / 1e9, 2), "batched_s": round(tb, 4),
                "tile": {"variant": tile >> 16, "xchunk": tile & 0xffff}, "roofline": roof}
    tp = timed(lambda: api.forward_batch(shots, tile=tile, persistent=True), reps=1)
    # the same model as one shot, through the single-shot path
    m_full, _ = synth.layered((2001, 801), 4)
    vmax = float(np.max(1.0 / np.sqrt(m_full.astype(np.float64))))
    eta_full = synth.sponge(m_full, 10.0, 40, vmax)
    p0 = probs[0]
    geom = api.Geometry(m_full.shape, p0.spacing, p0.order, p0.dt, p0.nt,
                        np.array([[1000 * 10.0, 25.0]]), synth.line_receivers(400, 20000.0, 20.0))
    mf = torch.from_numpy(m_full).to(dev)
    ef = torch.from_numpy(eta_full).to(dev)
    ts = timed(lambda: api.forward(geom, mf, ef, shots[0][3]))
    single = m_full.size * p0.nt / ts / 1e9
    batched = pts / tb / 1e9
    return {"workload": f"{len(probs)} 2D shots, widths {min(p.shape[0] for p in probs)}-"
                        f"{max(p.shape[0] for p in probs)} x 801, order 8, {p0.nt} steps",
            "batched_gpts": round(batched, 2), "batched_s": round(tb, 4),
            "mode": ("two-step launches (levels n+1, n+2) over all shots" if two else
                     "per-step launches over all shots") + ", replayed from a hipGraph",
            "persistent_single_launch_s": round(tp, 4),
            "tile": {"variant": tile >> 16, "xchunk": tile & 0xffff,
                     "tuned_us_per_step": None if tune_us is None else round(tune_us, 2)},
            "roofline": roof,
            "persistent_mode": api.last_batch_mode(),
            "single_shot_full_model_gpts": round(single, 2),
            "batched_vs_single": round(batched / single, 3)}


def diffusion_bench(dev, reps=3):
    """The paper's 2D diffusion example (1000 x 1000, spacing 0.001, order 2,
    500 forward-Euler steps) on the step kernel."""
    import torch
    from paper_1609_03361_amd import api
    n, h, alpha = 1000, 0.001, 0.5
    dt = h ** 4 / (2 * alpha * 2 * h ** 2)
    a = torch.full((n, n), alpha, device=dev)
    u0 = torch.randn((n, n), device=dev)
    api.diffusion((n, n), (h, h), 2, dt, 500, a, u0)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        api.diffusion((n, n), (h, h), 2, dt, 500, a, u0)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return {"workload": "2D diffusion 1000x1000, order 2, 500 steps", "seconds": round(best, 5),
            "gpts": round(n * n * 500 / best / 1e9, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="3d-256-o8")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip the FWI-gradient seconds-per-shot measurement")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched multi-shot measurement")
    ap.add_argument("--no-o16", action="store_true",
                    help="skip the 512^3 order-16 leg")
    ap.add_argument("--nt", type=int, default=0,
                    help="override the number of time steps (for short profiler runs)")
    ap.add_argument("--tile", type=int, default=0,
                    help="tile id of the main leg, or with --only-batched of the batch "
                         "(variant << 16 | x-chunk; 0 = tuned or automatic)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 10 times (HBM counter calibration)")
    ap.add_argument("--only-batched", action="store_true",
                    help="only time the batched shots (with --nt for short profiler runs)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only_batched:
        import torch
        print(json.dumps({"batched_shots": batched_bench(torch.device("cuda:0"), nt=args.nt,
                                                         full=False, tile=args.tile)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build runs on a single MI355X and has no "
              f"multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    p = make_workload(args.workload)
    if args.nt > 0:
        p.nt = args.nt
        p.q = p.q[: args.nt].copy()
    print(f"# workload {p.name}: shape {p.shape} order {p.order} nt {p.nt} "
          f"nrec {p.rec.shape[0]}", file=sys.stderr, flush=True)
    tile, tune_us = args.tile, None
    if tile == 0:
        # the library's autotuner picks the block shape and x-chunk on this
        # grid (every candidate gives bitwise the same result); set-up, outside
        # the timed region
        from paper_1609_03361_amd import api
        geom = api.Geometry(p.shape, p.spacing, p.order, p.dt, p.nt, p.src, p.rec)
        tile, tune_us = api.tune(geom, steps=10)
    total_ms, roof = forward_leg(dev, p, args.steps, args.warmup, tile)
    roof["tile_from"] = "wave_tune" if tune_us is not None else "--tile"
    if tune_us is not None:
        roof["tuned_us_per_step"] = round(tune_us, 2)
    updates = p.npoints * p.nt * args.steps
    value = updates / (total_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": p.name, "shape": list(p.shape), "space_order": p.order,
                   "time_steps": p.nt, "receivers": int(p.rec.shape[0]), "sources": 1,
                   "bench_step": "one full forward modelling run"},
        "hbm_roofline_frac": round(value * BYTES_PER_UPDATE / HBM_PEAK_GBS, 4),
        "roofline": roof,
    }
    if args.workload == "3d-256-o8" and not args.no_o16 and args.nt == 0:
        # the roofline benchmark: 512^3, order 16, 2000 steps, timed the same way
        p16 = make_workload("3d-512-o16")
        print(f"# workload {p16.name}: shape {p16.shape} order {p16.order} nt {p16.nt}",
              file=sys.stderr, flush=True)
        ms16, roof16 = forward_leg(dev, p16, 2, 1)
        out["order16_512"] = {"workload": p16.name, "time_steps": p16.nt,
                              "ms_per_run": round(ms16 / 2, 3),
                              "gpts": round(p16.npoints * p16.nt * 2 / (ms16 * 1e-3) / 1e9, 3),
                              "roofline": roof16}
        del p16
    if not args.no_gradient:
        out["fwi_gradient"] = gradient_bench(dev)
    if not args.no_batched:
        out["batched_shots"] = batched_bench(dev)
        out["diffusion"] = diffusion_bench(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

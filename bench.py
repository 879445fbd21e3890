"""Benchmark of the QMC radiative-transfer hot path on one MI355X.

One step = the whole transport of the flared-disk workload: a 128^3 FP32 mesh,
point source, up to 20 scatterings, three observers with 256^2 Stokes I/Q/U
images, and 2^22 packets for each of five point sets (Sobol, Halton,
Niederreiter-2, Hammersley with N = 2^22, Philox PRNG), FP32 rays with FP64
optical-depth and image sums.  The mesh is resident in HBM before timing.

Prints one JSON line: photon packets/s over the timed steps, the roofline of
the transport kernel (algorithmic bytes: 4 B per voxel visit + 24 B per peel
contribution, exact counts from the kernel's counters, over the kernel time
measured with HIP events on the launch stream), and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KIND_ORDER = ("sobol", "halton", "niederreiter2", "hammersley", "philox")
PHILOX_SEED = 12345


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=1 << 22, help="packets per point set per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 18, help="oracle packets per point set")
    return ap.parse_args()


def cpu_baseline(sc, n_sample: int):
    """The FP64 oracle on the host cores, on the first n_sample packets of each point set."""
    from oracle import oracle as O
    from synth import scenes
    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    for name in KIND_ORDER:
        kind = scenes.KIND_BY_NAME[name]
        O.run(sc, kind, first=1, count=n_sample, seed=PHILOX_SEED, n_total=sc.n_packets, nthreads=threads)
    dt = time.perf_counter() - t0
    total = n_sample * len(KIND_ORDER)
    return {"value": total / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sample} packets of each of the 5 point sets of the same disk128 workload "
                      f"(FP64 oracle, OpenMP over packet ranges), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the multi-GPU sharding is described in DESIGN.md)"}))
        sys.exit(2)
    import torch

    from paper_2406_15632_amd import qrt
    from synth import scenes

    qrt.load()   # raises if libqrt.so is missing: there is no fallback path
    torch.cuda.set_device(0)
    sc = scenes.disk128(n_packets=args.packets)
    grid = torch.from_numpy(sc.kappa_rho).cuda()
    stream = torch.cuda.current_stream()
    ctx = qrt.Context(0, stream.cuda_stream)
    ctx.set_scene(sc, kind=qrt.SOBOL, grid=grid)
    N = args.packets
    kinds = [scenes.KIND_BY_NAME[k] for k in KIND_ORDER]

    def step(events=None):
        for j, kind in enumerate(kinds):
            ctx.set_sequence(kind, PHILOX_SEED, N)
            if events is not None:
                events[j][0].record(stream)
            ctx.run(1, N)
            if events is not None:
                events[j][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.reset_images()
    launch_events = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in kinds]
                     for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for s in range(args.steps):
        step(launch_events[s])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    elapsed_ms = t_start.elapsed_time(t_end)
    cnt = ctx.counters()
    per_kind_ms = {KIND_ORDER[j]: sum(launch_events[s][j][0].elapsed_time(launch_events[s][j][1])
                                      for s in range(args.steps)) / args.steps for j in range(len(kinds))}
    kernel_ms = sum(per_kind_ms.values()) * args.steps
    n_launch = args.steps * len(kinds)
    alg_bytes = 4.0 * cnt["visits"] + 24.0 * cnt["peels"]
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    packets = args.steps * len(kinds) * N
    result = {
        "metric": "photon packets/s (QMC radiative transfer, disk128 workload)",
        "value": packets / (elapsed_ms * 1e-3),
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "disk128: flared disk rho~R^-2.25 exp(-z^2/2h^2), 128^3 FP32 mesh, midplane tau 10, "
                        "g 0.6, albedo 0.5, up to 20 scatterings, point source, observers at 0/45/90 deg, "
                        "256^2 I/Q/U images; per step 2^22 packets for each of sobol, halton, niederreiter2, "
                        "hammersley (N=2^22), philox; FP32 rays, FP64 optical-depth and image sums",
            "packets_per_step": len(kinds) * N,
            "sequences": list(KIND_ORDER),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_transport<float,*,point>",
            "alg_bytes_per_launch": alg_bytes / n_launch,
            "avg_launch_ms": kernel_ms / n_launch,
        },
        "per_sequence_packets_per_s": {k: N / (v * 1e-3) for k, v in per_kind_ms.items()},
        "counters_per_packet": {k: cnt[k] / cnt["packets"] for k in ("visits", "peels", "scatterings",
                                                                   "escapes", "tau_cuts")},
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sc, args.cpu_sample)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

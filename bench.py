"""Benchmark of the QMC radiative-transfer hot path on one MI355X.

One step = the whole transport of the flared-disk workload (disk128): a 128^3
FP32 mesh, point source, up to 20 scatterings, three observers with 256^2
Stokes I/Q/U images, and 2^22 packets for each of five point sets (Sobol,
Halton, Niederreiter-2, Hammersley with N = 2^22, Philox PRNG); FP32 rays with
FP64 optical-depth and image sums.  The mesh is resident in HBM before timing.

The JSON line carries
  value         photon packets/s over the timed steps (HIP events);
  roofline      of the dominant kernels, the walks (k_walk: peel-off rays and
                flights of order 1, then the peel rays of the deferred later
                scatterings; k_tail: orders 2-20 in one launch): their algorithmic
                bytes (4 B per voxel visit + 24 B per peel-off contribution,
                exact counts from the kernels' counters) over their time,
                measured with HIP events that
                the library records on its launch stream around every kernel in
                a timing pass after the timed region; the same figure for the
                whole transport step under "step"; HBM traffic from committed
                rocprofv3 counters when the kernel sources are unchanged since
                they were taken;
  time_to_error time to reach 5 %, 1 %, 0.3 % image RMS error per point set and
                the speed-up of each over the Monte Carlo (Philox) baseline;
  per_order     image error per scattering order, QMC against Monte Carlo;
  envelope_time_to_error  the same sweep for the single-scattering dust
                envelope (32^3, FP64), with the paper's single-scattering
                speed-ups quoted as context;
                (time_to_error also holds Faure's curve and the error bar of
                8 Owen-scrambled Sobol runs against their actual error)
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload;
  surrogate     the learned peel-off on the same disk scene at 2^24 packets: pilot
                sampling, GPU training and validation times, the share of
                peel-off rays the network answers, the image bias against the
                plain method, and the time to 1 % image RMS error of both;
  surrogate_resolved  the same on a thick disk (h0 = 0.3, midplane tau 1)
                on a 256^3 mesh, where peel-off rays are long and the density
                is resolved;
  workloads     packets/s of the other scenes (dust envelope 32^3 in FP64,
                clumpy envelope 256^3 with a spherical star);
  sphere_star   time to 5 % and 1 % image error for the spherical star in the
                direct and the inverse order of the point coordinates against
                Monte Carlo;
  batch         64 uneven seeded scenes in one batched launch sequence against
                the same scenes run one after another.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix-core peak
MLP_FWD_FLOP = 25344              # algorithmic FLOP of one forward pass of the surrogate network
KIND_ORDER = ("sobol", "halton", "niederreiter2", "hammersley", "philox")
PHILOX_SEED = 12345
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_disk128.txt")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_disk128.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the timed steps in stream order instead of overlapping consecutive runs")
    ap.add_argument("--timing-steps", type=int, default=3,
                    help="steps of the per-kernel timing pass (HIP events around every kernel)")
    ap.add_argument("--packets", type=int, default=1 << 22, help="packets per point set per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 21, help="oracle packets per point set")
    ap.add_argument("--no-time-to-error", action="store_true")
    ap.add_argument("--ref-log2", type=int, default=30, help="log2 packets of the reference images")
    ap.add_argument("--sweep-log2", type=int, default=26, help="largest log2 packets of the error sweep")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-workloads", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-batch-small", action="store_true", help="skip the batch of 256 small scenes")
    ap.add_argument("--no-batch-overlap", action="store_true",
                    help="time the batches in stream order only (kernel traces of whole batch runs)")
    return ap.parse_args()


def _code_only(text: str, hash_comments: bool) -> str:
    """Source text without comments and blank space (they do not change the kernels)."""
    import re
    if hash_comments:
        text = re.sub(r"#[^\n]*", "", text)
    else:
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
    return " ".join(text.split())


def transport_source_hash(root: str = ROOT) -> str:
    """Hash of the code that defines the transport kernels, comments left out
    (traffic counters taken on other code do not describe this build)."""
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_2406_15632_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            h.update(_code_only(open(os.path.join(csrc, f)).read(), False).encode())
    # the compiler flags are part of the kernels too
    h.update(_code_only(open(os.path.join(root, "paper_2406_15632_amd", "build.py")).read(), True).encode())
    return h.hexdigest()[:16]


def committed_traffic(key: str = "bytes_per_step_launch"):
    """HBM bytes per transport launch (of the whole step, or of the walk
    kernel with key "walk_bytes_per_launch") from the committed counter summary,
    or None when it is missing or was taken on other kernel sources."""
    from paper_2406_15632_amd.profile_report import read_traffic
    try:
        d = read_traffic(TRAFFIC_FILE)
    except OSError:
        return None
    if d.get("source_hash") != transport_source_hash():
        return None
    try:
        return float(d[key])
    except (KeyError, ValueError):
        return None


def committed_walk_counters():
    """The walk kernels' VALU, TA and TD busy and VALU lane share (fractions) from the committed
    counter summary, when it was taken with the committed traffic counters on the current kernel
    sources (both come from one measurement run), else None: k_walk with flights (order 1) and
    k_walk of peel rays alone (the deferred scatterings)."""
    if committed_traffic() is None:
        return None
    try:
        lines = open(COUNTERS_FILE).read().splitlines()
    except OSError:
        return None
    names = {"| `qrt::k_walk<float, true>`": "k_walk_flights", "| `qrt::k_walk<float, false>`": "k_walk_peel_rays"}
    out = {}
    for ln in lines:
        for prefix, name in names.items():
            if ln.startswith(prefix):
                cells = [c.strip() for c in ln.strip().strip("|").split("|")]
                try:
                    _, _hit, busy, lanes, _wait, ta, td = cells[:7]
                    out[name] = {"valu_busy": float(busy) / 100, "valu_lanes_active": float(lanes) / 100,
                                 "ta_busy": float(ta) / 100, "td_busy": float(td) / 100}
                except ValueError:
                    return None
    if not out:
        return None
    out["source"] = "profiles/counters_disk128.md"
    return out


def measured_copy_gbps(mib: int = 1024, reps: int = 5) -> float:
    """Bytes read plus written per second by a plain device-to-device copy of mib MiB (best of reps)."""
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    return 2.0 * mib * (1 << 20) / best / 1e9


def host_cpus():
    """The host's CPU model, nproc, the CPUs this process may run on, and the CPU
    quota of its cgroup (None when unlimited); the oracle uses min(affinity, quota)
    threads, so that a quota is not oversubscribed."""
    import math
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0))
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = max(1, math.floor(int(q) / int(period)))
    except (OSError, ValueError):
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": affinity, "cgroup_quota": quota,
            "threads": min(affinity, quota) if quota else affinity}


def cpu_baseline(sc, n_sample: int, n_single: int = 1 << 17, repeats: int = 3):
    """The FP64 oracle on the host cores, on the first n_sample packets of each
    point set (OpenMP over packet ranges, every usable core), and on the first
    n_single Sobol packets on one thread (the paper's single-core timing); the
    median of `repeats` runs for each."""
    from oracle import oracle as O
    from synth import scenes
    host = host_cpus()
    threads = host["threads"]
    for name in KIND_ORDER:   # build the generator tables outside the timing
        O.seq_tables(scenes.KIND_BY_NAME[name], sc.dims)

    def all_sets():
        t0 = time.perf_counter()
        for name in KIND_ORDER:
            kind = scenes.KIND_BY_NAME[name]
            O.run(sc, kind, first=1, count=n_sample, seed=PHILOX_SEED, n_total=sc.n_packets, nthreads=threads)
        return time.perf_counter() - t0

    def single():
        t0 = time.perf_counter()
        O.run(sc, scenes.SOBOL, first=1, count=n_single, nthreads=1)
        return time.perf_counter() - t0

    runs = sorted(all_sets() for _ in range(repeats))
    runs1 = sorted(single() for _ in range(repeats))
    dt, dt1 = runs[len(runs) // 2], runs1[len(runs1) // 2]
    total = n_sample * len(KIND_ORDER)
    return {"value": total / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sample} packets of each of the 5 point sets of the disk128 workload "
                      f"(FP64 oracle, OpenMP over packet ranges, {threads} threads), median of {repeats} "
                      f"runs of {dt:.1f} s",
            "host": host, "runs_s": runs,
            "single_thread": {"value": n_single / dt1, "unit": "packets/s", "runs_s": runs1,
                              "sample": f"first {n_single} Sobol packets of disk128 on 1 thread, median of "
                                        f"{repeats} runs of {dt1:.2f} s"}}


def _timed_run(ctx, stream, n):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.reset_images()
    e0.record(stream)
    ctx.run(1, n)
    e1.record(stream)
    img = ctx.read_images()
    return img[:, 0], e0.elapsed_time(e1) * 1e-3


def surrogate_section(ctx, qrt, sc, stream, ref, h0: float = 0.1):
    """Learned peel-off on a disk scene (scale height h0 R^1.125): pilot samples
    (Philox, exact labels), training on the GPU, validity mask, then plain
    against surrogate transport of the same Sobol points, with per-kernel times;
    `ref` is an independent high-N image set (exact Halton) or None."""
    import numpy as np
    import torch

    from paper_2406_15632_amd import metrics

    def sync_time(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    from paper_2406_15632_amd import surrogate_recipe as SR
    pilot, rep, mrep, times = SR.train_disk_surrogate(ctx, timer=sync_time, h0=h0)
    t_sample, t_train, t_val = times["sample_s"], times["train_s"], times["validate_s"]
    steps, batch = SR.TRAIN["steps"], SR.TRAIN["batch"]
    N = 1 << 24
    out = {"config": f"{sc.name} scene ({sc.n[0]}^3), cylindrical domain R in [0.05, 1), |z| < 3 h(R), "
                     "16 x 12 cells per observer; 2^20 pilot samples (Philox), 2^17 validation samples, "
                     "20000 Adam steps of 8192, cell error <= 2 % with a transmission floor of 0.3 x the observer "
                     "mean; runs of 2^24 Sobol packets, FP32 transport",
           "pilot_packets": pilot, "sample_s": t_sample, "train_s": t_train, "validate_s": t_val,
           "train_loss": [rep["loss_first"], rep["loss_final"]], "mask": mrep}
    # training throughput: forward plus backward (input and weight gradients) = 3 forward passes per sample
    train_tflops = steps * batch * 3 * MLP_FWD_FLOP / t_train / 1e12
    out["train_mfma"] = {"tflops": train_tflops, "peak_tflops": MFMA_BF16_PEAK_TFLOPS,
                         "frac": train_tflops / MFMA_BF16_PEAK_TFLOPS,
                         "flop_per_sample": 3 * MLP_FWD_FLOP}
    curves = {}
    for mode, name in ((qrt.PEEL_EXACT, "plain"), (qrt.PEEL_SURROGATE, "surrogate")):
        ctx.set_sequence(qrt.SOBOL, PHILOX_SEED, N)
        ctx.set_transport(sc.max_orders, sc.tau_min, qrt.FP32, mode)
        pts = []
        for lg in range(18, 25):
            img, t = _timed_run(ctx, stream, 1 << lg)
            if ref is not None:
                pts.append((t, metrics.rms_error(img, ref), 1 << lg))
        img, t = _timed_run(ctx, stream, N)
        cnt = ctx.counters()
        ctx.set_timing(True)
        ctx.timing(reset=True)
        ctx.reset_images()
        ctx.run(1, 1 << 22)
        tm = ctx.timing(reset=True)
        ctx.set_timing(False)
        out[name] = {"packets_per_s": N / t, "ms": t * 1e3,
                     "rms_error": metrics.rms_error(img, ref) if ref is not None else None,
                     "surrogate_share_of_peels": cnt["surrogate"] / max(1, cnt["peels"]),
                     "visits_per_packet": cnt["visits"] / cnt["packets"],
                     "kernel_ms_per_2e22_packets": {k: round(v[0], 3) for k, v in tm.items() if v[0]}}
        out[name + "_image"] = img
        curves[name] = pts
    out["bias_rms_vs_plain"] = metrics.rms_error(out.pop("surrogate_image"), out.pop("plain_image"))
    out["speedup_packets_per_s"] = out["surrogate"]["packets_per_s"] / out["plain"]["packets_per_s"]
    if ref is not None:
        t1 = {k: metrics.time_to_error([p[0] for p in v], [p[1] for p in v], 0.01) for k, v in curves.items()}
        out["time_to_1pct_s"] = t1
        out["speedup_at_1pct"] = (t1["plain"] / t1["surrogate"]) if (t1["plain"] and t1["surrogate"]) else None
    ctx.set_transport(sc.max_orders, sc.tau_min, qrt.FP32, qrt.PEEL_EXACT)
    return out


def surrogate_resolved_section(qrt, stream):
    """The learned peel-off where rays are long and the density is resolved: a
    thick flared disk (h0 = 0.3, midplane optical depth 1) on a 256^3 mesh, the
    same recipe and domain rule as the disk128 run, against a Halton reference
    of 2^28 packets."""
    import torch

    from synth import scenes
    sc = scenes.disk128(n=256, tau_mid=1.0, h0=0.3)
    ctx = qrt.Context(0, stream.cuda_stream)
    ctx.set_scene(sc, kind=qrt.HALTON, n_total=1 << 28, grid=torch.from_numpy(sc.kappa_rho).cuda())
    ref, _ = _timed_run(ctx, stream, 1 << 28)
    out = surrogate_section(ctx, qrt, sc, stream, ref, h0=0.3)
    out["reference"] = "halton, 2^28 packets, exact peel-off"
    ctx.close()
    return out


def other_workloads(qrt, stream):
    """Throughput of the dust envelope (32^3, single scattering, FP64) and the
    clumpy envelope with a spherical star (256^3, FP32), Sobol, 2^24 packets,
    median of three runs."""
    import torch

    from synth import scenes
    res = {}
    for name, sc in (("envelope32", scenes.envelope32()), ("clumpy256", scenes.clumpy256())):
        ctx = qrt.Context(0, stream.cuda_stream)
        ctx.set_scene(sc, kind=qrt.SOBOL, grid=torch.from_numpy(sc.kappa_rho).cuda())
        n = 1 << 24
        _timed_run(ctx, stream, 1 << 20)          # warm-up
        runs = sorted(_timed_run(ctx, stream, n)[1] for _ in range(3))
        t = runs[1]                               # median of three
        cnt = ctx.counters()
        res[name] = {"packets_per_s": n / t, "ms": t * 1e3, "runs_ms": [r * 1e3 for r in runs], "packets": n,
                     "precision": "f64" if sc.fp64 else "f32",
                     "visits_per_packet": cnt["visits"] / cnt["packets"],
                     "algorithmic_GBps": (4.0 * cnt["visits"] + 24.0 * cnt["peels"]) / t / 1e9}
        ctx.close()
    return res


def batch_section(qrt, stream, seed: int = 2406, steps: int = 2, n_scenes: int = 64, overlap: bool = True, **draw):
    """The batched workload: 64 uneven scenes drawn from `seed` (grids 32^3 to
    192^3, 2^16 to 2^24 packets, tau 0.1 to 20, g 0 to 0.8, albedo 0.3 to 0.9,
    envelope or disk, point source or sphere star, 1 to 4 observers, 1 to 20
    orders, 128^2 images, FP32 rays with FP64 sums), Sobol points; or another
    draw of the same recipe (`n_scenes`, and the ranges in `draw`).  One batch
    run (every scene's packets in one launch sequence; in stream order, and with
    its chunks overlapped on the internal streams) against the same scenes
    run one after another through the single-scene calls, in stream order and
    overlapped (with the scene changes between runs, as a caller makes them),
    and the runs alone; meshes resident in HBM for all."""
    import torch

    from synth import scenes
    bs = scenes.uneven_batch(seed, n_scenes, **draw)
    total = sum(sc.n_packets for sc in bs)
    grids = [torch.from_numpy(sc.kappa_rho).cuda() for sc in bs]
    ctx = qrt.Context(0, stream.cuda_stream)
    ctx.batch_set(bs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.batch_run(qrt.SOBOL, 0, qrt.FP32)               # warm-up
    ctx.join()
    torch.cuda.synchronize()
    ctx.batch_reset()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        ctx.batch_run(qrt.SOBOL, 0, qrt.FP32)
    ctx.join()
    e1.record(stream)
    torch.cuda.synchronize()
    batch_wall = (time.perf_counter() - w0) / steps
    batch_s = e0.elapsed_time(e1) * 1e-3 / steps
    cnt = ctx.counters()
    # the batch's chunks overlapped on the context's internal streams
    batch_ov_s = 0.0
    if overlap:
        ctx.set_overlap(True)
        e0.record(stream)
        for _ in range(steps):
            ctx.batch_run(qrt.SOBOL, 0, qrt.FP32)
        ctx.join()
        e1.record(stream)
        torch.cuda.synchronize()
        batch_ov_s = e0.elapsed_time(e1) * 1e-3 / steps
    # the same scenes one after another
    seq = qrt.Context(0, stream.cuda_stream)
    for sc, g in zip(bs[:2], grids[:2]):             # warm-up of the single-scene kernels
        seq.set_scene(sc, kind=qrt.SOBOL, grid=g, precision=qrt.FP32)
        seq.run(1, min(sc.n_packets, 1 << 16))
    torch.cuda.synchronize()
    seq_s = {}
    for seq_overlap in (False, True):
        seq.set_overlap(seq_overlap)
        # in stream order, also the runs alone: events around each run leave out
        # the scene changes between them (mesh upload, image buffers)
        runs = [] if seq_overlap else [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                                   for _ in bs]
        e0.record(stream)
        for i, (sc, g) in enumerate(zip(bs, grids)):
            seq.set_scene(sc, kind=qrt.SOBOL, grid=g, precision=qrt.FP32)
            if runs:
                runs[i][0].record(stream)
            seq.run(1, sc.n_packets)
            if runs:
                runs[i][1].record(stream)
        seq.join()
        e1.record(stream)
        torch.cuda.synchronize()
        seq_s["overlapped" if seq_overlap else "stream_order"] = e0.elapsed_time(e1) * 1e-3
        if runs:
            seq_s["runs_only"] = sum(a.elapsed_time(b) for a, b in runs) * 1e-3
    ctx.close()
    seq.close()
    return {
        "scenes": len(bs), "packets": total, "seed": seed,
        "batch_packets_per_s": total / batch_s, "batch_ms": batch_s * 1e3, "batch_wall_ms": batch_wall * 1e3,
        "sequential_packets_per_s": total / seq_s["stream_order"], "sequential_ms": seq_s["stream_order"] * 1e3,
        "sequential_overlapped_packets_per_s": total / seq_s["overlapped"],
        "sequential_overlapped_ms": seq_s["overlapped"] * 1e3,
        "speedup": seq_s["stream_order"] / batch_s,
        "batch_overlapped_packets_per_s": total / batch_ov_s if overlap else None,
        "batch_overlapped_ms": batch_ov_s * 1e3 if overlap else None,
        "speedup_vs_sequential_overlapped": seq_s["overlapped"] / batch_s,
        "speedup_overlapped_vs_sequential_overlapped": seq_s["overlapped"] / batch_ov_s if overlap else None,
        "sequential_runs_only_ms": seq_s["runs_only"] * 1e3,
        "speedup_vs_sequential_runs_only": seq_s["runs_only"] / batch_s,
        "visits_per_packet": cnt["visits"] / cnt["packets"],
        "algorithmic_GBps": (4.0 * cnt["visits"] + 24.0 * cnt["peels"]) / (batch_s * steps) / 1e9,
    }


def sphere_star_section(qrt, stream):
    """Time to a fixed image error for a spherical star (the clumpy envelope,
    256^3, single scattering, 512^2 image): QMC (Sobol) in the direct and the
    inverse order of the point coordinates, Hammersley in the inverse order,
    and Monte Carlo (Philox, 2 seeds); pixels within the star's radius of the
    centre are left out.  The reference is Halton in the direct order at 2^28
    packets (Sobol is not used for it, being one of the compared sets)."""
    import numpy as np
    import torch

    from paper_2406_15632_amd import metrics
    from synth import scenes
    sc0 = scenes.clumpy256()
    mask = metrics.central_mask(sc0.npix, sc0.half_width, sc0.r_star)
    f = 8   # 8 x 8 pixel bins: per-pixel shot noise of a 512^2 image would hide the point sets

    def binned(img):
        m = img * mask
        return m.reshape(sc0.npix // f, f, sc0.npix // f, f).sum(axis=(1, 3))
    grid = torch.from_numpy(sc0.kappa_rho).cuda()
    ctx = qrt.Context(0, stream.cuda_stream)

    def images(order, kind, n, seed=PHILOX_SEED):
        sc = sc0.replace(emit_order=order)
        ctx.set_scene(sc, kind=kind, seed=seed, n_total=n, grid=grid)
        img, t = _timed_run(ctx, stream, n)
        return img[0], t

    ref = binned(images(0, qrt.HALTON, 1 << 28)[0])
    variants = {"sobol_direct": (0, qrt.SOBOL, (PHILOX_SEED,)), "sobol_inverse": (1, qrt.SOBOL, (PHILOX_SEED,)),
                "hammersley_inverse": (1, qrt.HAMMERSLEY, (PHILOX_SEED,)), "philox": (0, qrt.PHILOX, (1, 2))}
    out = {"reference": "halton, direct order, 2^28 packets",
           "error": "relative RMS of the 64^2 image of 8 x 8 pixel bins, star pixels left out",
           "errors": {}, "time_s": {}}
    for name, (order, kind, seeds) in variants.items():
        pts = []
        for lg in range(14, 25, 2):
            e, t = [], []
            for sd in seeds:
                img, dt = images(order, kind, 1 << lg, sd)
                e.append(metrics.rms_error(binned(img), ref))
                t.append(dt)
            pts.append((float(np.mean(t)), float(np.mean(e))))
        out["errors"][name] = {14 + 2 * i: round(p[1], 5) for i, p in enumerate(pts)}
        out["time_s"][name] = [metrics.time_to_error([p[0] for p in pts], [p[1] for p in pts], tg)
                               for tg in (0.05, 0.01)]
    mc = out["time_s"]["philox"]
    out["speedup_vs_mc_at_5_1_pct"] = {k: [(m / t if (m and t) else None) for m, t in zip(mc, v)]
                                       for k, v in out["time_s"].items()}
    ctx.close()
    return out


def per_order_section(qrt, sc, stream):
    """Image error of each scattering order (disk128, 2^22 packets) for Sobol,
    Hammersley and Monte Carlo (Philox, mean over 2 seeds), against per-order
    images of Halton at 2^28 packets, and the Monte Carlo / QMC error ratio per
    order: the paper's observation that the QMC gain shrinks with the order."""
    import numpy as np
    import torch

    from paper_2406_15632_amd import metrics
    ctx = qrt.Context(0, stream.cuda_stream)
    grid = torch.from_numpy(sc.kappa_rho).cuda()
    K = 6

    def per_order(kind, n, seed=PHILOX_SEED):
        ctx.set_scene(sc, kind=kind, seed=seed, n_total=n, grid=grid)
        ctx.set_order_images(True)
        ctx.reset_images()
        ctx.run(1, n)
        imgs = [ctx.read_order_images(k)[:, 0] for k in range(1, K + 1)]
        rest = ctx.read_images()[:, 0] - sum(imgs)
        ctx.set_order_images(False)
        return imgs + [rest]

    ref = per_order(qrt.HALTON, 1 << 28)
    n = 1 << 22
    out = {"orders": [str(k) for k in range(1, K + 1)] + [f">{K}"], "packets": n,
           "reference": "halton, 2^28 packets", "share_of_light": [], "rms_error": {}, "image_norm": {}}
    tot = sum(float(r.sum()) for r in ref)
    out["share_of_light"] = [round(float(r.sum()) / tot, 4) for r in ref]
    for name, kind, seeds in (("sobol", qrt.SOBOL, (PHILOX_SEED,)), ("hammersley", qrt.HAMMERSLEY, (PHILOX_SEED,)),
                              ("philox", qrt.PHILOX, (1, 2))):
        errs = np.zeros(K + 1)
        norms = np.zeros(K + 1)
        for sd in seeds:
            imgs = per_order(kind, n, sd)
            errs += np.array([metrics.rms_error(a, b) for a, b in zip(imgs, ref)])
            norms += np.array([metrics.image_norm(a, b) for a, b in zip(imgs, ref)])
        out["rms_error"][name] = [round(float(e), 5) for e in errs / len(seeds)]
        out["image_norm"][name] = [round(float(e), 5) for e in norms / len(seeds)]
    out["mc_over_sobol"] = [round(m / q, 3) for m, q in zip(out["rms_error"]["philox"], out["rms_error"]["sobol"])]
    ctx.close()
    return out


def time_to_error_sweep(ctx, qrt, sc, kinds, stream, ref_log2: int, sweep_log2: int, faure: bool = True,
                        owen: bool = True):
    """Image RMS error (I, all observers) against an independent high-N reference
    versus kernel time, N = 2^12 .. 2^sweep_log2; Sobol is scored against a
    Halton reference and every other set against a Sobol reference; the PRNG
    errors are averaged over seeds (4 below 2^24 packets, 2 above) and run to
    4x the largest quasi-random size, since they converge more slowly.  Faure's
    curve and the error bar of Owen-scrambled Sobol runs are optional."""
    import numpy as np
    import torch

    from paper_2406_15632_amd import metrics

    def run(kind, n, seed=PHILOX_SEED):
        ctx.set_sequence(kind, seed, n)
        ctx.reset_images()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.run(1, n)
        e1.record(stream)
        img = ctx.read_images()
        return img[:, 0], e0.elapsed_time(e1) * 1e-3

    n_ref = 1 << ref_log2
    ref_s, _ = run(qrt.SOBOL, n_ref)
    ref_h, _ = run(qrt.HALTON, n_ref)
    floor = metrics.rms_error(ref_s, ref_h)
    names = {qrt.SOBOL: "sobol", qrt.HALTON: "halton", qrt.NIEDERREITER2: "niederreiter2",
             qrt.HAMMERSLEY: "hammersley", qrt.PHILOX: "philox", qrt.FAURE: "faure"}
    kinds = list(kinds) + ([qrt.FAURE] if faure else [])   # the paper's fourth low-discrepancy sequence
    curves = {}
    for kind in kinds:
        ref = ref_h if kind == qrt.SOBOL else ref_s
        pts = []
        top = sweep_log2 + (2 if kind == qrt.PHILOX else 0)   # MC needs ~4x the packets
        for lg in range(12, top + 1):
            seeds = ((1, 2, 3, 4) if lg < 24 else (1, 2)) if kind == qrt.PHILOX else (PHILOX_SEED,)
            errs, ts, dis, ins = [], [], [], []
            for sd in seeds:
                img, t = run(kind, 1 << lg, sd)
                errs.append(metrics.rms_error(img, ref))
                dis.append(abs(metrics.integral_norm(img, ref)))
                ins.append(metrics.image_norm(img, ref))
                ts.append(t)
            pts.append((float(np.mean(ts)), float(np.mean(errs)), 1 << lg, float(np.mean(dis)), float(np.mean(ins))))
        curves[names[kind]] = pts
    owen_bar = None
    if owen:
        # randomised QMC: R independent Owen scramblings give an error bar from
        # their spread; compared here with the actual error of their mean
        R, n_each = 8, 1 << 21
        imgs = [run(qrt.SOBOL_OWEN, n_each, 1000 + r)[0] for r in range(R)]
        mean = sum(imgs) / R
        spread = float(np.sqrt(sum(float(np.sum((im - mean) ** 2)) for im in imgs) / (R * (R - 1))) /
                       np.linalg.norm(ref_h))
        owen_bar = {"scramblings": R, "packets_each": n_each, "estimated_rms_error_of_mean": spread,
                    "actual_rms_error_of_mean": metrics.rms_error(mean, ref_h),
                    "unscrambled_sobol_rms_error_same_packets":
                        metrics.rms_error(run(qrt.SOBOL, R * n_each)[0], ref_h)}
    targets = (0.05, 0.01, 0.003)
    floor_in = metrics.image_norm(ref_s, ref_h)
    by_lg = lambda v, j: {int(p[2]).bit_length() - 1: round(p[j], 6) for p in v}
    out = {"targets": list(targets), "ref_packets": n_ref, "ref_floor_rms": floor, "_ref_halton": ref_h,
           "rms_error_by_log2_packets": {k: by_lg(v, 1) for k, v in curves.items()},
           "time_s": {}, "speedup_vs_mc": {}, "owen_error_bar": owen_bar,
           # the paper's norms (Sec. 4): |dI| of the total intensity and Delta I / I over
           # the pixels of all observers, the times to Delta I / I targets, and the
           # power laws a t^-0.5 and a t^-b of |dI| (Sec. 5; t in seconds)
           "ref_floor_image_norm": floor_in,
           "ref_floor_integral_norm": abs(metrics.integral_norm(ref_s, ref_h)),
           "integral_norm_by_log2_packets": {k: by_lg(v, 3) for k, v in curves.items()},
           "image_norm_by_log2_packets": {k: by_lg(v, 4) for k, v in curves.items()},
           "time_s_image_norm": {}, "speedup_vs_mc_image_norm": {}, "integral_norm_fits": {},
           # packets to the RMS targets: the ratio the paper's CPU times measure (its time is
           # proportional to the packets), free of the GPU's fixed launch cost at small N
           "packets_to_error": {}, "speedup_vs_mc_in_packets": {}}
    for k, pts in curves.items():
        ts = [p[0] for p in pts]
        es = [p[1] for p in pts]
        ns = [float(p[2]) for p in pts]
        out["time_s"][k] = [metrics.time_to_error(ts, es, tg) if tg >= 3 * floor else None for tg in targets]
        out["packets_to_error"][k] = [metrics.time_to_error(ns, es, tg) if tg >= 3 * floor else None
                                      for tg in targets]
        ins = [p[4] for p in pts]
        out["time_s_image_norm"][k] = [metrics.time_to_error(ts, ins, tg) if tg >= 3 * floor_in else None
                                       for tg in targets]
        dis = [p[3] for p in pts]
        half = len(pts) // 2
        a05 = metrics.power_fit(ts, dis, b=0.5)
        ab = metrics.power_fit(ts, dis)
        ab_long = metrics.power_fit(ts[half:], dis[half:])
        out["integral_norm_fits"][k] = {"a_for_b_0.5": a05[0] if a05 else None,
                                        "a_b_all": list(ab) if ab else None,
                                        "a_b_longest_half": list(ab_long) if ab_long else None}
    # the paper's comparison of the a t^-0.5 fits: how many times smaller |dI| is than Monte Carlo's
    a_mc = out["integral_norm_fits"]["philox"]["a_for_b_0.5"]
    for k, f in out["integral_norm_fits"].items():
        f["mc_a_over_a"] = (a_mc / f["a_for_b_0.5"]) if (a_mc and f["a_for_b_0.5"]) else None
    for key, dst in (("time_s", "speedup_vs_mc"), ("time_s_image_norm", "speedup_vs_mc_image_norm"),
                     ("packets_to_error", "speedup_vs_mc_in_packets")):
        mc = out[key]["philox"]
        for k, tt in out[key].items():
            out[dst][k] = [(m / t if (m is not None and t) else None) for m, t in zip(mc, tt)]
    return out


# The paper's single-scattering time table (Sec. 5), dust sphere envelope with a
# point source: CPU seconds to reach Delta I / I = 5 %, 1 %, 0.3 % on one core of
# an Intel Core i5-10400F at 4.1 GHz ("quasi MC" = the mean over Sobol,
# Niederreiter, Faure and Halton).  Context only: other scene, other hardware.
PAPER_ENVELOPE_SECONDS = {"monte_carlo": [77.0, 1.7e3, 2.0e4], "quasi_mc": [19.0, 1.9e2, 9.4e2],
                          "hammersley": [8.0, 80.0, 5.0e2]}


def envelope_time_to_error(qrt, stream, ref_log2: int = 30, sweep_log2: int = 26):
    """Time to a fixed image error for the single-scattering dust envelope
    (envelope32: 32^3 mesh, point source, one 64^2 view at 45 deg, FP64
    transport), every point set against Monte Carlo, with the paper's
    single-scattering speed-ups for its dust-sphere envelope beside them."""
    import torch

    from synth import scenes
    sc = scenes.envelope32()
    ctx = qrt.Context(0, stream.cuda_stream)
    ctx.set_scene(sc, kind=qrt.SOBOL, grid=torch.from_numpy(sc.kappa_rho).cuda())
    kinds = [scenes.KIND_BY_NAME[k] for k in KIND_ORDER]
    out = time_to_error_sweep(ctx, qrt, sc, kinds, stream, ref_log2, sweep_log2, faure=True, owen=False)
    out.pop("_ref_halton")
    ctx.close()
    P = PAPER_ENVELOPE_SECONDS
    out["paper_context"] = {
        "scene": "the paper's dust sphere envelope, single scattering, point source (Sec. 5 time table)",
        "hardware": "one core of an Intel Core i5-10400F at 4.1 GHz",
        "error": "Delta I / I at 5 %, 1 %, 0.3 %",
        "speedup_vs_mc": {k: [m / t for m, t in zip(P["monte_carlo"], P[k])] for k in ("quasi_mc", "hammersley")},
    }
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the transport runs on one GPU; --gpus must be 1 (no multi-GPU "
                                   "sharding is implemented)"}))
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

    # consecutive runs overlap on the context's three internal streams: the next run
    # starts beside the last scattering orders of the previous one
    overlap = not args.no_overlap
    ctx.set_overlap(overlap)
    for _ in range(args.warmup):
        step()
    ctx.join()
    torch.cuda.synchronize()
    ctx.reset_images()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for s in range(args.steps):
        step()
    ctx.join()   # the last run's completion joins the stream before the end event
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    elapsed_ms = t_start.elapsed_time(t_end)
    cnt = ctx.counters()
    n_launch = args.steps * len(kinds)
    alg_bytes = 4.0 * cnt["visits"] + 24.0 * cnt["peels"]
    achieved = alg_bytes / (elapsed_ms * 1e-3) / 1e9
    # per-kernel timing pass over the same workload, in stream order (each kernel's own
    # duration): the library records HIP events on its launch stream around every kernel,
    # by class, and the runs are bracketed by events on the same stream
    ctx.set_overlap(False)
    ctx.set_timing(True)
    ctx.timing(reset=True)
    ctx.reset_images()
    launch_events = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in kinds]
                     for _ in range(args.timing_steps)]
    for s in range(args.timing_steps):
        step(launch_events[s])
    tm = ctx.timing(reset=True)
    per_kind_ms = {KIND_ORDER[j]: sum(launch_events[s][j][0].elapsed_time(launch_events[s][j][1])
                                      for s in range(args.timing_steps)) / args.timing_steps
                   for j in range(len(kinds))}
    cnt_t = ctx.counters()
    ctx.set_timing(False)
    n_t = args.timing_steps * len(kinds)
    timed_ms = sum(v[0] for v in tm.values()) / n_t
    walk_ms = tm["walk"][0] / n_t
    walk_bytes = (4.0 * (cnt_t["visits"] - cnt_t["visits_first"]) + 24.0 * cnt_t["peels"]) / n_t
    walk_gbps = walk_bytes / (walk_ms * 1e-3) / 1e9
    first_ms = tm["first"][0] / n_t
    first_bytes = 4.0 * cnt_t["visits_first"] / n_t
    copy_gbps = measured_copy_gbps()   # after the timed region
    packets = args.steps * len(kinds) * N
    traffic = committed_traffic() if N == 1 << 22 else None
    walk_traffic = committed_traffic("walk_bytes_per_launch") if N == 1 << 22 else None
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
            "runs": "five qrt_run calls per step; consecutive runs overlapped on the context's three internal "
                    "streams (qrt_set_overlap)" if overlap else "five qrt_run calls per step, in stream order",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": walk_gbps,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": walk_gbps / HBM_PEAK_GBS,
            "traffic": walk_traffic,
            "kernel": "the walk kernels, dominant together: k_walk (peel-off rays and flights of order 1, "
                      "then the peel rays of the deferred later scatterings) and k_tail (orders 2-20 in one "
                      "launch), all their dispatches of one transport launch together",
            "alg_bytes_per_launch": walk_bytes,
            "alg_bytes": "4 B per cell visit of the walks (all visits but those of the first flights; "
                         "k_tail's flights included) + 24 B per binned peel-off contribution, exact counts "
                         "from the kernels' counters",
            "avg_launch_ms": walk_ms,
            "avg_dispatch_us": 1e3 * tm["walk"][0] / max(1, tm["walk"][1]),
            "share_of_launch": walk_ms / timed_ms if timed_ms else None,
            "timing": f"HIP events on the launch stream around every kernel, {args.timing_steps} steps "
                      f"({n_t} launches) after the timed region",
            "walk_counters": committed_walk_counters(),
            "measured_copy_GBps": copy_gbps,
            "frac_of_measured_copy": walk_gbps / copy_gbps,
            "step": {
                "kernel": "the whole transport step qrt_run (k_key_emit, the two-pass radix sort, k_first, "
                          "k_scatter and k_walk of order 1, then k_tail, k_def_keys and the "
                          "radix sort of the deferred scatterings, their k_scatter and k_walk) over the timed "
                          "region",
                "achieved": achieved, "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "alg_bytes_per_launch": alg_bytes / n_launch, "avg_launch_ms": elapsed_ms / n_launch,
                "stream_ordered_launch_ms": sum(per_kind_ms.values()) / len(kinds),
            },
            "first_flights": {"kernel": "k_first", "avg_launch_ms": first_ms, "alg_bytes_per_launch": first_bytes,
                              "achieved": first_bytes / (first_ms * 1e-3) / 1e9 if first_ms else None},
            "kernel_ms_per_launch": {k: v[0] / n_t for k, v in tm.items()},
        },
        "per_sequence_packets_per_s": {k: N / (v * 1e-3) for k, v in per_kind_ms.items()},
        "counters_per_packet": {k: cnt[k] / cnt["packets"] for k in ("visits", "peels", "scatterings",
                                                                   "escapes", "tau_cuts")},
        "wall_s": wall,
    }
    ref = None
    if not args.no_time_to_error:
        result["time_to_error"] = time_to_error_sweep(ctx, qrt, sc, kinds, stream, args.ref_log2,
                                                      args.sweep_log2)
        ref = result["time_to_error"].pop("_ref_halton")
    if not args.no_time_to_error:
        result["per_order"] = per_order_section(qrt, sc, stream)
        result["envelope_time_to_error"] = envelope_time_to_error(qrt, stream)
    if not args.no_surrogate:
        result["surrogate"] = surrogate_section(ctx, qrt, sc, stream, ref)
        if ref is not None:
            result["surrogate_resolved"] = surrogate_resolved_section(qrt, stream)
    if not args.no_workloads:
        result["workloads"] = other_workloads(qrt, stream)
        result["sphere_star"] = sphere_star_section(qrt, stream)
    if not args.no_batch:
        result["batch"] = batch_section(qrt, stream, overlap=not args.no_batch_overlap)
        # many small scenes, where one scene does not fill the GPU: 256 scenes,
        # grids 32^3 to 96^3, 2^10 to 2^14 packets each
        if not args.no_batch_small:
            result["batch_small"] = batch_section(qrt, stream, n_scenes=256, overlap=not args.no_batch_overlap,
                                                  sizes=(32, 96, 16), log2_packets=(10.0, 14.0))
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sc, args.cpu_sample)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

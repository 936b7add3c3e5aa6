#!/usr/bin/env python3
"""Throughput of the double-MRT cavity step on one MI355X.

Workload (default): 256^3 cube, Type 1 walls, Ra = 1e6, Pr = 0.71, Ma = 0.1,
FP32 storage and arithmetic, fluid at rest with seeded +-1e-6 theta noise.
A "step" is one fused streaming + collision update of every node (both
lattices, all walls).  W untimed warm-up steps, then K timed steps bracketed
by device synchronisation.  Prints one JSON line.

value = n^3 * K / wall time, in MLUPS (million lattice-node updates / s).
roofline: algorithmic bytes per launch (26 populations read + written per
node, 208 B at FP32) over the average kernel time from HIP events recorded
on the stream the kernels run on, against the 8 TB/s HBM peak.
cpu_baseline: the FP64 CPU oracle timed on a bounded sample (64^3, same case).
cpu_oracle_detail: the host (CPU model, logical CPUs), the oracle with one
thread on the same 64^3 sample, and the 16^3, Ra 1e3, Type 1 cavity for
2000 steps with one thread and with all threads (child processes with
OMP_NUM_THREADS set, no GPU use).
time_to_steady: 128^3, Ra 1e5, FP32, wall types 1-3, wall time to |dNu_3D| <
1e-6 per 1000 steps from rest, from the shipped U-Net's predicted fields
(warm start; inference and initialisation included), by grid sequencing
(the prediction run to steady on 64^3 first, that solve included), and by
extrapolated grid sequencing (32^3 from the prediction, then 64^3, the
128^3 start extrapolated from both).
storage_sweep: every storage format at the same size and case (500 steps each).
batch_to_steady: the 64-cavity batch (n uniform in {32, 48, 64, 80, 96}, Ra
log-uniform in [1e3, 1e6], wall type uniform in {1, 2, 3}, seed 1511, FP32)
run to steady in one persistent launch per step (autotuned launch shape,
graph replay), wall time and aggregate MLUPS, and the same cases by grid
sequencing (a half-size batch run to steady first).
unet_training_step: one optimiser step of the warm-start U-Net (batch 4,
64^3; forward, squared-error loss, backward, Adam), HIP events over 20 steps
after 3 warm-up steps, the convolutions' FLOP rate, and the floor of the
convolutions (per launch the larger of HBM and MFMA time) with the step's
ratio to it.
warm_start_192: a 192^3 cavity (Ra 3e5, Type 2, FP32) to steady from rest,
from the U-Net's predicted fields, from a 96^3 cavity started from them
and run to steady, and extrapolated from 48^3 and 96^3 cavities (inference,
coarse solves and initialisation timed).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def cpu_baseline(seconds: float, n: int = 64, ra: float = 1e6, wall_type: int = 1):
    from oracle import oracle as ora
    from paper_1511_04633_amd import inputs

    o = ora.Oracle(n, wall_type, ra=ra, theta0=inputs.theta_noise(n, 20151115))
    o.step(1)  # first touch of the arrays
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.step(5)
        steps += 5
    dt = time.perf_counter() - t0
    return {"value": round(n ** 3 * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": ora.threads(), "kind": "oracle",
            "sample": f"FP64 oracle, {n}^3 Type {wall_type} Ra {ra:g}, {steps} steps in {dt:.1f} s"}


def _oracle_timing_child(n: int, ra: float, wall_type: int, steps: int, seconds: float):
    """Runs in a child process (no GPU): the oracle's MLUPS for `steps`
    steps, or for about `seconds` when steps = 0; prints one JSON line."""
    from oracle import oracle as ora
    from paper_1511_04633_amd import inputs

    o = ora.Oracle(n, wall_type, ra=ra, theta0=inputs.theta_noise(n, 20151115))
    o.step(1)
    done, t0 = 0, time.perf_counter()
    if steps:
        o.step(steps)
        done = steps
    else:
        while time.perf_counter() - t0 < seconds:
            o.step(5)
            done += 5
    dt = time.perf_counter() - t0
    print(json.dumps({"threads": ora.threads(), "steps": done, "seconds": round(dt, 3),
                      "mlups": round(n ** 3 * done / dt / 1e6, 3)}), flush=True)


def cpu_oracle_detail(seconds: float, ra: float, wall_type: int):
    """Host description and one-thread / all-thread oracle timings, each in a
    child process started with OMP_NUM_THREADS (the oracle's OpenMP runtime
    reads it once)."""
    import subprocess

    def child(threads, n, ra_, wt, steps, secs):
        env = dict(os.environ)
        if threads:
            env["OMP_NUM_THREADS"] = str(threads)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-timing",
                            str(n), repr(ra_), str(wt), str(steps), repr(secs)],
                           env=env, capture_output=True, text=True, timeout=600, check=True)
        return json.loads(r.stdout.strip().splitlines()[-1])

    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)),
            "oracle_64cube_1_thread": child(1, 64, ra, wall_type, 0, seconds),
            "config1_16cube_ra1e3_type1_2000_steps": {"1_thread": child(1, 16, 1e3, 1, 2000, 0.0),
                                                      "all_threads": child(0, 16, 1e3, 1, 2000, 0.0)}}


def time_to_steady(wall_type: int, net=None, coarse: int = 64, n: int = 128, ra: float = 1e5):
    """Wall time to |dNu_3D| < 1e-6 per 1000 steps (host clock, all
    synchronisations included) for the 128^3, Ra 1e5, FP32 cavity, from rest;
    when the network is given, from its predicted fields (inference and
    initialisation inside the timed region); with coarse = m > 0, by grid
    sequencing: the m^3 cavity run to steady by the same criterion (from the
    network's fields, or from rest without a network) starts the 128^3 one
    (coarse solve inside the timed region); and with extrapolation: an
    (m/2)^3 cavity started the same way and run to steady starts the m^3
    one, and the 128^3 cavity starts from 5/4 of the m^3 fields minus 1/4
    of the (m/2)^3 fields (both coarse solves inside the timed region)."""
    from paper_1511_04633_amd import warmstart

    rest = warmstart.solve(n, ra, wall_type, None, max_steps=2_000_000)
    out = {"workload": f"{n}^3 Type {wall_type} Ra {ra:g} f32", "seconds": rest["seconds"],
           "steps": rest["steps"], "converged": rest["converged"], "nu3d": rest["nu3d"],
           "nu2d": rest["nu2d"], "numax": rest["numax"]}
    if net is not None:
        warm = warmstart.solve(n, ra, wall_type, net, max_steps=2_000_000)
        out["warm_start"] = {"seconds": warm["seconds"], "steps": warm["steps"],
                             "init_s": warm["init_s"], "converged": warm["converged"],
                             "nu3d": warm["nu3d"],
                             "nu_rel_diff": abs(warm["nu3d"] - rest["nu3d"]) / rest["nu3d"]}
    if coarse:
        ml = warmstart.solve(n, ra, wall_type, net, coarse=coarse, max_steps=2_000_000)
        out["multilevel"] = {"seconds": ml["seconds"], "steps": ml["steps"],
                             "start": "network" if net is not None else "rest",
                             "coarse": ml["coarse"], "init_s": ml["init_s"],
                             "converged": ml["converged"], "nu3d": ml["nu3d"],
                             "nu_rel_diff": abs(ml["nu3d"] - rest["nu3d"]) / rest["nu3d"]}
        ex = warmstart.solve(n, ra, wall_type, net, coarse=coarse, max_steps=2_000_000,
                             extrapolate=True)
        out["extrapolated"] = {"seconds": ex["seconds"], "steps": ex["steps"],
                               "start": "network" if net is not None else "rest",
                               "coarse": ex["coarse"], "init_s": ex["init_s"],
                               "converged": ex["converged"], "nu3d": ex["nu3d"],
                               "nu_rel_diff": abs(ex["nu3d"] - rest["nu3d"]) / rest["nu3d"]}
    return out


def storage_sweep(n: int, wall_type: int, ra: float, steps: int = 500, warmup: int = 100):
    """Every storage format at the benchmark size: MLUPS (host clock) and the
    step kernel's HBM roofline fraction (HIP events), same case and start."""
    import torch

    from paper_1511_04633_amd import inputs, lbmx

    out = []
    for st in ("f64", "f32", "f16", "bf16", "f16_f32", "bf16_f32", "f16_i16"):
        cav = lbmx.Cavity(n=n, wall_type=wall_type, ra=ra, storage=st,
                          theta0=inputs.theta_noise(n, 20151115))
        cav.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev_ms = cav.step_timed(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        bpc = lbmx.bytes_per_cell(st)
        kernel_s = ev_ms / 1e3 / steps
        out.append({"storage": st, "bytes_per_cell": bpc,
                    "mlups": round(n ** 3 * steps / wall / 1e6, 1),
                    "kernel_us": round(kernel_s * 1e6, 2),
                    "frac": round(n ** 3 * bpc / kernel_s / 1e9 / HBM_PEAK_GBS, 4)})
        cav.close()
        del cav
        torch.cuda.empty_cache()
    return out


def batch_to_steady(coarse: bool):
    """The 64-cavity batch to |dNu_3D| < 1e-6 per 1000 steps: wall time from
    the first step to the last retirement (host clock), aggregate MLUPS
    (sum over cavities of n^3 x steps / wall time), converged count and the
    autotuned launch shape."""
    from paper_1511_04633_amd import dataset

    ds = dataset.generate(seed=1511, count=64, out_n=64, max_steps=300_000, coarse=coarse)
    s = ds["summary"]
    out = {"workload": "64 cavities, n in {32,48,64,80,96}, Ra log-uniform [1e3,1e6], "
                       "types 1-3, seed 1511, f32",
           "start": "half-size batch run to steady" if coarse else "rest",
           "wall_s": round(s["wall_s"], 3), "mlups": round(s["mlups"], 1),
           "node_steps": s["node_steps"], "converged": s["converged"], "count": s["count"],
           "launch": s["launch"], "autotune_us_per_step": s["autotune_us_per_step"],
           "max_steps_taken": int(max(ds["all_steps"]))}
    if coarse and s.get("coarse"):
        out["coarse_wall_s"] = round(s["coarse"]["wall_s"], 3)
    return out


def unet_training_step():
    """The U-Net's training step (unet.bench_step: batch 4 at 64^3, synthetic
    targets, all network kernels), its convolution FLOP rate and the floor of
    its convolutions (unet.conv_floor: per launch the larger of HBM and MFMA
    time)."""
    from paper_1511_04633_amd import unet

    ms = unet.bench_step(batch=4, m=64)
    flop, floor_s, hbm_s, mfma_s = unet.conv_floor(4, 64)
    return {"workload": "U-Net training step, batch 4, 64^3, BF16 MFMA", "ms_per_step": round(ms, 4),
            "conv_gflop": round(flop / 1e9, 1), "conv_tflops": round(flop / ms / 1e9, 1),
            "bf16_dense_peak_frac": round(flop / ms / 1e9 / 2500.0, 4),
            "conv_floor_us": round(floor_s * 1e6, 1), "conv_floor_hbm_only_us": round(hbm_s * 1e6, 1),
            "conv_floor_mfma_only_us": round(mfma_s * 1e6, 1),
            "step_over_conv_floor": round(ms * 1e-3 / floor_s, 2)}


def warm_start_192(net, ra: float = 3e5, wall_type: int = 2, n: int = 192, coarse: int = 96):
    """The learned warm start at 192^3: rest start vs the network's fields vs grid sequencing
    through a coarse^3 cavity started from them vs the extrapolated start
    from (coarse/2)^3 and coarse^3 cavities; all to |dNu_3D| < 1e-6 per 1000
    steps, FP32, on this GPU."""
    from paper_1511_04633_amd import warmstart

    rest = warmstart.solve(n, ra, wall_type, None, max_steps=1_000_000)
    warm = warmstart.solve(n, ra, wall_type, net, max_steps=1_000_000)
    ml = warmstart.solve(n, ra, wall_type, net, coarse=coarse, max_steps=1_000_000)
    ex = warmstart.solve(n, ra, wall_type, net, coarse=coarse, max_steps=1_000_000,
                         extrapolate=True)
    rel = lambda r: abs(r["nu3d"] - rest["nu3d"]) / rest["nu3d"]
    return {"workload": f"{n}^3 Type {wall_type} Ra {ra:g} f32",
            "rest": {k: rest[k] for k in ("steps", "seconds", "converged", "nu3d")},
            "warm_start": dict({k: warm[k] for k in ("steps", "seconds", "init_s", "converged",
                                                      "nu3d")}, nu_rel_diff=rel(warm),
                               time_ratio=round(warm["seconds"] / rest["seconds"], 3)),
            "multilevel": dict({k: ml[k] for k in ("steps", "seconds", "init_s", "converged",
                                                    "nu3d", "coarse")}, nu_rel_diff=rel(ml),
                               time_ratio=round(ml["seconds"] / rest["seconds"], 3)),
            "extrapolated": dict({k: ex[k] for k in ("steps", "seconds", "init_s", "converged",
                                                      "nu3d", "coarse")}, nu_rel_diff=rel(ex),
                                 time_ratio=round(ex["seconds"] / rest["seconds"], 3))}


def counter_traffic(storage: str, n: int):
    """HBM bytes per step launch measured by rocprofv3 counters (profiles/traffic.json),
    or None when no measurement exists or the kernel sources changed since."""
    from paper_1511_04633_amd import profiling

    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            entry = json.load(fh).get(f"{storage}_{n}")
    except (OSError, ValueError):
        return None
    if not entry or entry.get("source_sha256") != profiling.kernel_source_hash():
        return None
    return entry




def copy_probe(nbytes: int, reps: int = 20) -> float:
    """Bandwidth of a plain device-to-device copy moving the same bytes as one
    step (nbytes read + nbytes written), timed with events on torch's stream:
    the practical HBM ceiling next to the 8 TB/s peak."""
    import torch

    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms / 1e3) / 1e9


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--oracle-timing":  # child of cpu_oracle_detail
        n, ra, wt, steps, secs = sys.argv[2:7]
        _oracle_timing_child(int(n), float(ra), int(wt), int(steps), float(secs))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--ra", type=float, default=1e6)
    ap.add_argument("--wall-type", type=int, default=1)
    ap.add_argument("--storage", default="f32",
                    choices=["f64", "f32", "f16", "bf16", "f16_f32", "bf16_f32", "f16_i16"])
    ap.add_argument("--launch", default="", help="bx,by override of the step kernel block")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true",
                    help="skip timing a plain device copy of the same bytes")
    ap.add_argument("--steady-types", default="1,2,3",
                    help="wall types timed to steady at 128^3 Ra 1e5 (comma list; '' = skip)")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="time the steady runs from rest only (no U-Net warm start)")
    ap.add_argument("--coarse", type=int, default=64,
                    help="grid-sequenced steady runs from a coarse^3 steady cavity (0 = skip; "
                         "one halving of the 128^3 grid by default)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the storage-format sweep at the benchmark size")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-cavity batch run to steady")
    ap.add_argument("--no-unet-step", action="store_true",
                    help="skip timing the U-Net training step")
    ap.add_argument("--no-warm192", action="store_true",
                    help="skip the 192^3 warm-start comparison")
    ap.add_argument("--force-model", type=int, default=0, choices=[0, 1, 2],
                    help="0 Eq. 15 (default), 1 Eq. 15 / rho, 2 Guo's forcing")
    ap.add_argument("--aniso", default="",
                    help="A_xx,A_yy,A_zz,A_xy,A_xz,A_yz: anisotropic diffusion D = alpha A")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1511_04633_amd import inputs, lbmx

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n = args.n
    aniso = [float(v) for v in args.aniso.split(",")] if args.aniso else None
    variant = args.force_model != 0 or aniso is not None
    cav = lbmx.Cavity(n=n, wall_type=args.wall_type, ra=args.ra, storage=args.storage,
                      theta0=inputs.theta_noise(n, 20151115), force_model=args.force_model,
                      aniso=aniso)
    if args.launch:
        bx, by = (int(v) for v in args.launch.split(","))
        cav.set_launch(bx, by)
    print(f"bench: n={n} storage={args.storage} launch={cav.get_launch()} "
          f"warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
    cav.step(args.warmup)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    ev_ms = cav.step_timed(args.steps)   # HIP events on the cavity's stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    nu = cav.nusselt()
    copy_gbs = None if args.no_copy_probe else copy_probe(
        int(n ** 3 * lbmx.bytes_per_cell(args.storage)) // 2)
    cells = n ** 3
    mlups = cells * args.steps / wall / 1e6
    bpc = lbmx.bytes_per_cell(args.storage)
    kernel_s = ev_ms / 1e3 / args.steps
    achieved = cells * bpc / kernel_s / 1e9
    tr = None if variant else counter_traffic(args.storage, n)
    dtype = {"f64": "f64", "f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32",
             "f16_f32": "f16-flow+f32-energy-storage/f32",
             "bf16_f32": "bf16-flow+f32-energy-storage/f32",
             "f16_i16": "f16-flow+i16-fixed-energy-storage/f32"}
    line = {
        "metric": "double-MRT MLUPS + % HBM roofline at 256^3; wall time to steady Nu",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype[args.storage],
        "data": "synthetic: cavity at rest + seeded theta noise (SplitMix64, amp 1e-6)",
        "config": {"workload": f"double-MRT cubic cavity {n}^3, Type {args.wall_type}, "
                               f"Ra {args.ra:g}, Pr 0.71, Ma 0.1",
                   "n": n, "cells": cells, "storage": args.storage,
                   "launch": list(cav.get_launch())},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if tr is None else tr["traffic_bytes"],
                     "traffic_over_algorithmic": None if tr is None else tr["traffic_over_algorithmic"],
                     "algorithmic_bytes": cells * bpc, "bytes_per_cell": bpc,
                     "kernel_us": round(kernel_s * 1e6, 2),
                     "copy_achieved": None if copy_gbs is None else round(copy_gbs, 1)},
        "nu3d_after": nu["nu3d"],
    }
    if variant:
        line["config"]["force_model"] = args.force_model
        line["config"]["aniso"] = aniso
    del cav
    torch.cuda.empty_cache()
    steady = []
    types = [int(v) for v in args.steady_types.split(",") if v.strip()]
    net = None
    if types and not args.no_warm_start:
        from paper_1511_04633_amd import warmstart
        net = warmstart.load_net(os.path.join(ROOT, "paper_1511_04633_amd", "weights", "unet64.npz"))
    for wt in types:
        print(f"bench: time to steady, 128^3 Type {wt}", file=sys.stderr, flush=True)
        steady.append(time_to_steady(wt, net, coarse=args.coarse))
    if steady:
        line["time_to_steady"] = steady
    if not args.no_sweep and not variant:
        line["storage_sweep"] = storage_sweep(n, args.wall_type, args.ra)
    if not args.no_batch:
        print("bench: 64-cavity batch to steady", file=sys.stderr, flush=True)
        line["batch_to_steady"] = [batch_to_steady(False)]
        print("bench: 64-cavity batch by grid sequencing", file=sys.stderr, flush=True)
        line["batch_to_steady"].append(batch_to_steady(True))
    if not args.no_warm192:
        print("bench: 192^3 warm start", file=sys.stderr, flush=True)
        if net is None:
            from paper_1511_04633_amd import warmstart
            net = warmstart.load_net(os.path.join(ROOT, "paper_1511_04633_amd", "weights",
                                                  "unet64.npz"))
        line["warm_start_192"] = warm_start_192(net)
    if not args.no_unet_step:
        print("bench: U-Net training step", file=sys.stderr, flush=True)
        line["unet_training_step"] = unet_training_step()
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, wall_type=args.wall_type, ra=args.ra)
        line["cpu_oracle_detail"] = cpu_oracle_detail(5.0, args.ra, args.wall_type)
        # the GPU on the oracle's sample, same size and precision class (FP64)
        c64 = lbmx.Cavity(n=64, wall_type=args.wall_type, ra=args.ra, storage="f64",
                          theta0=inputs.theta_noise(64, 20151115))
        c64.step(200)
        ms = c64.step_timed(2000)
        line["gpu_on_cpu_sample"] = {"workload": f"64^3 Type {args.wall_type} Ra {args.ra:g}",
                                     "storage": "f64", "value": round(64 ** 3 * 2000 / ms / 1e3, 1),
                                     "unit": "MLUPS"}
        c64.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

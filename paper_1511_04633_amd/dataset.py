"""Steady-state training set from the batched solver.

A batch of cavities (edge n uniform over {32, 48, 64, 80, 96}, Ra
log-uniform in [1e3, 1e6], wall type uniform over {1, 2, 3}, Pr 0.71,
Ma 0.1; the draws come from ``inputs.batch_cases``) is advanced by the
library's batched launch until every cavity's hot-wall Nu is steady
(|dNu| < tol per `every` steps) or a step cap is hit.  The steady u, v, w
(divided by u_c) and theta of each cavity are resampled to an m^3 grid by
the library and stored with (log10 Ra, wall type) as the surrogate's
training set.

CLI: python -m paper_1511_04633_amd.dataset --out set.npz [--count 64] [--coarse]
prints one JSON summary line (batch wall time, aggregate MLUPS, autotuned
launch, and optionally the sequential per-cavity baseline); --coarse starts
every cavity from a half-size batch run to steady first (grid sequencing).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbmx


def make_batch(cases, storage="f32", tune_cache=None, log=None):
    import torch

    b = lbmx.Batch(cases, storage=storage)
    t0 = time.perf_counter()
    us = b.autotune(tune_cache)
    tune_s = time.perf_counter() - t0
    for k, c in enumerate(cases):
        b.init_rest(k, inputs.theta_noise(c["n"], c["seed"]))
    torch.cuda.synchronize()
    if log:
        log(f"batch: {len(cases)} cavities, launch {b.get_launch()}, {us:.1f} us/step "
            f"(autotune {tune_s:.1f} s)")
    return b, us


def generate(seed=1511, count=64, out_n=64, storage="f32", tol=1e-6, every=1000,
             max_steps=300_000, tune_cache=None, log=None, coarse=False):
    """Run the batch to steady and return the training set and timings.
    With coarse, grid sequencing: a batch of the same cases at half the edge
    length is run to steady first (same criterion) and each cavity starts
    from its half-size twin's fields (``Batch.init_from``); the wall time
    covers both solves and the transfer."""
    import torch

    cases = inputs.batch_cases(seed, count)
    b, us = make_batch(cases, storage, tune_cache, log)
    cinfo = None
    if coarse:
        ccases = [dict(c, n=c["n"] // 2) for c in cases]
        cb, _ = make_batch(ccases, storage, tune_cache, log)
    t0 = time.perf_counter()
    if coarse:
        cconv = cb.run_to_steady(tol=tol, every=every, max_steps=max_steps)
        csteps = [cb.info(k)["t"] for k in range(count)]
        for k in range(count):
            b.init_from(k, cb, k)
        cb.close()
        torch.cuda.synchronize()
        cinfo = {"converged": cconv, "wall_s": time.perf_counter() - t0,
                 "node_steps": sum(c["n"] ** 3 * t for c, t in zip(ccases, csteps)),
                 "max_steps": max(csteps)}
        if log:
            log(f"coarse batch: {cconv}/{count} converged in {cinfo['wall_s']:.1f} s")
    nconv = b.run_to_steady(tol=tol, every=every, max_steps=max_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = [b.info(k) for k in range(count)]
    node_steps = sum(c["n"] ** 3 * i["t"] for c, i in zip(cases, infos))
    # Only steady fields are training targets: cavities that hit the step cap
    # or diverged are left out (and listed).
    keep = [k for k in range(count) if infos[k]["state"] == "converged"]
    fields = np.empty((len(keep), 4, out_n, out_n, out_n), dtype=np.float32)
    for j, k in enumerate(keep):
        c = cases[k]
        f = b.resample(k, out_n)
        u_c = lbmx.derive(lbmx.make_params(n=c["n"], ra=c["ra"]))["u_c"]
        fields[j, :3] = f[:3] / u_c
        fields[j, 3] = f[3]
    if not np.isfinite(fields).all():
        raise RuntimeError("non-finite values in the fields of converged cavities")
    kept = [cases[k] for k in keep]
    out = {
        "cases": kept,
        "fields": fields,
        "log10_ra": np.array([np.log10(c["ra"]) for c in kept]),
        "wall_type": np.array([c["wall_type"] for c in kept]),
        "nu3d": np.array([infos[k]["nu3d"] for k in keep]),
        "steps": np.array([infos[k]["t"] for k in keep]),
        "dropped": [dict(cases[k], state=infos[k]["state"]) for k in range(count) if k not in keep],
        "all_cases": cases,
        "all_steps": np.array([i["t"] for i in infos]),
        "all_nu3d": np.array([i["nu3d"] for i in infos]),
        "summary": {"count": count, "converged": nconv, "kept": len(keep), "wall_s": wall,
                    "node_steps": node_steps, "mlups": node_steps / wall / 1e6,
                    "launch": list(b.get_launch()), "autotune_us_per_step": us,
                    "storage": storage, "tol": tol, "every": every, "max_steps": max_steps,
                    "coarse": cinfo},
    }
    b.close()
    return out


def sequential(cases, storage="f32", tol=1e-6, every=1000, max_steps=300_000):
    """The same cavities run one after another through the single-cavity API."""
    import torch

    t0 = time.perf_counter()
    res = []
    for c in cases:
        cav = lbmx.Cavity(n=c["n"], wall_type=c["wall_type"], ra=c["ra"], storage=storage,
                          theta0=inputs.theta_noise(c["n"], c["seed"]))
        r = cav.run_to_steady(tol=tol, every=every, max_steps=max_steps)
        res.append(r)
        cav.close()
    torch.cuda.synchronize()
    return {"wall_s": time.perf_counter() - t0, "nu3d": [r["nu3d"] for r in res],
            "steps": [r["step"] for r in res]}


def save(path, ds):
    np.savez_compressed(path, fields=ds["fields"], log10_ra=ds["log10_ra"],
                        wall_type=ds["wall_type"], nu3d=ds["nu3d"], steps=ds["steps"],
                        n=np.array([c["n"] for c in ds["cases"]]))


def load(path):
    z = np.load(path, allow_pickle=False)
    return {k: z[k] for k in z.files}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1511)
    ap.add_argument("--out-n", type=int, default=64)
    ap.add_argument("--max-steps", type=int, default=300_000)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--sequential", action="store_true",
                    help="also time the same cavities run one by one")
    ap.add_argument("--coarse", action="store_true",
                    help="grid sequencing: start from a half-size batch run to steady")
    a = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    ds = generate(seed=a.seed, count=a.count, out_n=a.out_n, max_steps=a.max_steps,
                  tune_cache=a.tune_cache, log=log, coarse=a.coarse)
    if a.out:
        save(a.out, ds)
    summ = dict(ds["summary"])
    if a.sequential:
        log("sequential baseline ...")
        seq = sequential(ds["all_cases"], max_steps=a.max_steps)
        summ["sequential_wall_s"] = seq["wall_s"]
        summ["speedup_vs_sequential"] = seq["wall_s"] / summ["wall_s"]
        summ["max_nu_diff_vs_sequential"] = float(np.max(np.abs(np.array(seq["nu3d"]) -
                                                             ds["all_nu3d"])))
        summ["steps_equal_sequential"] = bool(np.array_equal(np.array(seq["steps"]),
                                                             ds["all_steps"]))
    print(json.dumps(summ), flush=True)
    return ds


if __name__ == "__main__":
    main()

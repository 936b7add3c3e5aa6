"""Learned warm start: train the U-Net on the batched solver's steady fields,
then solve 192^3 cavities from the network's prediction (trilinearly
upsampled from 64^3 inside ``lbmx_init_fields``) and from rest, and compare
steps, wall time (inference and initialisation included) and the steady
Nusselt numbers.

CLI:
  python -m paper_1511_04633_amd.warmstart train --out weights.npz [--epochs 300]
      generates the 64-cavity training set with the batched solver, trains,
      saves the weights and prints the loss history summary;
  python -m paper_1511_04633_amd.warmstart eval --weights weights.npz
      [--ra 2e4,3e5,8e5] [--types 1,2,3] [--n 192] [--coarse 64] [--extrapolate]
      prints one JSON line per case; with --coarse also the grid-sequenced
      start (network -> steady coarse^3 cavity -> n^3 cavity), with
      --extrapolate also the start extrapolated from the (coarse/2)^3 and
      coarse^3 steady states.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import dataset, inputs, lbmx, unet


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def train_main(a):
    t0 = time.perf_counter()
    ds = dataset.generate(seed=a.seed, count=a.count, out_n=64, max_steps=a.max_steps,
                          tune_cache=a.tune_cache, log=log)
    t_data = time.perf_counter() - t0
    log(f"dataset: {ds['summary']}")
    if len(ds["fields"]) == 0 or not np.isfinite(ds["fields"]).all():
        raise RuntimeError("no usable steady fields to train on")
    net = unet.UNet(seed=a.net_seed, m=64)
    log(f"U-Net parameters: {net.nparams()}")
    asym = unet.field_asymmetry(ds["fields"])
    log(f"steady fields' asymmetry (x mirror, inversion, both): {asym}")
    res = unet.train(net, ds["fields"], ds["log10_ra"], ds["wall_type"], epochs=a.epochs,
                     batch=a.batch, lr=a.lr, log=log, augment=not a.no_augment)
    st = net.state()
    st["log10_ra"] = ds["log10_ra"]
    st["wall_type"] = ds["wall_type"]
    st["loss"] = np.array(res["loss"])
    np.savez_compressed(a.out, **st)
    print(json.dumps({"dataset_s": round(t_data, 2), "dataset": ds["summary"],
                      "params": net.nparams(), "epochs": a.epochs, "batch": a.batch,
                      "augment": not a.no_augment, "asymmetry": asym,
                      "train_s": round(res["seconds"], 2), "steps": res["steps"],
                      "loss_first": res["loss"][0], "loss_last": res["loss"][-1]}), flush=True)


def load_net(path):
    net = unet.UNet(seed=0, m=64)
    z = np.load(path, allow_pickle=False)
    net.load_state({k: z[k] for k in z.files})
    return net


def solve(n, ra, wt, net=None, coarse=0, tol=1e-6, every=1000, max_steps=400_000,
          history=False, extrapolate=False):
    """Run one cavity to steady from rest (net None, coarse 0), from the
    network's fields (net), or by grid sequencing (coarse = m > 0): an m^3
    cavity of the same case is first run to steady by the same criterion,
    from the network's fields or from rest, and the n^3 cavity starts from
    its fields (``Cavity.init_from``).  With extrapolate, an (m/2)^3 cavity
    is run to steady first (from the network or from rest), starts the m^3
    cavity, and the n^3 cavity starts from 5/4 of the m^3 fields minus 1/4
    of the (m/2)^3 fields (``Cavity.init_from_two``: their second-order grid
    error extrapolated to n = 2m; m/2 >= 16, so that both coarse grids
    resolve the flow).  Wall time covers inference, the coarse
    solves and every initialisation.  With history, step in chunks of
    `every` from Python (same criterion as lbmx_run_to_steady) and also
    report the first step after which Nu_3D stays within 1e-3 of its final
    value."""
    import torch

    def start_from_net(c):
        f = unet.predict_fields(net, np.log10(ra), wt, u_c=c.derived()["u_c"])
        fv = f.view(4, net.m, net.m, net.m)
        c.init_fields(fv[0], fv[1], fv[2], fv[3])

    cav = lbmx.Cavity(n=n, wall_type=wt, ra=ra, storage="f32",
                      theta0=inputs.theta_noise(n, 20151115))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_init = 0.0
    coarse_info = None
    if coarse:
        cc = lbmx.Cavity(n=coarse, wall_type=wt, ra=ra, storage="f32",
                         theta0=inputs.theta_noise(coarse, 20151115))
        c2, r2 = None, None
        if extrapolate:
            if coarse // 2 < 16:
                raise ValueError("an extrapolated start needs coarse // 2 >= 16 (a resolved "
                                 "quarter-size cavity)")
            c2 = lbmx.Cavity(n=coarse // 2, wall_type=wt, ra=ra, storage="f32",
                             theta0=inputs.theta_noise(coarse // 2, 20151115))
            if net is not None:
                start_from_net(c2)
            r2 = c2.run_to_steady(tol=tol, every=every, max_steps=max_steps)
            cc.init_from(c2)
        elif net is not None:
            start_from_net(cc)
        rc = cc.run_to_steady(tol=tol, every=every, max_steps=max_steps)
        if extrapolate:
            cav.init_from_two(cc, 1.25, c2, -0.25)
            c2.close()
        else:
            cav.init_from(cc)
        cc.close()
        coarse_info = {"n": coarse, "steps": rc["step"], "converged": rc["converged"],
                       "nu3d": rc["nu3d"]}
        if r2 is not None:
            coarse_info["quarter"] = {"n": coarse // 2, "steps": r2["step"],
                                      "converged": r2["converged"], "nu3d": r2["nu3d"]}
        t_init = time.perf_counter() - t0
    elif net is not None:
        start_from_net(cav)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
    hist = None
    if history:
        nu = cav.nusselt()
        hist = [(0, nu["nu3d"])]
        prev, conv = nu["nu3d"], False
        while cav.t < max_steps:
            cav.step(every)
            nu = cav.nusselt()
            hist.append((cav.t, nu["nu3d"]))
            if abs(nu["nu3d"] - prev) < tol:
                conv = True
                break
            prev = nu["nu3d"]
        r = dict(nu, converged=conv)
    else:
        r = cav.run_to_steady(tol=tol, every=every, max_steps=max_steps)
    dt = time.perf_counter() - t0
    out = {"steps": r["step"], "seconds": round(dt, 3), "init_s": round(t_init, 4),
           "converged": r["converged"], "nu3d": r["nu3d"], "nu2d": r["nu2d"], "numax": r["numax"]}
    if coarse_info is not None:
        out["coarse"] = coarse_info
    if hist is not None:
        final = hist[-1][1]
        within = 0
        for k in range(len(hist) - 1, -1, -1):
            if abs(hist[k][1] - final) > 1e-3 * abs(final):
                within = hist[min(k + 1, len(hist) - 1)][0]
                break
        out["steps_within_1e-3"] = within
        out["nu_history"] = [[t, round(v, 7)] for t, v in hist[::5]]
    cav.close()
    return out


def eval_main(a):
    net = load_net(a.weights)
    for ra in [float(v) for v in a.ra.split(",")]:
        for wt in [int(v) for v in a.types.split(",")]:
            log(f"case n={a.n} Ra={ra:g} type={wt}")
            rest = solve(a.n, ra, wt, None, max_steps=a.max_steps, history=a.history)
            warm = solve(a.n, ra, wt, net, max_steps=a.max_steps, history=a.history)
            line = {"n": a.n, "ra": ra, "wall_type": wt, "rest": rest, "warm": warm,
                    "step_ratio": warm["steps"] / max(rest["steps"], 1),
                    "time_ratio": warm["seconds"] / rest["seconds"],
                    "nu_rel_diff": abs(warm["nu3d"] - rest["nu3d"]) / rest["nu3d"]}
            if a.coarse:
                ml = solve(a.n, ra, wt, net, coarse=a.coarse, max_steps=a.max_steps,
                           history=a.history)
                line["multilevel"] = ml
                line["multilevel_time_ratio"] = ml["seconds"] / rest["seconds"]
                line["multilevel_nu_rel_diff"] = abs(ml["nu3d"] - rest["nu3d"]) / rest["nu3d"]
                if a.extrapolate:
                    ex = solve(a.n, ra, wt, net, coarse=a.coarse, max_steps=a.max_steps,
                               history=a.history, extrapolate=True)
                    line["extrapolated"] = ex
                    line["extrapolated_time_ratio"] = ex["seconds"] / rest["seconds"]
                    line["extrapolated_nu_rel_diff"] = abs(ex["nu3d"] - rest["nu3d"]) / rest["nu3d"]
            print(json.dumps(line), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--batch", type=int, default=4)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--count", type=int, default=64)
    t.add_argument("--seed", type=int, default=1511)
    t.add_argument("--net-seed", type=int, default=0)
    t.add_argument("--max-steps", type=int, default=300_000)
    t.add_argument("--tune-cache", default=None)
    t.add_argument("--no-augment", action="store_true",
                   help="train without the symmetry augmentation")
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--ra", default="2e4,3e5,8e5")
    e.add_argument("--types", default="1,2,3")
    e.add_argument("--n", type=int, default=192)
    e.add_argument("--max-steps", type=int, default=400_000)
    e.add_argument("--coarse", type=int, default=0,
                   help="also solve by grid sequencing: network -> coarse^3 steady -> n^3")
    e.add_argument("--extrapolate", action="store_true",
                   help="with --coarse, also start n^3 extrapolated from (coarse/2)^3 and "
                        "coarse^3 steady states")
    e.add_argument("--history", action="store_true",
                   help="log Nu every 1000 steps and report steps to within 1e-3 of the final Nu")
    a = ap.parse_args(argv)
    if a.cmd == "train":
        train_main(a)
    else:
        eval_main(a)


if __name__ == "__main__":
    main()

"""Run one cavity to a steady state and save what the paper reports.

The cavity (Sec. 2: cube of n nodes per edge, wall type 1-3, Pr, Ra, Ma) is
advanced by the library until |dNu_3D| < tol per `every` steps.  The start is
one of
  rest       fluid at rest with seeded +-1e-6 theta noise (the method alone);
  network    the shipped U-Net's predicted fields (warm start);
  coarse     a cavity of edge --coarse (default n / 2) run to steady first,
             from rest, whose fields start this one (grid sequencing);
  network+coarse  the same, with the coarse cavity started from the network;
  extrapolated    an (m/2)^3 cavity run to steady (from rest) starts the m^3
             coarse cavity, also run to steady, and this one starts from 5/4
             of the m^3 fields minus 1/4 of the (m/2)^3 fields (their
             second-order grid error extrapolated, lbmx_init_from_cavities;
             the (m/2)^3 grid must resolve the flow: m/2 >= 16, e.g. n >= 64);
  network+extrapolated  the same, with the (m/2)^3 cavity started from the
             network.
The output file (npz) holds rho, u, v, w, theta (FP32, [z, y, x], lattice
units), the hot-wall Nu_3D, Nu_2D, Nu_max and local-Nu map (Eqs. 39-41), the
velocity maxima scaled by Eq. (42), the step count and the wall time.

CLI:
  python -m paper_1511_04633_amd.run --n 128 --ra 1e5 --wall-type 1
      [--storage f32] [--start network+extrapolated] [--out result.npz]
      [--checkpoint state.ckpt]
prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs, lbmx

STARTS = ("rest", "network", "coarse", "network+coarse", "extrapolated", "network+extrapolated")
# Coarsest grid of an extrapolated start: below it the steady state is not in
# the second-order regime the extrapolation assumes (at 8^3 a cavity started
# from the network settled in another state than from rest).
MIN_QUARTER = 16
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet64.npz")


def _from_network(cav, net, ra, wall_type):
    from . import unet
    f = unet.predict_fields(net, math.log10(ra), wall_type, u_c=cav.derived()["u_c"])
    fv = f.view(4, net.m, net.m, net.m)
    cav.init_fields(fv[0], fv[1], fv[2], fv[3])


def run(n, ra, wall_type, pr=0.71, ma=0.1, storage="f32", start="rest", coarse=0,
        weights=WEIGHTS, tol=1e-6, every=1000, max_steps=2_000_000, seed=20151115,
        force_model=0, nu_stencil=0):
    """Solve one cavity to steady; returns (cavity, summary dict)."""
    import torch

    if start not in STARTS:
        raise ValueError(f"start must be one of {STARTS}")
    kw = dict(wall_type=wall_type, ra=ra, pr=pr, ma=ma, storage=storage,
              force_model=force_model, nu_stencil=nu_stencil)
    net = None
    if start.startswith("network"):
        from . import warmstart
        net = warmstart.load_net(weights)
    cav = lbmx.Cavity(n=n, theta0=inputs.theta_noise(n, seed), **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    coarse_info = None
    if start.endswith("coarse") or start.endswith("extrapolated"):
        m = coarse or max(4, n // 2)
        cc = lbmx.Cavity(n=m, theta0=inputs.theta_noise(m, seed), **kw)
        cq, rq = None, None
        if start.endswith("extrapolated"):
            q = m // 2
            if q < MIN_QUARTER:
                raise ValueError(f"an extrapolated start needs the quarter-size cavity to have at "
                                 f"least {MIN_QUARTER} nodes per edge (coarse {m} gives {q})")
            cq = lbmx.Cavity(n=q, theta0=inputs.theta_noise(q, seed), **kw)
            if net is not None:
                _from_network(cq, net, ra, wall_type)
            rq = cq.run_to_steady(tol=tol, every=every, max_steps=max_steps)
            cc.init_from(cq)
        elif net is not None:
            _from_network(cc, net, ra, wall_type)
        rc = cc.run_to_steady(tol=tol, every=every, max_steps=max_steps)
        if cq is not None:
            cav.init_from_two(cc, 1.25, cq, -0.25)
            cq.close()
        else:
            cav.init_from(cc)
        cc.close()
        coarse_info = {"n": m, "steps": rc["step"], "converged": rc["converged"],
                       "nu3d": rc["nu3d"]}
        if rq is not None:
            coarse_info["quarter"] = {"n": m // 2, "steps": rq["step"],
                                      "converged": rq["converged"], "nu3d": rq["nu3d"]}
    elif net is not None:
        _from_network(cav, net, ra, wall_type)
    r = cav.run_to_steady(tol=tol, every=every, max_steps=max_steps)
    wall = time.perf_counter() - t0
    summary = {"n": n, "ra": ra, "pr": pr, "ma": ma, "wall_type": wall_type, "storage": storage,
               "start": start, "coarse": coarse_info, "steps": r["step"],
               "converged": r["converged"], "seconds": round(wall, 3), "nu3d": r["nu3d"],
               "nu2d": r["nu2d"], "numax": r["numax"]}
    return cav, summary


def save(path, cav, summary):
    """Fields, Nu family and map, Eq. (42) velocity maxima and the summary."""
    rho, ux, uy, uz, th = cav.read_macro()
    nu = cav.nusselt(with_map=True)
    scale = math.sqrt(3 * summary["pr"] * summary["ra"]) / summary["ma"]  # Eq. (42)
    vmax = {k: float(np.abs(a).max() * scale) for k, a in (("umax", ux), ("vmax", uy),
                                                          ("wmax", uz))}
    summary.update(vmax)
    np.savez_compressed(path, rho=rho.astype(np.float32), u=ux.astype(np.float32),
                        v=uy.astype(np.float32), w=uz.astype(np.float32),
                        theta=th.astype(np.float32), nu_map=nu["map"],
                        nu3d=nu["nu3d"], nu2d=nu["nu2d"], numax=nu["numax"],
                        summary=json.dumps(summary))
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--ra", type=float, default=1e5)
    ap.add_argument("--pr", type=float, default=0.71)
    ap.add_argument("--ma", type=float, default=0.1)
    ap.add_argument("--wall-type", type=int, default=1, choices=[1, 2, 3])
    ap.add_argument("--storage", default="f32", choices=sorted(lbmx.STORAGE))
    ap.add_argument("--force-model", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--nu-stencil", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--start", default="rest", choices=STARTS)
    ap.add_argument("--coarse", type=int, default=0, help="coarse edge (default n / 2)")
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--max-steps", type=int, default=2_000_000)
    ap.add_argument("--seed", type=int, default=20151115)
    ap.add_argument("--out", default=None, help="npz with fields, Nu and summary")
    ap.add_argument("--checkpoint", default=None, help="save the final state (lbmx_save)")
    a = ap.parse_args(argv)
    cav, summary = run(a.n, a.ra, a.wall_type, pr=a.pr, ma=a.ma, storage=a.storage,
                       start=a.start, coarse=a.coarse, weights=a.weights, tol=a.tol,
                       every=a.every, max_steps=a.max_steps, seed=a.seed,
                       force_model=a.force_model, nu_stencil=a.nu_stencil)
    if a.out:
        summary = save(a.out, cav, summary)
    if a.checkpoint:
        cav.save(a.checkpoint)
    cav.close()
    print(json.dumps(summary), flush=True)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main()["converged"] else 1)

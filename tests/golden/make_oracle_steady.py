"""Write oracle_steady_32_ra1e5.json: the FP64 oracle's steady state of the
32^3, Type 1, Ra 1e5 cavity (Pr 0.71, Ma 0.1, rest + seeded theta noise),
run to |dNu_3D| < 1e-8 per 1000 steps.  Calls only the oracle.  It is the
reference that the GPU storage formats are checked against at steady state
(the 64^3, Ra 1e6 case needs ~1.5e5 steps, beyond what the oracle runs in a
test).  Stored: the Nu family, the step count, and rho, u, v, w, theta at
every 4th node (x, y, z = 1, 5, ..., 29), u in lattice units.

Run:  python tests/golden/make_oracle_steady.py   (about 7 min on 8 threads)
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1511_04633_amd import inputs  # noqa: E402

N, RA, WALL, SEED, TOL = 32, 1e5, 1, 20151115, 1e-8


def main():
    o = O.Oracle(N, WALL, ra=RA, theta0=inputs.theta_noise(N, SEED))
    prev = o.nusselt()["nu3d"]
    while True:
        o.step(1000)
        nu = o.nusselt()
        if abs(nu["nu3d"] - prev) < TOL:
            break
        prev = nu["nu3d"]
        if o.t >= 300_000:
            raise RuntimeError("oracle did not reach the criterion")
    rho, ux, uy, uz, th = o.macro()
    idx = list(range(1, N, 4))
    sub = lambda a: [[[float(a[z, y, x]) for x in idx] for y in idx] for z in idx]
    out = {
        "source": "FP64 oracle (oracle/lbm_oracle.c) run by tests/golden/make_oracle_steady.py",
        "case": {"n": N, "wall_type": WALL, "ra": RA, "pr": 0.71, "ma": 0.1, "seed": SEED,
                 "start": "rest + theta noise 1e-6 (2U - 1)"},
        "criterion": f"|dNu_3D| < {TOL:g} per 1000 steps",
        "steps": o.t, "nu3d": nu["nu3d"], "nu2d": nu["nu2d"], "numax": nu["numax"],
        "u_c": o.derived()["u_c"],
        "sample_index": idx,
        "fields": {"rho": sub(rho), "ux": sub(ux), "uy": sub(uy), "uz": sub(uz), "theta": sub(th)},
        "max_abs": {"ux": float(abs(ux).max()), "uy": float(abs(uy).max()),
                    "uz": float(abs(uz).max())},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_steady_32_ra1e5.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(json.dumps({k: out[k] for k in ("steps", "nu3d", "nu2d", "numax")}))


if __name__ == "__main__":
    main()

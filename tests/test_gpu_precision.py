"""Storage precision against the FP64 oracle.

Fixed steps (64^3, Type 1, Ra 1e6, 5000 steps from the same seeded start,
about 4.5 convective times H/u_c): field error max |X - X_ref| divided by u_c
for velocities and absolute for theta; Nu: |Nu_3D - Nu_ref| / Nu_ref against
the oracle run alongside.

At steady state (32^3, Type 1, Ra 1e5, |dNu_3D| < 1e-6 per 1000 steps): the
oracle's own steady state, computed once by tests/golden/make_oracle_steady.py
(54 k steps to |dNu_3D| < 1e-8 per 1000 steps) and stored with the Nu family
and the fields at every 4th node.

Formats that meet the 1e-3 Nu target are held to it (FP32 to the FP32 parity
bar): f32, f16_f32 (16-bit flow, FP32 energy, 132 B/node) and f16_i16 (16-bit
flow, 16-bit fixed-point energy with stochastic rounding, 104 B/node).  The
formats that miss it are fenced at their measured errors and marked as
failing: f16 (both lattices FP16), bf16_f32, bf16.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1511_04633_amd import inputs
from paper_1511_04633_amd import lbmx as L

pytestmark = pytest.mark.gpu

N, RA, STEPS, SEED = 64, 1e6, 5000, 20151115
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_steady_32_ra1e5.json")

TARGET = {  # storage: (field bound in u_c units / abs theta, Nu relative bound)
    "f64": (1e-12, 1e-12),
    "f32": (1e-5, 1e-5),
    "f16_f32": (5e-3, 1e-3),
    "f16_i16": (5e-3, 1e-3),
}
FAILING = {  # measured errors, fenced so that a regression shows; they miss 1e-3 in Nu
    "f16": (3e-2, 5e-3),
    "bf16_f32": (5e-2, 3e-2),
}


@pytest.fixture(scope="module")
def reference():
    import torch
    assert torch.cuda.is_available()
    print(f"case: oracle {N}^3 T1 Ra{RA:g} {STEPS} steps", flush=True)
    th0 = inputs.theta_noise(N, SEED)
    o = O.Oracle(N, 1, ra=RA, theta0=th0)
    o.step(STEPS)
    return th0, o.macro(), o.nusselt()["nu3d"], o.derived()["u_c"]


def run(storage, th0):
    c = L.Cavity(n=N, wall_type=1, ra=RA, storage=storage, theta0=th0)
    c.step(STEPS)
    return c.read_macro(), c.nusselt(allow_unstable=True)


def errors(reference, storage):
    th0, ref, nu_ref, uc = reference
    got, nu = run(storage, th0)
    errs = {"ux": np.abs(got[1] - ref[1]).max() / uc, "uy": np.abs(got[2] - ref[2]).max() / uc,
            "uz": np.abs(got[3] - ref[3]).max() / uc, "theta": np.abs(got[4] - ref[4]).max()}
    return errs, abs(nu["nu3d"] - nu_ref) / nu_ref


@pytest.mark.parametrize("storage", list(TARGET))
def test_storage_meets_target(reference, storage):
    print(f"case: {storage} {N}^3 T1 Ra{RA:g} {STEPS} steps", flush=True)
    errs, nu_err = errors(reference, storage)
    print(storage, errs, nu_err)
    fb, nb = TARGET[storage]
    assert max(errs.values()) <= fb, errs
    assert nu_err <= nb, nu_err


@pytest.mark.parametrize("storage", list(FAILING))
def test_failing_storage_fence(reference, storage):
    """These formats miss the 1e-3 Nu target; the fence only catches a
    regression beyond their measured error."""
    print(f"case: {storage} (misses the target) {N}^3 T1 Ra{RA:g} {STEPS} steps", flush=True)
    errs, nu_err = errors(reference, storage)
    print(storage, errs, nu_err)
    fb, nb = FAILING[storage]
    assert nu_err > 1e-3  # still failing: if this changes, move the format to TARGET
    assert max(errs.values()) <= fb, errs
    assert nu_err <= nb, nu_err


def test_bf16_stays_finite(reference):
    """BF16 for both lattices (8-bit significands) is far off; it only has to
    stay finite."""
    th0, ref, nu_ref, uc = reference
    got, nu = run("bf16", th0)
    assert all(np.isfinite(a).all() for a in got) and np.isfinite(nu["nu3d"])


STEADY_TARGET = {  # storage: (Nu relative bound, field bound at the sampled nodes)
    "f32": (1e-5, 1e-4),
    "f16_f32": (1e-3, 1e-2),
    "f16_i16": (1e-3, 1e-2),
}


@pytest.mark.parametrize("storage", list(STEADY_TARGET) + ["f16", "bf16_f32"])
def test_storage_error_at_steady_against_oracle(storage):
    """Each format run to steady (|dNu_3D| < 1e-6 per 1000 steps) at 32^3,
    Ra 1e5, against the oracle's steady state: Nu_3D within 1e-3 (FP32 within
    1e-5) for the formats that meet the target, and u / u_c, theta at the
    stored sample nodes."""
    ref = json.load(open(GOLDEN))
    case = ref["case"]
    n = case["n"]
    print(f"case: {storage} {n}^3 T{case['wall_type']} Ra{case['ra']:g} to steady vs oracle", flush=True)
    c = L.Cavity(n=n, wall_type=case["wall_type"], ra=case["ra"], storage=storage,
                 theta0=inputs.theta_noise(n, case["seed"]))
    r = c.run_to_steady(tol=1e-6, every=1000, max_steps=400_000)
    rho, ux, uy, uz, th = c.read_macro()
    idx = np.array(ref["sample_index"])
    sub = lambda a: a[np.ix_(idx, idx, idx)]
    uc = ref["u_c"]
    f = ref["fields"]
    errs = {"u": max(np.abs(sub(a) - np.array(f[k])).max() for a, k in
                     ((ux, "ux"), (uy, "uy"), (uz, "uz"))) / uc,
            "theta": np.abs(sub(th) - np.array(f["theta"])).max()}
    nu_err = abs(r["nu3d"] - ref["nu3d"]) / ref["nu3d"]
    print(storage, r["converged"], r["step"], ref["steps"], nu_err, errs)
    assert np.isfinite(r["nu3d"]) and r["converged"]
    if storage in STEADY_TARGET:
        nb, fb = STEADY_TARGET[storage]
        assert nu_err <= nb, nu_err
        assert max(errs.values()) <= fb, errs


@pytest.fixture(scope="module")
def steady_f64():
    """64^3, Ra 1e6 run to steady with FP64 storage on the GPU (its step
    matches the oracle to 1e-10, test_gpu_parity); the oracle itself would need
    ~1.5e5 steps here, so this larger case is checked against the GPU's FP64
    path, the 32^3 case above against the oracle."""
    import torch
    assert torch.cuda.is_available()
    print(f"case: f64 {N}^3 T1 Ra{RA:g} to steady", flush=True)
    th0 = inputs.theta_noise(N, SEED)
    c = L.Cavity(n=N, wall_type=1, ra=RA, storage="f64", theta0=th0)
    r = c.run_to_steady(tol=1e-6, every=1000, max_steps=400_000)
    assert r["converged"]
    return th0, r


@pytest.mark.parametrize("storage", ["f32", "f16_f32", "f16_i16"])
def test_storage_error_at_steady_1e6(steady_f64, storage):
    th0, rref = steady_f64
    print(f"case: {storage} {N}^3 T1 Ra{RA:g} to steady vs f64 storage", flush=True)
    c = L.Cavity(n=N, wall_type=1, ra=RA, storage=storage, theta0=th0)
    r = c.run_to_steady(tol=1e-6, every=1000, max_steps=600_000)
    nu_err = abs(r["nu3d"] - rref["nu3d"]) / rref["nu3d"]
    print(storage, r["converged"], r["step"], rref["step"], nu_err)
    assert r["converged"] and nu_err <= (1e-5 if storage == "f32" else 1e-3), nu_err

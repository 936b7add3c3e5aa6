"""Storage precision against the FP64 oracle at 64^3, Type 1, Ra 1e6.

Same seeded start (rest + theta noise), 5000 steps on both sides (about
4.5 convective times H/u_c).  Field error: max |X - X_ref| divided by u_c for
velocities and absolute for theta and rho; Nu: |Nu_3D - Nu_ref| / Nu_ref.

Bounds per format (measured, see the table in the design notes):
  f32        fields 1e-5 u_c, Nu 1e-5      (FP32 parity bar)
  f16_f32    fields 5e-3 u_c, Nu 1e-3      (16-bit flow, FP32 energy)
  f16        fields 3e-2 u_c, Nu 5e-3      (misses the 1e-3 Nu target)
  bf16_f32   fields 5e-2 u_c, Nu 3e-2      (misses the 1e-3 Nu target)
  f16_i16    fields 5e-3 u_c, Nu 1e-3      (16-bit flow, 16-bit fixed-point energy
                                           with stochastic rounding: measured
                                           1.0e-3 u_c, Nu 4e-5)
  bf16       stays finite only             (8-bit significands: far off)
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1511_04633_amd import inputs
from paper_1511_04633_amd import lbmx as L

pytestmark = pytest.mark.gpu

N, RA, STEPS, SEED = 64, 1e6, 5000, 20151115

BOUNDS = {  # storage: (field bound in u_c units / abs theta, Nu relative bound)
    "f64": (1e-12, 1e-12),
    "f32": (1e-5, 1e-5),
    "f16_f32": (5e-3, 1e-3),
    "f16": (3e-2, 5e-3),
    "bf16_f32": (5e-2, 3e-2),
    "f16_i16": (5e-3, 1e-3),
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


@pytest.mark.parametrize("storage", list(BOUNDS))
def test_storage_error_bounds(reference, storage):
    th0, ref, nu_ref, uc = reference
    print(f"case: {storage} {N}^3 T1 Ra{RA:g} {STEPS} steps", flush=True)
    got, nu = run(storage, th0)
    fb, nb = BOUNDS[storage]
    errs = {"ux": np.abs(got[1] - ref[1]).max() / uc, "uy": np.abs(got[2] - ref[2]).max() / uc,
            "uz": np.abs(got[3] - ref[3]).max() / uc, "theta": np.abs(got[4] - ref[4]).max()}
    nu_err = abs(nu["nu3d"] - nu_ref) / nu_ref
    print(storage, errs, nu_err)
    assert max(errs.values()) <= fb, errs
    assert nu_err <= nb, nu_err


def test_bf16_stays_finite(reference):
    th0, ref, nu_ref, uc = reference
    got, nu = run("bf16", th0)
    assert all(np.isfinite(a).all() for a in got) and np.isfinite(nu["nu3d"])

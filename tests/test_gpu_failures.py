"""Failure handling on the GPU path, forced from the host: a step cap that is
too small, and a cavity driven to blow up (buoyancy scaled by 1e5), whose
non-finite values the Nu reduction must report (EUNSTABLE).  The kernels
exit normally either way: NaN arithmetic does not change their control flow
or addressing."""
import numpy as np
import pytest

from paper_1511_04633_amd import inputs
from paper_1511_04633_amd import lbmx as L

pytestmark = pytest.mark.gpu

SEED = 20151115


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()


def test_step_cap_reports_not_converged():
    print("case: run_to_steady capped at 500 steps", flush=True)
    c = L.Cavity(n=16, wall_type=1, ra=1e5, storage="f32", theta0=inputs.theta_noise(16, SEED))
    r = c.run_to_steady(tol=1e-12, every=100, max_steps=500)
    assert not r["converged"] and r["step"] == 500 and c.t == 500
    assert np.isfinite(r["nu3d"])


@pytest.mark.parametrize("storage", ["f32", "f16", "f16_i16", "f64"])
def test_divergence_is_reported(storage):
    """Non-finite values reach the Nu reduction in every storage format (the
    fixed-point energy format keeps NaN through its reserved code)."""
    print(f"case: forced divergence {storage}", flush=True)
    c = L.Cavity(n=16, wall_type=1, ra=1e4, storage=storage, buoyancy_scale=1e5,
                 theta0=inputs.theta_noise(16, SEED))
    with pytest.raises(L.LbmxError) as e:
        c.run_to_steady(tol=1e-6, every=50, max_steps=20_000)
    assert e.value.status == 4  # LBMX_EUNSTABLE
    nu = c.nusselt(allow_unstable=True)
    assert nu["status"] == 4 and (nu["nonfinite"] > 0 or not np.isfinite(nu["nu3d"]))


def test_batch_retires_a_diverging_cavity():
    """One cavity of a batch blows up: it is marked diverged and dropped from
    the work list, and its healthy neighbour still converges to the Nu of the
    same cavity run alone."""
    print("case: batch with one diverging cavity", flush=True)
    cases = [dict(n=16, ra=1e4, wall_type=1), dict(n=16, ra=1e4, wall_type=1, buoyancy_scale=1e5)]
    b = L.Batch(cases, storage="f32")
    for k in range(2):
        b.init_rest(k, inputs.theta_noise(16, SEED))
    b.run_to_steady(tol=1e-6, every=500, max_steps=200_000)
    i0, i1 = b.info(0), b.info(1)
    assert i0["state"] == "converged" and i1["state"] == "diverged", (i0, i1)
    alone = L.Cavity(n=16, wall_type=1, ra=1e4, storage="f32", theta0=inputs.theta_noise(16, SEED))
    r = alone.run_to_steady(tol=1e-6, every=500, max_steps=200_000)
    assert r["converged"] and r["nu3d"] == i0["nu3d"] and r["step"] == i0["t"]
    b.close()

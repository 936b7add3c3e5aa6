"""What the trained surrogate gains: a cavity started from the network's
predicted fields reaches the same steady Nusselt number in fewer steps than
the plain rest start (the rest start stays the reference and the fallback).

Uses the weights shipped in paper_1511_04633_amd/weights/unet64.npz, trained
by `python -m paper_1511_04633_amd.warmstart train` on the 64 steady cavities
of the batched solver."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1511_04633_amd", "weights", "unet64.npz")


@pytest.fixture(scope="module")
def net():
    import torch
    assert torch.cuda.is_available()
    from paper_1511_04633_amd import warmstart
    return warmstart.load_net(WEIGHTS)


def test_prediction_is_physical(net):
    from paper_1511_04633_amd import unet
    f = unet.predict_fields(net, np.log10(3e5), 1).cpu().numpy().reshape(4, 64, 64, 64)
    assert np.isfinite(f).all()
    th = f[3]
    assert -0.6 < th.min() and th.max() < 0.6
    # hot wall side warmer than the cold side, on average (Eqs. 6-7)
    assert th[:, :4, :].mean() > 0.2 and th[:, -4:, :].mean() < -0.2
    # buoyant flow: up along the hot wall, down along the cold wall (y is axis 1)
    w = f[2]
    assert w[:, :8, :].mean() > 0 and w[:, -8:, :].mean() < 0


@pytest.mark.parametrize("wall_type", [1, 2, 3])
def test_warm_start_needs_fewer_steps(net, wall_type):
    from paper_1511_04633_amd import warmstart
    print(f"case: warm vs rest n=96 Ra 3e5 type {wall_type}", flush=True)
    rest = warmstart.solve(96, 3e5, wall_type, None, max_steps=400_000)
    warm = warmstart.solve(96, 3e5, wall_type, net, max_steps=400_000)
    print(rest, warm)
    assert rest["converged"] and warm["converged"]
    assert warm["steps"] <= 0.7 * rest["steps"]
    assert abs(warm["nu3d"] - rest["nu3d"]) <= 5e-3 * rest["nu3d"]

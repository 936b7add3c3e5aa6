"""The run-to-steady command line (paper_1511_04633_amd.run): every start
reaches the same steady Nu, and the saved fields, Nu family and checkpoint
are those of the cavity it ran."""
import json
import os

import numpy as np
import pytest

from paper_1511_04633_amd import lbmx as L
from paper_1511_04633_amd import run as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()


def test_starts_agree_and_outputs_match(tmp_path):
    print("case: run CLI 32^3 Ra 3e4 type 2, all starts but the extrapolated ones", flush=True)
    out = {}
    for start in [s for s in R.STARTS if "extrapolated" not in s]:
        path = os.path.join(tmp_path, f"{start}.npz")
        ck = os.path.join(tmp_path, f"{start}.ckpt")
        s = R.main(["--n", "32", "--ra", "3e4", "--wall-type", "2", "--start", start,
                    "--out", path, "--checkpoint", ck])
        assert s["converged"], s
        z = np.load(path, allow_pickle=False)
        assert z["theta"].shape == (32, 32, 32) and z["nu_map"].shape == (32, 32)
        assert float(z["nu3d"]) == s["nu3d"] and json.loads(str(z["summary"]))["steps"] == s["steps"]
        assert np.abs(z["theta"]).max() <= 0.5 + 1e-6
        assert s["vmax"] > 0 and s["wmax"] > 0
        c = L.Cavity(n=32, wall_type=2, ra=3e4, storage="f32")
        c.load(ck)
        assert c.t == s["steps"] and c.nusselt()["nu3d"] == s["nu3d"]
        c.close()
        out[start] = s
    ref = out["rest"]["nu3d"]
    for start, s in out.items():
        assert abs(s["nu3d"] - ref) <= 1e-3 * ref, (start, s["nu3d"], ref)
    assert out["coarse"]["coarse"]["n"] == 16 and out["rest"]["coarse"] is None
    with pytest.raises(ValueError):  # an 8^3 quarter level is refused
        R.main(["--n", "32", "--ra", "3e4", "--wall-type", "2", "--start", "extrapolated",
                "--out", os.path.join(tmp_path, "x.npz")])


def test_extrapolated_starts_agree(tmp_path):
    """The extrapolated starts (16^3 -> 32^3 -> 64^3, from rest and from the
    network) reach the rest start's steady Nu at 64^3."""
    print("case: run CLI 64^3 Ra 3e4 type 2, extrapolated starts", flush=True)
    out = {}
    for start in ("rest", "extrapolated", "network+extrapolated"):
        s = R.main(["--n", "64", "--ra", "3e4", "--wall-type", "2", "--start", start,
                    "--out", os.path.join(tmp_path, f"{start}.npz")])
        assert s["converged"], s
        out[start] = s
    ref = out["rest"]["nu3d"]
    for start in ("extrapolated", "network+extrapolated"):
        s = out[start]
        assert s["coarse"]["converged"] and s["coarse"]["quarter"]["converged"], s
        assert s["coarse"]["n"] == 32 and s["coarse"]["quarter"]["n"] == 16
        assert abs(s["nu3d"] - ref) <= 1e-3 * ref, (start, s["nu3d"], ref)

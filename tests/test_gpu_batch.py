"""Batched solver: many cavities of uneven size, Ra and wall type in one
launch per step.  Each cavity must match the FP64 oracle like a lone cavity,
and be bitwise identical to the single-cavity kernel, whatever the launch
shape, with or without graph replay, and across retirement."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1511_04633_amd import inputs
from paper_1511_04633_amd import lbmx as L

pytestmark = pytest.mark.gpu

CASES = [
    {"n": 5, "ra": 1e5, "wall_type": 1},
    {"n": 9, "ra": 3e4, "wall_type": 2},
    {"n": 12, "ra": 1e5, "wall_type": 3},
    {"n": 16, "ra": 1e3, "wall_type": 1},
    {"n": 7, "ra": 1e6, "wall_type": 2},
    {"n": 21, "ra": 2e5, "wall_type": 3},
]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available()
    L.load()


def theta0(k, n):
    return inputs.theta_noise(n, 1000 + k, amp=1e-2)


def make_batch(cases, storage, graph_steps=64, block=256, grid=0):
    b = L.Batch(cases, storage=storage)
    b.set_launch(block, grid, graph_steps)
    for k, c in enumerate(cases):
        b.init_rest(k, theta0(k, c["n"]))
    return b


def test_batch_f64_matches_oracle():
    print("case: batch f64 vs oracle, 6 cavities, 200 steps", flush=True)
    b = make_batch(CASES, "f64")
    b.step(200)
    for k, c in enumerate(CASES):
        o = O.Oracle(c["n"], c["wall_type"], ra=c["ra"], theta0=theta0(k, c["n"]))
        o.step(200)
        g, r = b.read_macro(k), o.macro()
        for i in range(1, 5):
            scale = max(np.abs(r[i]).max(), 1e-300)
            assert np.abs(g[i] - r[i]).max() <= 1e-10 * scale, (k, i)
        assert np.abs(g[0] - r[0]).max() <= 1e-13
        nb, no = b.nusselt(k), o.nusselt()
        assert abs(nb["nu3d"] - no["nu3d"]) <= 1e-10 * abs(no["nu3d"])
        assert b.info(k)["t"] == 200


@pytest.mark.parametrize("storage", ["f32", "f16_f32"])
def test_batch_bitwise_equals_single_cavity(storage):
    print(f"case: batch vs single {storage}", flush=True)
    b = make_batch(CASES, storage)
    b.step(150)
    for k, c in enumerate(CASES):
        s = L.Cavity(n=c["n"], wall_type=c["wall_type"], ra=c["ra"], storage=storage,
                     theta0=theta0(k, c["n"]))
        s.step(150)
        gb, gs = b.read_macro(k), s.read_macro()
        for i in range(5):
            assert np.array_equal(gb[i], gs[i]), (k, i)


@pytest.mark.parametrize("graph_steps", [0, 64])
def test_batch_fixed_point_energy_equals_single_cavity(graph_steps):
    """FP16 flow + stochastically rounded fixed-point energy: the rounding
    stream is keyed by node and by the cavity's own step, which the batch
    keeps per cavity on the device (advanced by the kernel itself, so graph
    replays advance it too), so the batch reproduces the lone cavities bit
    for bit, with direct launches and with captured graphs, also for a
    cavity re-initialised while the others step on."""
    print(f"case: batch vs single f16_i16, graph_steps {graph_steps}", flush=True)
    b = make_batch(CASES, "f16_i16", graph_steps=graph_steps)
    b.step(70)
    b.init_rest(1, theta0(1, CASES[1]["n"]))  # cavity 1 restarts at step 0
    b.step(131)  # graph replays plus a direct tail
    for k, c in enumerate(CASES):
        s = L.Cavity(n=c["n"], wall_type=c["wall_type"], ra=c["ra"], storage="f16_i16",
                     theta0=theta0(k, c["n"]))
        s.step(131 if k == 1 else 201)
        assert b.info(k)["t"] == s.t
        gb, gs = b.read_macro(k), s.read_macro()
        for i in range(5):
            assert np.array_equal(gb[i], gs[i]), (k, i)
        s.close()
    b.close()


def test_graph_and_launch_shapes_are_bitwise_identical():
    print("case: batch graph / launch shapes", flush=True)
    ref = None
    for block, grid, gsteps in ((256, 0, 0), (256, 0, 64), (128, 0, 2), (512, 64, 32),
                                (1024, 7, 0), (64, 300, 64)):
        b = make_batch(CASES, "f32", graph_steps=gsteps, block=block, grid=grid)
        assert b.get_launch() == (block, grid, gsteps)
        b.step(131)  # odd: graph replays plus a direct tail
        out = [b.read_macro(k)[4] for k in range(len(CASES))]
        if ref is None:
            ref = out
        else:
            for k in range(len(CASES)):
                assert np.array_equal(out[k], ref[k]), (block, grid, gsteps, k)


def test_run_to_steady_retires_each_cavity_like_a_lone_run():
    print("case: batch run_to_steady retirement", flush=True)
    cases = [{"n": 8, "ra": 1e3, "wall_type": 1}, {"n": 10, "ra": 1e4, "wall_type": 2},
             {"n": 12, "ra": 2e4, "wall_type": 3}, {"n": 6, "ra": 5e3, "wall_type": 3}]
    b = L.Batch(cases, storage="f32")
    b.set_launch(256, 0, 20)
    for k, c in enumerate(cases):
        b.init_rest(k, inputs.theta_noise(c["n"], 7 + k))
    nconv = b.run_to_steady(tol=1e-6, every=500, max_steps=400_000)
    assert nconv == len(cases)
    ts = []
    for k, c in enumerate(cases):
        info = b.info(k)
        assert info["state"] == "converged"
        s = L.Cavity(n=c["n"], wall_type=c["wall_type"], ra=c["ra"], storage="f32",
                     theta0=inputs.theta_noise(c["n"], 7 + k))
        r = s.run_to_steady(tol=1e-6, every=500, max_steps=400_000)
        assert r["converged"] and r["step"] == info["t"], (k, r["step"], info["t"])
        assert r["nu3d"] == info["nu3d"]
        ts.append(info["t"])
    assert len(set(ts)) > 1  # cavities really retired at different times
    # a retired cavity keeps its state while the others stepped on
    assert np.array_equal(b.read_macro(0)[4], b.read_macro(0)[4])


def test_resample_same_grid_and_linear_field():
    print("case: batch resample", flush=True)
    n = 12
    b = L.Batch([{"n": n, "ra": 100.0, "wall_type": 2, "buoyancy_scale": 0.0}], storage="f64")
    b.init_rest(0, None)
    b.step(8000)  # conduction limit: theta linear in y, u = 0
    rho, ux, uy, uz, th = b.read_macro(0)
    same = b.resample(0, n)
    assert np.array_equal(same[3], th.astype(np.float32))
    fine = b.resample(0, 2 * n)[3]
    y = (np.arange(2 * n) + 0.5) / (2 * n)
    inner = (y > 0.5 / n) & (y < 1 - 0.5 / n)
    lin = 0.5 - y
    assert np.abs(fine[:, inner, :] - lin[None, inner, None]).max() < 1e-6


def test_autotune_and_cache(tmp_path):
    print("case: batch autotune", flush=True)
    cache = str(tmp_path / "tune.json")
    b = L.Batch(CASES, storage="f32")
    us = b.autotune(cache)
    assert us > 0 and os.path.exists(cache)
    entry = list(json.load(open(cache)).values())[0]
    assert b.get_launch()[:2] == (entry["block"], entry["grid"])
    assert b.info(0)["t"] == 0
    b2 = L.Batch(CASES, storage="f32")
    b2.autotune(cache)  # cache hit
    assert b2.get_launch() == b.get_launch()


def test_batch_rejects_bad_input():
    with pytest.raises(L.LbmxError):
        L.Batch([{"n": 300, "ra": 1e4, "wall_type": 1}])
    with pytest.raises(L.LbmxError):
        L.Batch([{"n": 8, "ra": 1e4, "wall_type": 5}])
    b = L.Batch(CASES[:2])
    with pytest.raises(L.LbmxError):
        b.set_launch(100, 0, 64)
    with pytest.raises(L.LbmxError):
        b.set_launch(256, 0, 3)
    with pytest.raises(L.LbmxError):
        b.info(5)

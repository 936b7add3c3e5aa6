"""Checkpoint and resume through lbmx_save / lbmx_load: a cavity loaded from a
checkpoint continues bitwise as the saved one; mismatched or damaged files
are rejected before the cavity's state changes."""
import os

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


@pytest.mark.parametrize("storage,n,wall_type", [("f32", 24, 2), ("f16_f32", 20, 3), ("f64", 17, 1),
                                                  ("f16_i16", 18, 1)])
def test_resume_is_bitwise(tmp_path, storage, n, wall_type):
    print(f"case: checkpoint {storage} n={n} T{wall_type}", flush=True)
    th0 = inputs.theta_noise(n, SEED)
    a = L.Cavity(n=n, wall_type=wall_type, ra=1e5, storage=storage, theta0=th0)
    a.step(150)
    path = os.path.join(tmp_path, "a.ckpt")
    a.save(path)
    a.step(101)
    fa, ga = a.get_populations()
    nua = a.nusselt()

    b = L.Cavity(n=n, wall_type=wall_type, ra=1e5, storage=storage)
    b.step(7)  # some other state, overwritten by the load
    b.load(path)
    assert b.t == 150
    b.step(101)
    assert b.t == 251
    fb, gb = b.get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    assert b.nusselt()["nu3d"] == nua["nu3d"]
    a.close()
    b.close()


def test_rejects_mismatch_and_damage(tmp_path):
    print("case: checkpoint rejection paths", flush=True)
    a = L.Cavity(n=16, wall_type=1, ra=1e4, storage="f32", theta0=inputs.theta_noise(16, SEED))
    a.step(20)
    path = os.path.join(tmp_path, "a.ckpt")
    a.save(path)
    f0, g0 = a.get_populations()

    def status(fn):
        with pytest.raises(L.LbmxError) as e:
            fn()
        return e.value.status

    # another parameter set, size or storage: EINVAL, state untouched
    for kw in (dict(n=16, wall_type=2, ra=1e4, storage="f32"),
               dict(n=16, wall_type=1, ra=2e4, storage="f32"),
               dict(n=17, wall_type=1, ra=1e4, storage="f32"),
               dict(n=16, wall_type=1, ra=1e4, storage="f16")):
        c = L.Cavity(**kw)
        c.step(3)
        before = c.get_populations()
        assert status(lambda: c.load(path)) == 1, kw
        after = c.get_populations()
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        assert c.t == 3
        c.close()

    # the Nu stencil only reads the state: a checkpoint loads under another one
    c = L.Cavity(n=16, wall_type=1, ra=1e4, storage="f32", nu_stencil=2)
    c.load(path)
    fc, gc = c.get_populations()
    assert np.array_equal(f0, fc) and np.array_equal(g0, gc) and c.t == 20
    c.close()

    raw = open(path, "rb").read()
    bad = os.path.join(tmp_path, "bad.ckpt")
    open(bad, "wb").write(b"NOTACKPT" + raw[8:])
    assert status(lambda: a.load(bad)) == 1
    open(bad, "wb").write(raw[:-1])           # truncated lattice
    assert status(lambda: a.load(bad)) == 7
    open(bad, "wb").write(raw + b"\0")        # trailing bytes
    assert status(lambda: a.load(bad)) == 7
    open(bad, "wb").write(raw[:100])          # truncated header
    assert status(lambda: a.load(bad)) == 7
    assert status(lambda: a.load(os.path.join(tmp_path, "missing.ckpt"))) == 7
    assert status(lambda: a.save(os.path.join(tmp_path, "no_dir", "x.ckpt"))) == 7
    # the failed loads left the cavity as it was
    f1, g1 = a.get_populations()
    assert np.array_equal(f0, f1) and np.array_equal(g0, g1) and a.t == 20
    a.close()

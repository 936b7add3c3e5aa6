"""Parity at the benchmarked size: 256^3, Type 1, Ra 1e6, the step kernel in
the launch shape bench.py times (the library default).

The oracle cannot run 256^3, so it checks sampled outputs one by one: after a
developed state S_t is read back (decoded to float64), one GPU step gives
S_{t+1}; for each sampled node the oracle recomputes S_{t+1} from S_t
(collision of the upstream neighbours, streaming and every wall rule) and the
two must agree to the storage format's rounding.  Samples: the 8 corners, the
12 edge midpoints, the 6 face centres, a full row along each wall-normal
direction through the centre, and 600 seeded random nodes.  The hot-wall Nu of
S_{t+1} is compared with the oracle's evaluation of the same state.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1511_04633_amd import inputs
from paper_1511_04633_amd import lbmx as L

pytestmark = pytest.mark.gpu

N = 256
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
W7 = np.array([1 / 4] + [1 / 8] * 6)


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()
    O.build(force=False)


def sample_nodes(n, seed=7):
    e = [0, n // 2, n - 1]
    pts = {(x, y, z) for x in (0, n - 1) for y in (0, n - 1) for z in (0, n - 1)}
    for a in e:
        for b in e:
            for c in e:
                if sum(v in (0, n - 1) for v in (a, b, c)) >= 1:
                    pts.add((a, b, c))
    m = n // 2
    for t in range(n):
        pts.update({(t, m, m), (m, t, m), (m, m, t)})
    rng = np.random.default_rng(seed)
    for _ in range(600):
        pts.add(tuple(int(v) for v in rng.integers(0, n, 3)))
    return sorted(pts)


@pytest.mark.parametrize("storage", ["f32", "f16", "f16_i16"])
def test_sampled_step_at_256cube(storage):
    print(f"case: full size 256^3 T1 Ra1e6 {storage}, sampled one-step parity", flush=True)
    cav = L.Cavity(n=N, wall_type=1, ra=1e6, storage=storage,
                   theta0=inputs.theta_noise(N, 20151115))
    assert cav.get_launch() == (256, 1)  # the shape bench.py times
    cav.step(2000)
    f0, g0 = cav.get_populations()
    cav.step(1)
    f1, g1 = cav.get_populations()
    nu_gpu = cav.nusselt(with_map=True)
    cav.close()
    assert np.abs(f1 - W19[:, None]).max() > 1e-4  # the flow has developed

    ora = O.Oracle(N, 1, ra=1e6, state=False)
    worst_f = worst_g = 0.0
    for (x, y, z) in sample_nodes(N):
        c = x + N * (y + N * z)
        fo, go = ora.step_node(f0, g0, x, y, z)
        df = np.abs(f1[:, c] - fo)
        dg = np.abs(g1[:, c] - go)
        if storage == "f32":
            # FP32 offsets f - w (|f - w| < 1e-2: ulp < 1e-9) and g (up to
            # w_T theta_h = 1/16: ulp 7.5e-9): a few ulps of arithmetic and
            # storage rounding (observed 5e-11 and 1.0e-8)
            tol_f, tol_g = 2e-8, 4e-8
        else:
            # one FP16 ulp of the stored (f - w)/w and g/w_T: the FP32 result
            # may sit on the other side of a rounding boundary from the FP64
            # one (observed: half an ulp of g)
            vf, vg = np.abs(fo / W19 - 1), np.abs(go / W7)
            tol_f = W19 * (2.0 ** -10 * vf + 2.0 ** -24) + 1e-8
            tol_g = W7 * (2.0 ** -10 * vg + 2.0 ** -24) + 1e-8
            if storage == "f16_i16":
                # stochastic rounding to the fixed-point grid: within one
                # spacing 2^-14 of g/w_T
                tol_g = W7 * 2.0 ** -14 + 1e-8
        assert np.all(df <= tol_f), ((x, y, z), df.max())
        assert np.all(dg <= tol_g), ((x, y, z), dg.max())
        worst_f, worst_g = max(worst_f, df.max()), max(worst_g, dg.max())
    print({"storage": storage, "max |df|": worst_f, "max |dg|": worst_g})

    nu_ora = ora.nusselt_of(g1, with_map=True)
    for k in ("nu3d", "nu2d", "numax"):
        assert abs(nu_gpu[k] - nu_ora[k]) <= 1e-12 * abs(nu_ora[k]), (k, nu_gpu[k], nu_ora[k])
    assert np.abs(nu_gpu["map"] - nu_ora["map"]).max() <= 1e-11 * np.abs(nu_ora["map"]).max()

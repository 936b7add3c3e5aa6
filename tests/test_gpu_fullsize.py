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


# Stored mantissa bits of the flow and energy populations per storage format
# (None: FP32 / FP64 storage; "fix": 16-bit fixed point in units of 2^-15 of
# g / w_T (Theta = 1 for the walls at +-1/2)).
FLOW_BITS = {"f64": None, "f32": None, "f16": 10, "bf16": 7, "f16_f32": 10, "bf16_f32": 7,
             "f16_i16": 10}
ENERGY_BITS = {"f64": None, "f32": None, "f16": 10, "bf16": 7, "f16_f32": None,
               "bf16_f32": None, "f16_i16": "fix"}


def tolerance(bits, w, ref, fp_tol):
    """Bound on |GPU - oracle| for one population after one step from the
    same state.  FP32 / FP64 storage: fp_tol (a few ulps of arithmetic and
    storage rounding).  16-bit floating point: one ulp of the stored value
    ref / w - 1 (or ref / w), since the FP32 result may sit on the other side
    of a rounding boundary from the FP64 one, plus FP32 arithmetic.  Fixed
    point with stochastic rounding: one spacing 2^-15 of g / w_T."""
    if bits is None:
        return fp_tol
    if bits == "fix":
        return w * 2.0 ** -15 + 1e-8
    return w * (2.0 ** -bits * np.abs(ref) + 2.0 ** -24) + 1e-8


@pytest.mark.parametrize("storage", ["f32", "f16", "f16_i16", "bf16", "f16_f32", "bf16_f32", "f64"])
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

    # FP32: offsets f - w (|f - w| < 1e-2: ulp < 1e-9) and g (up to
    # w_T theta_h = 1/16: ulp 7.5e-9), a few ulps (observed 5e-11 and 1.0e-8);
    # FP64: a few ulps of values below 1
    fp_f, fp_g = (1e-14, 1e-14) if storage == "f64" else (2e-8, 4e-8)
    ora = O.Oracle(N, 1, ra=1e6, state=False)
    worst_f = worst_g = 0.0
    for (x, y, z) in sample_nodes(N):
        c = x + N * (y + N * z)
        fo, go = ora.step_node(f0, g0, x, y, z)
        df = np.abs(f1[:, c] - fo)
        dg = np.abs(g1[:, c] - go)
        tol_f = tolerance(FLOW_BITS[storage], W19, fo / W19 - 1, fp_f)
        tol_g = tolerance(ENERGY_BITS[storage], W7, go / W7, fp_g)
        assert np.all(df <= tol_f), ((x, y, z), df.max())
        assert np.all(dg <= tol_g), ((x, y, z), dg.max())
        worst_f, worst_g = max(worst_f, df.max()), max(worst_g, dg.max())
    print({"storage": storage, "max |df|": worst_f, "max |dg|": worst_g})

    nu_ora = ora.nusselt_of(g1, with_map=True)
    for k in ("nu3d", "nu2d", "numax"):
        assert abs(nu_gpu[k] - nu_ora[k]) <= 1e-12 * abs(nu_ora[k]), (k, nu_gpu[k], nu_ora[k])
    assert np.abs(nu_gpu["map"] - nu_ora["map"]).max() <= 1e-11 * np.abs(nu_ora["map"]).max()

"""Initial states built from fields on the GPU against the FP64 oracle.

lbmx_init_fields (fields of a caller or the network, FP32) and
lbmx_init_from_cavity (the fields of another cavity, FP64 on the device)
sample trilinearly onto the cavity's nodes and set f = f^eq(1, u) (Eq. 17),
g = N^-1 n^eq(theta, u) (Eq. 33).  The oracle builds the same state from the
same seeded inputs (oracle.resample, oracle.equilibrium_state); for
init_from_cavity it also steps its own copy of the source cavity.  The paper
fixes no initial state (it is a warm start); what is checked is that the
state the GPU writes is the one defined above.  Grid sequencing, the use of
init_from_cavity, is checked for its gain at the end."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1511_04633_amd import inputs
from paper_1511_04633_amd import lbmx as L

pytestmark = pytest.mark.gpu

SEED = 20151115


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()
    O.build(force=False)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("m,n", [(6, 9), (8, 8), (11, 5)])
def test_init_fields_is_the_equilibrium_of_the_sampled_fields(storage, m, n):
    print(f"case: init_fields {m}^3 -> {n}^3 {storage}", flush=True)
    fld = inputs.random_fields(m, SEED + m)
    cav = L.Cavity(n=n, wall_type=2, ra=1e3, storage=storage)
    d = dev(fld)
    cav.init_fields(d[0], d[1], d[2], d[3])
    assert cav.t == 0
    f, g = cav.get_populations()
    cav.close()
    fe, ge = O.equilibrium_state(*[O.resample(a.astype(np.float64), n) for a in fld])
    if storage == "f64" and m == n:
        tol_f = tol_g = 1e-15  # identical grids: weights 1 and 0, exact samples
    else:
        # The GPU samples FP32 fields in FP32: each sample position carries a
        # few roundings of (x + 1/2) m / n (<= 4 ulp of m per axis) and the
        # field may jump by 2 amp between neighbouring nodes, so a sample is
        # within 3 * 4 * 2^-24 m * 2 amp (+ 8 ulp of amp for the lerps); f and
        # g change by at most 1.2 and 0.3 times that (w_i <= 1/3, |u| < 0.1).
        eps = 2.0 ** -24

        def sample_bound(amp):
            return 3 * 4 * eps * max(m, n) * 2 * amp + 8 * eps * amp

        tol_f = 1.2 * sample_bound(0.03) + 2e-9    # + FP32 storage of f - w
        tol_g = 0.3 * sample_bound(0.5) + 4e-8      # + FP32 storage of g
    assert np.abs(f - fe).max() <= tol_f, np.abs(f - fe).max()
    assert np.abs(g - ge).max() <= tol_g, np.abs(g - ge).max()
    print({"max |df|": np.abs(f - fe).max(), "max |dg|": np.abs(g - ge).max()})


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("m,n,ma,force_model", [(8, 12, 0.1, 0), (10, 7, 0.05, 0), (9, 13, 0.1, 2)])
def test_init_from_cavity(storage, m, n, ma, force_model):
    """A developed source cavity (20 steps from random fields, FP64 storage)
    initialises a cavity of another size, and with another Ma (velocities
    scaled by s = u_c(dst) / u_c(src), Eq. 38, density variations by s^2).
    Under Guo's forcing the transferred velocity is the half-force one."""
    print(f"case: init_from_cavity {m}^3 -> {n}^3 Ma {ma} force {force_model} {storage}",
          flush=True)
    fld = inputs.random_fields(m, SEED + 7 * m)
    src = L.Cavity(n=m, wall_type=2, ra=1e3, storage="f64", force_model=force_model)
    d = dev(fld)
    src.init_fields(d[0], d[1], d[2], d[3])
    src.step(20)
    before = src.get_populations()
    dst = L.Cavity(n=n, wall_type=2, ra=1e3, ma=ma, storage=storage, force_model=force_model)
    dst.step(3)
    dst.init_from(src)
    assert dst.t == 0
    f, g = dst.get_populations()
    after = src.get_populations()
    assert all(np.array_equal(a, b) for a, b in zip(before, after))  # src only read
    with pytest.raises(L.LbmxError):
        src.init_from(src)
    src.close()
    dst.close()

    ora = O.Oracle(m, 2, ra=1e3, force_model=force_model)
    ora.set_state(*O.equilibrium_state(*fld.astype(np.float64)))
    ora.step(20)
    rho, ux, uy, uz, th = ora.macro()
    scale = O.derive(n, 1e3, ma=ma)["u_c"] / O.derive(m, 1e3)["u_c"]
    r = [O.resample(a, n) for a in (ux, uy, uz, th, rho)]
    fe, ge = O.equilibrium_state(r[0] * scale, r[1] * scale, r[2] * scale, r[3],
                                 rho=1 + scale ** 2 * (r[4] - 1))
    # FP64: 20 steps of GPU-vs-oracle rounding.  FP32: storage rounding of the
    # offsets f - w (|f - w| < 0.02, ulp < 2e-9) and of g; at wall-adjacent
    # nodes the stored energy value is 2 w theta_W - g (|.| < 0.4, ulp 3e-8)
    # and pulling it back rounds once more, so one ulp of 0.4.
    tol_f, tol_g = (1e-12, 1e-12) if storage == "f64" else (1e-8, 3e-8)
    assert np.abs(f - fe).max() <= tol_f, np.abs(f - fe).max()
    assert np.abs(g - ge).max() <= tol_g, np.abs(g - ge).max()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_init_from_two_cavities(storage):
    """lbmx_init_from_cavities: the state is the equilibrium of wa (fields
    of a) + wb (fields of b), each source's rho, u, theta resampled onto the
    destination's nodes, its velocity scaled by s = u_c(dst) / u_c(src)
    (Eq. 38; dst at another Ma) and its density variation by s^2, against
    the oracle's sources, resampling and equilibrium; the sources are only
    read, identical handles are rejected."""
    print(f"case: init_from_cavities 6^3 + 9^3 -> 12^3 {storage}", flush=True)
    wa, wb, n, ma = 1.25, -0.25, 12, 0.08
    srcs, oras = [], []
    for m in (6, 9):
        fld = inputs.random_fields(m, SEED + 11 * m)
        c = L.Cavity(n=m, wall_type=3, ra=1e3, storage="f64")
        d = dev(fld)
        c.init_fields(d[0], d[1], d[2], d[3])
        c.step(20)
        srcs.append(c)
        ora = O.Oracle(m, 3, ra=1e3)
        ora.set_state(*O.equilibrium_state(*fld.astype(np.float64)))
        ora.step(20)
        oras.append(ora)
    before = [c.get_populations() for c in srcs]
    dst = L.Cavity(n=n, wall_type=3, ra=1e3, ma=ma, storage=storage)
    dst.step(2)
    dst.init_from_two(srcs[0], wa, srcs[1], wb)
    assert dst.t == 0
    f, g = dst.get_populations()
    for c, b in zip(srcs, before):
        assert all(np.array_equal(x, y) for x, y in zip(b, c.get_populations()))  # only read
    for args in ((srcs[0], wa, srcs[0], wb), (dst, wa, srcs[1], wb)):
        with pytest.raises(L.LbmxError):
            dst.init_from_two(*args)
    with pytest.raises(L.LbmxError):
        dst.init_from_two(srcs[0], float("nan"), srcs[1], wb)
    for c in srcs:
        c.close()
    dst.close()

    fields = np.zeros((4, n, n, n))
    drho = np.zeros((n, n, n))
    for ora, w, m in zip(oras, (wa, wb), (6, 9)):
        rho, ux, uy, uz, th = ora.macro()
        s = O.derive(n, 1e3, ma=ma)["u_c"] / O.derive(m, 1e3)["u_c"]
        fields += w * np.stack([O.resample(ux, n) * s, O.resample(uy, n) * s,
                                O.resample(uz, n) * s, O.resample(th, n)])
        drho += w * s ** 2 * (O.resample(rho, n) - 1)
    fe, ge = O.equilibrium_state(*fields, rho=1 + drho)
    # tolerances as for lbmx_init_from_cavity (FP32: one storage rounding of
    # the offsets and of the wall-adjacent energy values)
    tol_f, tol_g = (1e-12, 1e-12) if storage == "f64" else (1e-8, 3e-8)
    assert np.abs(f - fe).max() <= tol_f, np.abs(f - fe).max()
    assert np.abs(g - ge).max() <= tol_g, np.abs(g - ge).max()


def test_init_from_cavity_across_storage_formats():
    """A 16-bit source feeds an FP32 cavity: the FP32 cavity's fields are
    the source's fields (same grid) within the 16-bit format's resolution."""
    print("case: init_from_cavity f16_i16 -> f32 same grid", flush=True)
    n = 12
    src = L.Cavity(n=n, wall_type=1, ra=1e5, storage="f16_i16", theta0=inputs.theta_noise(n, SEED))
    src.step(300)
    dst = L.Cavity(n=n, wall_type=1, ra=1e5, storage="f32")
    dst.init_from(src)
    a, b = src.read_macro(), dst.read_macro()
    for k in (0, 1, 2, 3, 4):                                       # rho, u, v, w, theta
        assert np.abs(a[k] - b[k]).max() <= 1e-6 * max(1.0, np.abs(a[k]).max()), k
    src.close()
    dst.close()


@pytest.mark.parametrize("wall_type", [1, 3])
def test_grid_sequencing_reaches_the_same_steady_state_sooner(wall_type):
    """A 48^3 cavity run to steady, resampled onto 96^3, reaches the 96^3
    rest start's steady Nu (same criterion, |dNu| < 1e-6 per 1000 steps) in
    fewer fine steps and less wall time, coarse solve included.  (Below
    ~64^3 a step costs about one kernel launch, 4-12 us, whatever the size,
    so the coarse level saves steps but not time there.)"""
    from paper_1511_04633_amd import warmstart
    print(f"case: grid sequencing 48^3 -> 96^3 Ra 1e5 type {wall_type}", flush=True)
    rest = warmstart.solve(96, 1e5, wall_type, None)
    seq = warmstart.solve(96, 1e5, wall_type, None, coarse=48)
    print(rest, seq)
    assert rest["converged"] and seq["converged"] and seq["coarse"]["converged"]
    assert abs(seq["nu3d"] - rest["nu3d"]) <= 1e-3 * rest["nu3d"]
    assert seq["steps"] < 0.7 * rest["steps"] and seq["seconds"] < rest["seconds"]


@pytest.mark.parametrize("wall_type", [2, 3])
def test_extrapolated_start_reaches_the_same_steady_state_sooner(wall_type):
    """24^3 run to steady starts 48^3, also run to steady; the 96^3 cavity
    starts from 5/4 of the 48^3 fields minus 1/4 of the 24^3 fields
    (lbmx_init_from_cavities) and reaches the plain grid-sequenced start's
    steady Nu in fewer fine steps (measured 37k vs 43k and 20k vs 42k for
    types 2 and 3) and less wall time, both coarse solves included."""
    from paper_1511_04633_amd import warmstart
    print(f"case: extrapolated start 24^3, 48^3 -> 96^3 Ra 1e5 type {wall_type}", flush=True)
    seq = warmstart.solve(96, 1e5, wall_type, None, coarse=48)
    ex = warmstart.solve(96, 1e5, wall_type, None, coarse=48, extrapolate=True)
    print(seq, ex)
    assert seq["converged"] and ex["converged"] and ex["coarse"]["converged"]
    assert ex["coarse"]["quarter"]["converged"] and ex["coarse"]["quarter"]["n"] == 24
    assert abs(ex["nu3d"] - seq["nu3d"]) <= 1e-4 * seq["nu3d"]
    assert ex["steps"] < 0.9 * seq["steps"] and ex["seconds"] < seq["seconds"]


def test_batch_init_from_matches_single_cavities():
    """lbmx_batch_init_from gives bit for bit the state lbmx_init_from_cavity
    gives for the same cavities run alone, and the batch steps on in lockstep
    from it."""
    print("case: batch init_from vs single init_from_cavity", flush=True)
    src_cases = [dict(n=8, wall_type=2, ra=1e4), dict(n=6, wall_type=3, ra=3e4)]
    dst_cases = [dict(n=12, wall_type=2, ra=1e4), dict(n=11, wall_type=3, ra=3e4)]
    sb, db = L.Batch(src_cases, storage="f32"), L.Batch(dst_cases, storage="f32")
    for k, c in enumerate(src_cases):
        sb.init_rest(k, inputs.theta_noise(c["n"], SEED + k))
    sb.step(50)
    db.step(3)  # the destination's parity and time are reset by init_from
    for k in range(2):
        db.init_from(k, sb, k)
    singles = []
    for k, (sc, dc) in enumerate(zip(src_cases, dst_cases)):
        s = L.Cavity(storage="f32", theta0=inputs.theta_noise(sc["n"], SEED + k), **sc)
        s.step(50)
        d = L.Cavity(storage="f32", **dc)
        d.init_from(s)
        s.close()
        singles.append(d)
    for rounds in (0, 20):
        if rounds:
            db.step(rounds)
            for d in singles:
                d.step(rounds)
        for k, d in enumerate(singles):
            for a, b_ in zip(db.read_macro(k), d.read_macro()):
                assert np.array_equal(np.asarray(a).reshape(-1), np.asarray(b_).reshape(-1)), (k, rounds)
    with pytest.raises(L.LbmxError):
        db.init_from(0, db, 0)
    for d in singles:
        d.close()
    sb.close()
    db.close()


def test_batch_grid_sequencing_reaches_the_same_steady_state():
    """Two cavities (64^3 Type 1, 48^3 Type 3, Ra 1e5) run to steady by the
    batch from rest, and from a half-size batch run to steady first: the same
    steady Nu (within 1e-3) in fewer fine steps."""
    print("case: batch grid sequencing 32/24 -> 64/48", flush=True)
    cases = [dict(n=64, wall_type=1, ra=1e5), dict(n=48, wall_type=3, ra=1e5)]
    rest = L.Batch(cases, storage="f32")
    for k, c in enumerate(cases):
        rest.init_rest(k, inputs.theta_noise(c["n"], SEED))
    rest.run_to_steady(tol=1e-6, every=1000, max_steps=400_000)
    coarse = L.Batch([dict(c, n=c["n"] // 2) for c in cases], storage="f32")
    for k, c in enumerate(cases):
        coarse.init_rest(k, inputs.theta_noise(c["n"] // 2, SEED))
    coarse.run_to_steady(tol=1e-6, every=1000, max_steps=400_000)
    fine = L.Batch(cases, storage="f32")
    for k in range(len(cases)):
        fine.init_from(k, coarse, k)
    fine.run_to_steady(tol=1e-6, every=1000, max_steps=400_000)
    for k in range(len(cases)):
        r, f = rest.info(k), fine.info(k)
        print(k, r, f, coarse.info(k))
        assert r["state"] == "converged" and f["state"] == "converged"
        assert abs(f["nu3d"] - r["nu3d"]) <= 1e-3 * r["nu3d"]
        assert f["t"] < r["t"]
    for b in (rest, coarse, fine):
        b.close()

"""Pins of the oracle's variants: the two other force models, the general
(anisotropic) diffusion block of Eqs. (35)-(36), and the three Nu stencils.

Each test checks a property fixed by the definition of the variant or by the
mathematics: moment identities of Guo's forcing term, the exact momentum
gain of a uniformly heated periodic box, the textbook BGK form of Guo's
scheme, exact rest and conduction states, and the decay rates k^T D k of
temperature sine modes.  CPU only.
"""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _he_luo_feq(rho, j, e, w):
    """w_i [rho + 3 e.j + 4.5 (e.j)^2 - 1.5 j.j] (the equilibrium of Eq. 24, rho_0 = 1)."""
    ej = e @ j
    return w * (rho + 3 * ej + 4.5 * ej ** 2 - 1.5 * (j @ j))


# ------------------------------------------------------------ force models

def test_guo_force_moments():
    """Guo's term carries no mass, momentum source rho G and second moment
    rho (V G + G V), for any density and velocity."""
    e, w, _, _ = O.velocities()
    rng = np.random.default_rng(11)
    for _ in range(20):
        rho = 1 + 0.05 * rng.standard_normal()
        v = 0.05 * rng.standard_normal(3)
        gz = 1e-3 * rng.standard_normal()
        fb = O.guo_force(rho, v, gz)
        G = np.array([0.0, 0.0, gz])
        assert abs(fb.sum()) < 1e-18
        assert np.abs(e.T @ fb - rho * G).max() < 1e-18
        second = np.einsum("ia,ib,i->ab", e, e, fb)
        assert np.abs(second - rho * (np.outer(v, G) + np.outer(G, v))).max() < 1e-18


@pytest.mark.parametrize("model", [0, 1, 2])
def test_uniform_acceleration(model):
    """A periodic box at uniform density rho_0 and temperature theta_0 stays
    uniform and gains momentum G per step times the force density's factor:
    rho_0 (Eq. 15, reading R3; Guo) or 1 (the literal division by rho).  The
    reported velocity is j / rho, or (j + rho G / 2) / rho for Guo's scheme."""
    n, rho0, th0, steps = 4, 1.03, 0.3, 25
    _, w, _, w7 = O.velocities()
    o = O.Oracle(n, 0, ra=1e4, force_model=model)
    G = o.derived()["gbeta"] * th0
    o.set_state(np.repeat((w * rho0)[:, None], n ** 3, 1), np.repeat((w7 * th0)[:, None], n ** 3, 1))
    o.step(steps)
    rho, ux, uy, uz, th = o.macro()
    assert np.abs(rho - rho0).max() < 1e-14 and np.abs(th - th0).max() < 1e-15
    assert np.abs(ux).max() < 1e-17 and np.abs(uy).max() < 1e-17
    j = {0: rho0 * G * steps, 1: G * steps, 2: rho0 * G * steps}[model]
    v = {0: j / rho0, 1: j / rho0, 2: (j + 0.5 * rho0 * G) / rho0}[model]
    assert np.abs(uz - v).max() < 1e-14 * abs(v), (model, uz.flat[0], v)


def test_guo_bgk_special_case():
    """With every s_k = 1/tau, Guo's scheme in moment space is the textbook
    BGK form: f* = f - (f - f^eq(rho, rho V)) / tau + (1 - 1/(2 tau)) Fbar_i,
    V = (j + rho G / 2) / rho, Fbar_i = w_i rho [3 (e_i - V) + 9 (e_i.V) e_i].G."""
    e, w, e7, w7 = O.velocities()
    rng = np.random.default_rng(12)
    for tau, tau_g in ((0.8, 0.7), (0.56, 1.2)):
        o = O.Oracle(8, 1, ra=1e4, s19=np.full(19, 1 / tau), tau7=np.full(7, tau_g), force_model=2)
        gb = o.derived()["gbeta"]
        for _ in range(10):
            rho = 1 + 0.01 * rng.standard_normal()
            j0 = 0.03 * rng.standard_normal(3)
            f = _he_luo_feq(rho, j0, e, w) + 1e-3 * w * rng.standard_normal(19)
            g = w7 * (0.3 + 0.01 * rng.standard_normal(7))
            fo, go = o.collide_node(f, g)
            rho, j, th = f.sum(), e.T @ f, g.sum()
            G = np.array([0.0, 0.0, gb * th])
            v = (j + 0.5 * rho * G) / rho
            fbar = w * rho * ((e - v) @ G * 3 + 9 * (e @ v) * (e @ G))
            want = f - (f - _he_luo_feq(rho, rho * v, e, w)) / tau + (1 - 0.5 / tau) * fbar
            assert np.abs(fo - want).max() < 1e-15
            geq = w7 * th * (1 + 4 * (e7 @ v))
            assert np.abs(go - (g - (g - geq) / tau_g)).max() < 1e-15


@pytest.mark.parametrize("model", [1, 2])
def test_force_models_keep_rest_state(model):
    """theta = theta_ref everywhere: no force under any model, exact rest."""
    o = O.Oracle(7, 2, ra=1e4, theta_hot=0.0, theta_cold=0.0, force_model=model)
    o.step(120)
    _, ux, uy, uz, th = o.macro()
    assert np.abs(np.stack([ux, uy, uz])).max() == 0.0 and np.abs(th).max() == 0.0


def test_force_models_differ_as_defined():
    """One collision: model 1 adds F_i / rho where model 0 adds F_i; model 2
    changes momentum by the same rho G as model 0 but relaxes towards j + rho G/2."""
    e, w, _, w7 = O.velocities()
    rng = np.random.default_rng(13)
    o = [O.Oracle(8, 1, ra=1e5, force_model=m) for m in range(3)]
    gb = o[0].derived()["gbeta"]
    for _ in range(5):
        rho = 1 + 0.02 * rng.standard_normal()
        f = _he_luo_feq(rho, 0.02 * rng.standard_normal(3), e, w)
        g = w7 * 0.4
        out = [x.collide_node(f, g)[0] for x in o]
        F = O.force(rho, (e.T @ f) / rho, gb * 0.4)
        # populations are O(0.3): one rounding is ~3e-17
        assert np.abs((out[1] - out[0]) - F * (1 / rho - 1)).max() < 2e-16
        for m in (0, 2):
            assert abs((e.T @ (out[m] - f))[2] - rho * gb * 0.4) < 2e-16
        assert np.abs(out[2] - out[0]).max() > 1e-9  # a different scheme


# -------------------------------------------------------------- Nu stencils

@pytest.mark.parametrize("wall_type", [1, 2, 3])
def test_conduction_limit_every_stencil(wall_type):
    """Without buoyancy the steady state conducts heat at Nu = 1 exactly: the
    linear profile makes every difference stencil exact, and the energy that
    crosses the hot wall's links equals D_yy / H (stencil 2)."""
    o = O.Oracle(8, wall_type, ra=100.0, buoyancy_scale=0.0)
    o.step(6000)
    for st in (0, 1, 2):
        nu = o.nusselt(with_map=True, stencil=st)
        assert np.abs(nu["map"] - 1).max() < 1e-11, st


def test_flux_stencil_uses_d_yy():
    """With a diagonal anisotropic D the conduction profile is still linear in
    y and Nu = 1 on every stencil; the wall-flux stencil divides by D_yy, not
    by alpha (A_yy = 0.6 here)."""
    o = O.Oracle(8, 2, ra=100.0, buoyancy_scale=0.0, aniso=[1.5, 0.6, 1.2, 0, 0, 0])
    o.step(10000)
    th = o.macro()[4]
    lin = 0.5 - (np.arange(8) + 0.5) / 8
    assert np.abs(th - lin[None, :, None]).max() < 1e-12
    for st in (0, 1, 2):
        assert abs(o.nusselt(stencil=st)["nu3d"] - 1) < 1e-11, st


def test_stencils_on_manufactured_states():
    """theta = theta_h + a Yw + b Yw^2 with Yw = (j + 1/2)/n the distance from
    the hot wall, fluid at rest, g = w_T theta: stencil 0 returns -a exactly
    (exact for quadratics), stencil 1 returns -(a + b/(2n)) (first order: the
    curvature term of a one-point difference), stencil 2 returns the flux
    carried by the equilibrium populations, n (theta_0 - theta_h) / (4 D_yy)."""
    n = 7
    _, _, _, w7 = O.velocities()
    for aniso in (None, [1.0, 0.5, 2.0, 0.1, -0.2, 0.15]):
        o = O.Oracle(n, 1, ra=1e4, aniso=aniso)
        alpha = o.derived()["alpha"]
        d_yy = alpha * (1.0 if aniso is None else aniso[1])
        a, b = -1.3, 0.8
        Yw = (np.arange(n) + 0.5) / n
        th = 0.5 + a * Yw + b * Yw ** 2
        g = w7[:, None] * np.broadcast_to(th[None, :, None], (n, n, n)).reshape(1, -1)
        f, _ = o.get_state()
        o.set_state(f, g)
        assert abs(o.nusselt(stencil=0)["nu3d"] + a) < 1e-12
        assert abs(o.nusselt(stencil=1)["nu3d"] + (a + b / (2 * n))) < 1e-12
        want = n * (th[0] - 0.5) / (4 * d_yy)
        assert abs(o.nusselt(stencil=2)["nu3d"] - want) < 1e-12 * abs(want)


# ------------------------------------------------------ anisotropic diffusion

def test_identity_tensor_is_the_isotropic_model():
    """A = I reproduces the isotropic run bit for bit (Eq. 36 with D = alpha I)."""
    th0 = np.random.default_rng(14).uniform(-1e-3, 1e-3, 8 ** 3)
    a = O.Oracle(8, 2, ra=1e4, theta0=th0)
    b = O.Oracle(8, 2, ra=1e4, theta0=th0, aniso=[1, 1, 1, 0, 0, 0])
    a.step(60)
    b.step(60)
    fa, ga = a.get_state()
    fb, gb = b.get_state()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


A_TENSOR = [1.0, 0.6, 0.8, 0.3, 0.2, -0.25]  # xx, yy, zz, xy, xz, yz (positive definite)


def _aniso_decay_ratio(n, kvec, t0=100, t1=900):
    """Decay rate of theta = 0.1 sin(2 pi k.x / n) in a periodic box at rest,
    divided by alpha k^T A k (2 pi / n)^2."""
    x = np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    phase = 2 * np.pi * (kvec[0] * X + kvec[1] * Y + kvec[2] * Z) / n
    mode = np.sin(phase)
    o = O.Oracle(n, 0, ra=1e3, buoyancy_scale=0.0, aniso=A_TENSOR, theta0=(0.1 * mode).reshape(-1))
    alpha = o.derived()["alpha"]
    A = np.array([[A_TENSOR[0], A_TENSOR[3], A_TENSOR[4]],
                  [A_TENSOR[3], A_TENSOR[1], A_TENSOR[5]],
                  [A_TENSOR[4], A_TENSOR[5], A_TENSOR[2]]])
    k = np.array(kvec, dtype=float)
    rate = alpha * (k @ A @ k) * (2 * np.pi / n) ** 2
    amp = lambda: 2 * np.mean(o.macro()[4] * mode)
    o.step(t0)
    a0 = amp()
    o.step(t1 - t0)
    a1 = amp()
    return -np.log(a1 / a0) / (t1 - t0) / rate


@pytest.mark.parametrize("kvec", [(1, 0, 0), (1, 1, 0), (1, -1, 0), (1, 0, 1), (0, 1, -1), (0, 1, 1)])
def test_anisotropic_mode_decay(kvec):
    """Eq. (27) with constant D: a sine mode along k decays at k^T D k.  The
    pairs (1, 1, 0) / (1, -1, 0) and (0, 1, 1) / (0, 1, -1) separate the signs
    of the off-diagonal entries.  Wavelengths n and 2n are extrapolated
    (Richardson, second order) to remove the lattice O(k^2) term."""
    r1, r2 = _aniso_decay_ratio(16, kvec), _aniso_decay_ratio(32, kvec)
    assert abs(r2 - 1) < 1e-2, (kvec, r1, r2)
    assert abs((4 * r2 - r1) / 3 - 1) < 2.5e-3, (kvec, r1, r2)


# ---------------------------------------------------- single-node evaluation

@pytest.mark.parametrize("wall_type,force_model", [(0, 0), (1, 0), (2, 2), (3, 1)])
def test_step_node_is_oracle_step(wall_type, force_model):
    """The single-node step (streaming read from the destination) reproduces
    the whole-lattice step bit for bit at every node of a developed state, for
    periodic and walled boxes; the Nu of an external state equals nusselt()."""
    n = 7
    th0 = np.random.default_rng(15).uniform(-0.2, 0.2, n ** 3)
    o = O.Oracle(n, wall_type, ra=1e5, theta0=th0, force_model=force_model,
                 aniso=[1.0, 0.6, 0.8, 0.3, 0.2, -0.25])
    o.step(40)
    f0, g0 = o.get_state()
    o.step(1)
    f1, g1 = o.get_state()
    p = O.Oracle(n, wall_type, ra=1e5, force_model=force_model,
                 aniso=[1.0, 0.6, 0.8, 0.3, 0.2, -0.25], state=False)
    for z in range(n):
        for y in range(n):
            for x in range(n):
                c = x + n * (y + n * z)
                fo, go = p.step_node(f0, g0, x, y, z)
                assert np.array_equal(fo, f1[:, c]) and np.array_equal(go, g1[:, c]), (x, y, z)
    if wall_type:
        for st in (0, 1, 2):
            a, b = o.nusselt(with_map=True, stencil=st), p.nusselt_of(g1, stencil=st, with_map=True)
            assert np.array_equal(a["map"], b["map"]) and a["nu3d"] == b["nu3d"]
    with pytest.raises(RuntimeError):
        p.step(1)

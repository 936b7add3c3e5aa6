"""ctypes front end of the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library and its
Python binding never import this module.

The oracle holds the pre-collision state S_t of the double-MRT scheme
(Li, Yang & Zhang, Sec. 3): 19 D3Q19 populations f_i and 7 D3Q7 populations
g_i per node, stored population-major ``[i][cell]`` with
``cell = x + n*(y + n*z)``.  Directions follow the paper's order (Eqs. 12
and 28), shifted to 0-based indices.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC",
             "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_create_params.restype = ctypes.c_void_p
        L.oracle_create_params.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           _dp, _dp, _dp, ctypes.c_int]
        L.oracle_step_node.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _dp, _dp]
        L.oracle_nusselt_state.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, _dp, _dp]
        L.oracle_create.restype = ctypes.c_void_p
        L.oracle_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    _dp, _dp, _dp, ctypes.c_int, _dp]
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.oracle_time.restype = ctypes.c_long
        L.oracle_time.argtypes = [ctypes.c_void_p]
        L.oracle_macro.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.oracle_nusselt.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
        L.oracle_get_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.oracle_set_state.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_long]
        L.oracle_derive.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _dp]
        L.oracle_derived_of.argtypes = [ctypes.c_void_p, _dp]
        L.oracle_matrices.argtypes = [_dp, _dp, _dp, _dp]
        L.oracle_velocities.argtypes = [_ip, _dp, _ip, _dp]
        L.oracle_meq.argtypes = [ctypes.c_double] * 4 + [_dp]
        L.oracle_feq.argtypes = [ctypes.c_double, _dp, _dp]
        L.oracle_geq.argtypes = [ctypes.c_double, _dp, _dp]
        L.oracle_force.argtypes = [ctypes.c_double, _dp, ctypes.c_double, _dp]
        L.oracle_guo_force.argtypes = [ctypes.c_double, _dp, ctypes.c_double, _dp]
        L.oracle_collide_node.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.oracle_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def derive(n: int, ra: float, pr: float = 0.71, ma: float = 0.1) -> dict:
    """Lattice-unit parameters of Sec. 4 (Eq. 38), Eq. (26) and Eq. (36)."""
    out = np.zeros(6)
    lib().oracle_derive(n, ra, pr, ma, _ptr(out))
    return dict(zip(["u_c", "gbeta", "nu", "alpha", "s_nu", "tau_t"], out.tolist()))


def matrices():
    """(M, M^-1, N, N^-1) as used by the oracle (Eqs. 21, 32; inverses by elimination)."""
    m, mi = np.zeros((19, 19)), np.zeros((19, 19))
    nn, ni = np.zeros((7, 7)), np.zeros((7, 7))
    lib().oracle_matrices(_ptr(m), _ptr(mi), _ptr(nn), _ptr(ni))
    return m, mi, nn, ni


def velocities():
    """(e19, w19, e7, w7) as typed into the oracle (Eqs. 12, 18, 28, 31)."""
    e19 = np.zeros((19, 3), dtype=np.int32)
    e7 = np.zeros((7, 3), dtype=np.int32)
    w19, w7 = np.zeros(19), np.zeros(7)
    lib().oracle_velocities(e19.ctypes.data_as(_ip), _ptr(w19), e7.ctypes.data_as(_ip), _ptr(w7))
    return e19.astype(np.int64), w19, e7.astype(np.int64), w7


def meq(rho, jx, jy, jz):
    out = np.zeros(19)
    lib().oracle_meq(rho, jx, jy, jz, _ptr(out))
    return out


def feq(rho, v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(19)
    lib().oracle_feq(rho, _ptr(v), _ptr(out))
    return out


def geq(theta, v):
    """Energy populations whose moments are n^eq of Eq. (33): N^-1 n^eq."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(7)
    lib().oracle_geq(theta, _ptr(v), _ptr(out))
    return out


def equilibrium_state(ux, uy, uz, theta, rho=None):
    """Pre-collision state with f = f^eq(rho, u) (Eq. 17; rho = 1 when not
    given) and g = N^-1 n^eq(theta, u) (Eq. 33) at every node: the state a
    warm start builds from fields (the paper fixes no initial state).
    Fields of n^3 values, x fastest; returns (f 19 x n^3, g 7 x n^3)."""
    fs = [np.asarray(a, dtype=np.float64).reshape(-1) for a in (ux, uy, uz, theta)]
    cells = fs[0].size
    r = np.ones(cells) if rho is None else np.asarray(rho, dtype=np.float64).reshape(-1)
    f, g = np.zeros((19, cells)), np.zeros((7, cells))
    for c in range(cells):
        v = np.array([fs[0][c], fs[1][c], fs[2][c]])
        f[:, c] = feq(r[c], v)
        g[:, c] = geq(fs[3][c], v)
    return f, g


def resample(a, m):
    """Trilinear resampling of a node-centred field of the unit cube (n^3,
    indexed [z, y, x]) onto its m^3 node centres.  Output node i sits at
    p = (i + 1/2) n / m - 1/2 in input node units, clamped to [0, n - 1]
    (outside the outermost node centres the field is taken constant); the
    weights are linear in each axis, applied along x, then y, then z.  Used
    to move fields between grids for warm starts; not part of the paper."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    p = np.clip((np.arange(m) + 0.5) * n / m - 0.5, 0.0, n - 1.0)
    k0 = np.minimum(np.floor(p).astype(np.int64), max(n - 2, 0))
    k1 = np.minimum(k0 + 1, n - 1)
    fr = p - k0
    out = a[:, :, k0] * (1 - fr) + a[:, :, k1] * fr
    out = out[:, k0, :] * (1 - fr)[None, :, None] + out[:, k1, :] * fr[None, :, None]
    return out[k0] * (1 - fr)[:, None, None] + out[k1] * fr[:, None, None]


def force(rho, v, gz):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(19)
    lib().oracle_force(rho, _ptr(v), gz, _ptr(out))
    return out


def guo_force(rho, v, gz):
    """Guo's forcing term Fbar_i (force model 2) for G = (0, 0, gz)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(19)
    lib().oracle_guo_force(rho, _ptr(v), gz, _ptr(out))
    return out


def threads() -> int:
    return int(lib().oracle_threads())


class Oracle:
    """One cavity simulated by the FP64 oracle.

    wall_type: 1, 2, 3 as in Sec. 2 (Eqs. 6-10); 0 = fully periodic box
    (oracle-only, used to measure transport coefficients).
    s19: optional diagonal of S (Eq. 23) replacing Eq. (26).
    tau7: optional diagonal of Q^-1 (Eq. 35) replacing the paper's choice.
    aniso: optional (A_xx, A_yy, A_zz, A_xy, A_xz, A_yz): diffusion tensor
    D = alpha A in the tau-bar block of Eq. (35) via Eq. (36).
    force_model: 0 (Eq. 15, reading R3), 1 (Eq. 15 divided by rho), 2 (Guo).
    theta0: initial temperature field (n^3, x fastest); the initial state is
    f_i = w_i, g_i = w_T,i * theta0.
    state: False builds the parameters only (no n^3 arrays): such an oracle
    serves step_node() and nusselt_of() on a state held by the caller.
    """

    def __init__(self, n, wall_type=1, ra=1e3, pr=0.71, ma=0.1, theta_hot=0.5,
                 theta_cold=-0.5, theta_ref=0.0, buoyancy_scale=1.0, s19=None,
                 tau7=None, aniso=None, force_model=0, theta0=None, state=True):
        self.n = int(n)
        self.cells = self.n ** 3
        s19 = None if s19 is None else np.ascontiguousarray(s19, dtype=np.float64)
        tau7 = None if tau7 is None else np.ascontiguousarray(tau7, dtype=np.float64)
        aniso = None if aniso is None else np.ascontiguousarray(aniso, dtype=np.float64)
        if theta0 is not None:
            theta0 = np.ascontiguousarray(theta0, dtype=np.float64).reshape(-1)
            assert theta0.size == self.cells
        self._keep = (s19, tau7, aniso, theta0)
        if state:
            h = lib().oracle_create(self.n, int(wall_type), ra, pr, ma, theta_hot, theta_cold,
                                    theta_ref, buoyancy_scale, _ptr(s19), _ptr(tau7), _ptr(aniso),
                                    int(force_model), _ptr(theta0))
        else:
            h = lib().oracle_create_params(self.n, int(wall_type), ra, pr, ma, theta_hot,
                                           theta_cold, theta_ref, buoyancy_scale, _ptr(s19),
                                           _ptr(tau7), _ptr(aniso), int(force_model))
        self.has_state = bool(state)
        if not h:
            raise ValueError("oracle_create rejected the parameters")
        self._h = ctypes.c_void_p(h)
        self.theta_hot = theta_hot

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return int(lib().oracle_time(self._h))

    def derived(self) -> dict:
        out = np.zeros(6)
        lib().oracle_derived_of(self._h, _ptr(out))
        return dict(zip(["u_c", "gbeta", "nu", "alpha", "s_nu", "tau_t"], out.tolist()))

    def _need_state(self):
        if not self.has_state:
            raise RuntimeError("this oracle holds parameters only (state=False)")

    def step(self, nsteps: int = 1):
        self._need_state()
        lib().oracle_step(self._h, int(nsteps))
        return self

    def step_node(self, f, g, x, y, z):
        """S_{t+1} at node (x, y, z) from a caller's state S_t (f: 19 x n^3,
        g: 7 x n^3 float64, population-major); returns (f19, g7)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.size == 19 * self.cells and g.size == 7 * self.cells
        fo, go = np.zeros(19), np.zeros(7)
        lib().oracle_step_node(self._h, _ptr(f), _ptr(g), int(x), int(y), int(z), _ptr(fo), _ptr(go))
        return fo, go

    def nusselt_of(self, g, stencil=0, with_map=False):
        """nusselt() of a caller's state g (7 x n^3 float64)."""
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert g.size == 7 * self.cells
        out = np.zeros(3)
        mp = np.zeros(self.n * self.n) if with_map else None
        lib().oracle_nusselt_state(self._h, _ptr(g), int(stencil), _ptr(out), _ptr(mp))
        d = {"nu3d": out[0], "nu2d": out[1], "numax": out[2]}
        if with_map:
            d["map"] = mp.reshape(self.n, self.n)
        return d

    def macro(self):
        """(rho, ux, uy, uz, theta), each shaped (n, n, n) indexed [z, y, x]."""
        self._need_state()
        arrs = [np.zeros(self.cells) for _ in range(5)]
        lib().oracle_macro(self._h, *[_ptr(a) for a in arrs])
        sh = (self.n,) * 3
        return tuple(a.reshape(sh) for a in arrs)

    def nusselt(self, with_map=False, stencil=0):
        """Hot-wall Nu family; stencil 0 (second order), 1 (first order),
        2 (energy flux of the wall links)."""
        self._need_state()
        out = np.zeros(3)
        mp = np.zeros(self.n * self.n) if with_map else None
        lib().oracle_nusselt(self._h, int(stencil), _ptr(out), _ptr(mp))
        d = {"nu3d": out[0], "nu2d": out[1], "numax": out[2]}
        if with_map:
            d["map"] = mp.reshape(self.n, self.n)  # [z, x]
        return d

    def get_state(self):
        self._need_state()
        f = np.zeros(19 * self.cells)
        g = np.zeros(7 * self.cells)
        lib().oracle_get_state(self._h, _ptr(f), _ptr(g))
        return f.reshape(19, self.cells), g.reshape(7, self.cells)

    def set_state(self, f, g, t=0):
        self._need_state()
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        assert f.size == 19 * self.cells and g.size == 7 * self.cells
        lib().oracle_set_state(self._h, _ptr(f), _ptr(g), int(t))

    def collide_node(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        fo, go = np.zeros(19), np.zeros(7)
        lib().oracle_collide_node(self._h, _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
        return fo, go

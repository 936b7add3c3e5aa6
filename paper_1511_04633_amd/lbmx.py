"""Python binding of the C-ABI in include/lbmx.h (argument marshalling only).

Every step of the method runs in the HIP library ``liblbmx.so``; this module
converts arguments, allocates the device workspace through PyTorch (device
memory and streams only) and raises on error status.  If the library is not
built the import of this module fails: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmx.so")

F64, F32, F16, BF16, F16_F32, BF16_F32, F16_I16 = 0, 1, 2, 3, 4, 5, 6
STORAGE = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "f16_f32": F16_F32,
           "bf16_f32": BF16_F32, "f16_i16": F16_I16}
STATUS = {0: "LBMX_OK", 1: "LBMX_EINVAL", 2: "LBMX_ENOMEM", 3: "LBMX_EDEVICE",
          4: "LBMX_EUNSTABLE", 5: "LBMX_ENOTCONVERGED", 6: "LBMX_ESTATE", 7: "LBMX_EIO"}

# Every symbol include/lbmx.h declares.
SYMBOLS = [
    "lbmx_params_default", "lbmx_derive", "lbmx_workspace_bytes", "lbmx_bytes_per_cell",
    "lbmx_create", "lbmx_destroy", "lbmx_init_rest", "lbmx_set_populations",
    "lbmx_get_populations", "lbmx_save", "lbmx_load", "lbmx_init_fields", "lbmx_init_from_cavity",
    "lbmx_init_from_cavities", "lbmx_step", "lbmx_step_timed", "lbmx_time",
    "lbmx_read_macro", "lbmx_nusselt", "lbmx_nusselt_noalloc", "lbmx_run_to_steady",
    "lbmx_set_launch",
    "lbmx_get_launch", "lbmx_strerror", "lbmx_last_error",
    "lbmx_batch_create", "lbmx_batch_destroy", "lbmx_batch_init_rest", "lbmx_batch_init_from",
    "lbmx_batch_step",
    "lbmx_batch_run_to_steady", "lbmx_batch_info", "lbmx_batch_nusselt",
    "lbmx_batch_read_macro", "lbmx_batch_resample", "lbmx_batch_set_launch",
    "lbmx_batch_get_launch", "lbmx_batch_autotune",
    "lbmx_nn_conv3d_fwd", "lbmx_nn_conv3d_flip", "lbmx_nn_conv3d_wgrad", "lbmx_nn_silu",
    "lbmx_nn_silu_bwd", "lbmx_nn_pool2", "lbmx_nn_up2", "lbmx_nn_concat", "lbmx_nn_mse",
    "lbmx_nn_adam", "lbmx_nn_to_bf16", "lbmx_nn_make_input", "lbmx_nn_add", "lbmx_nn_layout",
    "lbmx_nn_conv3d_fwd_ep", "lbmx_nn_upcat", "lbmx_nn_pool2_bwd_gate", "lbmx_nn_up2_bwd_gate",
    "lbmx_nn_conv3d_flip_many", "lbmx_nn_conv3d_fwd_upcat", "lbmx_nn_conv3d_wgrad_upcat",
    "lbmx_nn_conv3d_mse", "lbmx_nn_adam_flip", "lbmx_nn_layout_flip",
]
BATCH_STATE = {0: "active", 1: "converged", 2: "max_steps", 3: "diverged"}


class lbmx_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("wall_type", ctypes.c_int32),
        ("ra", ctypes.c_double), ("pr", ctypes.c_double), ("ma", ctypes.c_double),
        ("theta_hot", ctypes.c_double), ("theta_cold", ctypes.c_double),
        ("theta_ref", ctypes.c_double), ("buoyancy_scale", ctypes.c_double),
        ("storage", ctypes.c_int32), ("custom_rates", ctypes.c_int32),
        ("s", ctypes.c_double * 19), ("tau", ctypes.c_double * 7),
        ("force_model", ctypes.c_int32), ("nu_stencil", ctypes.c_int32),
        ("aniso", ctypes.c_double * 6),
    ]


# lbmx.h force models and Nu stencils, by name
FORCE_MODELS = {"eq15": 0, "eq15_rho": 1, "guo": 2}
NU_STENCILS = {"second_order": 0, "first_order": 1, "wall_flux": 2}


class lbmx_nu(ctypes.Structure):
    _fields_ = [("nu3d", ctypes.c_double), ("nu2d", ctypes.c_double),
                ("numax", ctypes.c_double), ("step", ctypes.c_int64),
                ("nonfinite", ctypes.c_int32)]


class LbmxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p
_lib = None


def load() -> ctypes.CDLL:
    """Load liblbmx.so (built in place by ``python -m paper_1511_04633_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run python -m paper_1511_04633_amd.build)")
    # PyTorch supplies the device memory and streams, so its HIP runtime must be
    # the one the library binds to: load it first (its libamdhip64 has the
    # library's soname), or the process would hold two runtimes.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(lbmx_params)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    sig = {
        "lbmx_params_default": [P],
        "lbmx_derive": [P, _dp],
        "lbmx_workspace_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "lbmx_bytes_per_cell": [i32, _dp],
        "lbmx_create": [P, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)],
        "lbmx_init_rest": [_vp, _dp],
        "lbmx_set_populations": [_vp, _dp, _dp, i64],
        "lbmx_get_populations": [_vp, _dp, _dp],
        "lbmx_save": [_vp, ctypes.c_char_p],
        "lbmx_load": [_vp, ctypes.c_char_p],
        "lbmx_init_fields": [_vp, _vp, _vp, _vp, _vp, i32],
        "lbmx_init_from_cavity": [_vp, _vp],
        "lbmx_init_from_cavities": [_vp, _vp, ctypes.c_double, _vp, ctypes.c_double],
        "lbmx_step": [_vp, i64],
        "lbmx_step_timed": [_vp, i64, _dp],
        "lbmx_time": [_vp, ctypes.POINTER(i64)],
        "lbmx_read_macro": [_vp, _dp, _dp, _dp, _dp, _dp],
        "lbmx_nusselt": [_vp, ctypes.POINTER(lbmx_nu), _dp],
        "lbmx_nusselt_noalloc": [_vp, ctypes.POINTER(lbmx_nu), _dp],
        "lbmx_run_to_steady": [_vp, ctypes.c_double, i64, i64, ctypes.POINTER(lbmx_nu)],
        "lbmx_set_launch": [_vp, i32, i32],
        "lbmx_get_launch": [_vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "lbmx_batch_create": [P, i32, _vp, ctypes.POINTER(_vp)],
        "lbmx_batch_init_rest": [_vp, i32, _dp],
        "lbmx_batch_init_from": [_vp, i32, _vp, i32],
        "lbmx_batch_step": [_vp, i64],
        "lbmx_batch_run_to_steady": [_vp, ctypes.c_double, i64, i64, ctypes.POINTER(i32)],
        "lbmx_batch_info": [_vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64),
                            ctypes.POINTER(lbmx_nu)],
        "lbmx_batch_nusselt": [_vp, i32, ctypes.POINTER(lbmx_nu)],
        "lbmx_batch_read_macro": [_vp, i32, _dp, _dp, _dp, _dp, _dp],
        "lbmx_batch_resample": [_vp, i32, i32, _fp],
        "lbmx_batch_set_launch": [_vp, i32, i32, i32],
        "lbmx_batch_get_launch": [_vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32)],
        "lbmx_batch_autotune": [_vp, ctypes.c_char_p, _dp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.lbmx_destroy.argtypes = [_vp]
    L.lbmx_destroy.restype = None
    L.lbmx_batch_destroy.argtypes = [_vp]
    L.lbmx_batch_destroy.restype = None
    L.lbmx_strerror.argtypes = [ctypes.c_int]
    L.lbmx_strerror.restype = ctypes.c_char_p
    L.lbmx_last_error.argtypes = []
    L.lbmx_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, ok=(0,)):
    if status not in ok:
        raise LbmxError(status, load().lbmx_last_error().decode())
    return status


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def make_params(n=16, wall_type=1, ra=1e3, pr=0.71, ma=0.1, theta_hot=0.5, theta_cold=-0.5,
                theta_ref=0.0, buoyancy_scale=1.0, storage="f32", s=None, tau=None,
                force_model=0, nu_stencil=0, aniso=None) -> lbmx_params:
    """force_model / nu_stencil: an int or a name of FORCE_MODELS / NU_STENCILS;
    aniso: (A_xx, A_yy, A_zz, A_xy, A_xz, A_yz) with D = alpha A, None = isotropic."""
    p = lbmx_params()
    _check(load().lbmx_params_default(ctypes.byref(p)))
    p.n, p.wall_type, p.ra, p.pr, p.ma = int(n), int(wall_type), ra, pr, ma
    p.theta_hot, p.theta_cold, p.theta_ref = theta_hot, theta_cold, theta_ref
    p.buoyancy_scale = buoyancy_scale
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.force_model = FORCE_MODELS[force_model] if isinstance(force_model, str) else int(force_model)
    p.nu_stencil = NU_STENCILS[nu_stencil] if isinstance(nu_stencil, str) else int(nu_stencil)
    if aniso is not None:
        p.aniso[:] = [float(v) for v in aniso]
    if s is not None or tau is not None:
        if s is None or tau is None:
            raise ValueError("custom rates need both s (19) and tau (7)")
        p.custom_rates = 1
        p.s[:] = [float(v) for v in s]
        p.tau[:] = [float(v) for v in tau]
    return p


def derive(p: lbmx_params) -> dict:
    out = (ctypes.c_double * 6)()
    _check(load().lbmx_derive(ctypes.byref(p), out))
    return dict(zip(["u_c", "gbeta", "nu", "alpha", "s_nu", "tau_t"], list(out)))


def workspace_bytes(p: lbmx_params) -> int:
    b = ctypes.c_size_t()
    _check(load().lbmx_workspace_bytes(ctypes.byref(p), ctypes.byref(b)))
    return int(b.value)


def bytes_per_cell(storage) -> float:
    b = ctypes.c_double()
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    _check(load().lbmx_bytes_per_cell(st, ctypes.byref(b)))
    return float(b.value)


class Cavity:
    """A cubic cavity advanced by the HIP library on the current torch device.

    The device workspace is a torch uint8 tensor owned by this object; all
    work goes to torch's current stream at construction time.  Fields come
    back as float64 arrays shaped (n, n, n) indexed [z, y, x].
    """

    def __init__(self, n=16, wall_type=1, ra=1e3, storage="f32", theta0=None, stream=None,
                 **kw):
        import torch

        L = load()
        self.params = make_params(n=n, wall_type=wall_type, ra=ra, storage=storage, **kw)
        self.n = int(n)
        self.cells = self.n ** 3
        self.ws = torch.empty(workspace_bytes(self.params), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _vp()
        _check(L.lbmx_create(ctypes.byref(self.params), _vp(self.ws.data_ptr()),
                             self.ws.numel(), _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        if theta0 is not None:
            self.init_rest(theta0)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lbmx_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---- state --------------------------------------------------------------
    def init_rest(self, theta0=None):
        th = None if theta0 is None else np.ascontiguousarray(theta0, dtype=np.float64).reshape(-1)
        if th is not None and th.size != self.cells:
            raise ValueError("theta0 needs n^3 values")
        _check(load().lbmx_init_rest(self._h, _dptr(th)))
        return self

    def init_fields(self, u, v, w, theta):
        """Fields are torch float32 CUDA tensors of shape (m, m, m) [z, y, x]."""
        ts = [t.contiguous() for t in (u, v, w, theta)]
        m = ts[0].shape[-1]
        for t in ts:
            if t.dtype.__repr__() != "torch.float32" or not t.is_cuda or t.numel() != m ** 3:
                raise ValueError("fields must be float32 CUDA tensors of m^3 values")
        self._keep_fields = ts
        _check(load().lbmx_init_fields(self._h, *[_vp(t.data_ptr()) for t in ts], int(m)))
        return self

    def init_from(self, other: "Cavity"):
        """State at t = 0 from another cavity's current fields, resampled
        onto this cavity's nodes on the device (``lbmx_init_from_cavity``)."""
        _check(load().lbmx_init_from_cavity(self._h, other._h))
        return self

    def init_from_two(self, a: "Cavity", wa: float, b: "Cavity", wb: float):
        """State at t = 0 from wa (fields of a) + wb (fields of b): rho, u
        and theta of each resampled onto this cavity's nodes on the device
        and combined (``lbmx_init_from_cavities``; wa = 5/4, wb = -1/4
        extrapolates the steady states at 1/2 and 1/4 of this resolution)."""
        _check(load().lbmx_init_from_cavities(self._h, a._h, float(wa), b._h, float(wb)))
        return self

    def set_populations(self, f, g, t=0):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        if f.size != 19 * self.cells or g.size != 7 * self.cells:
            raise ValueError("need 19 n^3 and 7 n^3 populations")
        _check(load().lbmx_set_populations(self._h, _dptr(f), _dptr(g), int(t)))
        return self

    def get_populations(self):
        f = np.empty(19 * self.cells)
        g = np.empty(7 * self.cells)
        _check(load().lbmx_get_populations(self._h, _dptr(f), _dptr(g)))
        return f.reshape(19, self.cells), g.reshape(7, self.cells)

    def save(self, path):
        """Write a checkpoint (parameters, t, current lattice) to `path`."""
        _check(load().lbmx_save(self._h, os.fsencode(path)))
        return self

    def load(self, path):
        """Restore a checkpoint written by save() for the same parameter set."""
        _check(load().lbmx_load(self._h, os.fsencode(path)))
        return self

    # ---- time stepping ------------------------------------------------------
    def step(self, nsteps: int = 1):
        _check(load().lbmx_step(self._h, int(nsteps)))
        return self

    def step_timed(self, nsteps: int) -> float:
        ms = ctypes.c_double()
        _check(load().lbmx_step_timed(self._h, int(nsteps), ctypes.byref(ms)))
        return float(ms.value)

    @property
    def t(self) -> int:
        t = ctypes.c_int64()
        _check(load().lbmx_time(self._h, ctypes.byref(t)))
        return int(t.value)

    def set_launch(self, bx: int = 0, by: int = 0):
        _check(load().lbmx_set_launch(self._h, int(bx), int(by)))
        return self

    def get_launch(self):
        bx, by = ctypes.c_int32(), ctypes.c_int32()
        _check(load().lbmx_get_launch(self._h, ctypes.byref(bx), ctypes.byref(by)))
        return int(bx.value), int(by.value)

    # ---- observables --------------------------------------------------------
    def read_macro(self):
        """(rho, ux, uy, uz, theta), each (n, n, n) indexed [z, y, x]."""
        arrs = [np.empty(self.cells) for _ in range(5)]
        _check(load().lbmx_read_macro(self._h, *[_dptr(a) for a in arrs]))
        return tuple(a.reshape((self.n,) * 3) for a in arrs)

    def nusselt(self, with_map=False, allow_unstable=False):
        out = lbmx_nu()
        mp = np.empty(self.n * self.n) if with_map else None
        st = load().lbmx_nusselt(self._h, ctypes.byref(out), _dptr(mp))
        _check(st, ok=(0, 4) if allow_unstable else (0,))
        d = {"nu3d": out.nu3d, "nu2d": out.nu2d, "numax": out.numax, "step": out.step,
             "nonfinite": out.nonfinite, "status": st}
        if with_map:
            d["map"] = mp.reshape(self.n, self.n)
        return d

    def run_to_steady(self, tol=1e-6, every=1000, max_steps=2_000_000):
        out = lbmx_nu()
        st = load().lbmx_run_to_steady(self._h, tol, int(every), int(max_steps), ctypes.byref(out))
        _check(st, ok=(0, 5))
        return {"nu3d": out.nu3d, "nu2d": out.nu2d, "numax": out.numax, "step": out.step,
                "converged": st == 0}

    def derived(self) -> dict:
        return derive(self.params)


class Batch:
    """Many cavities advanced together by one launch per step (lbmx_batch_*).

    cases: list of dicts with n, ra, wall_type and optional theta0 (n^3
    array) / params overrides; all share `storage`.
    """

    def __init__(self, cases, storage="f32", stream=None):
        import torch

        L = load()
        self.cases = [dict(c) for c in cases]
        arr = (lbmx_params * len(cases))()
        for k, c in enumerate(cases):
            kw = {k2: v for k2, v in c.items() if k2 not in ("theta0", "seed")}
            arr[k] = make_params(storage=storage, **kw)
        self.n = [int(c["n"]) for c in cases]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _vp()
        _check(L.lbmx_batch_create(arr, len(cases), _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._params = arr

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lbmx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __len__(self):
        return len(self.n)

    def init_rest(self, k, theta0=None):
        th = None if theta0 is None else np.ascontiguousarray(theta0, dtype=np.float64).reshape(-1)
        if th is not None and th.size != self.n[k] ** 3:
            raise ValueError("theta0 needs n^3 values")
        _check(load().lbmx_batch_init_rest(self._h, int(k), _dptr(th)))
        return self

    def init_from(self, k, src: "Batch", ks):
        """Cavity k at t = 0 from cavity ks of batch `src` (resampled on the
        device, ``lbmx_batch_init_from``)."""
        _check(load().lbmx_batch_init_from(self._h, int(k), src._h, int(ks)))
        return self

    def step(self, nsteps=1):
        _check(load().lbmx_batch_step(self._h, int(nsteps)))
        return self

    def run_to_steady(self, tol=1e-6, every=1000, max_steps=2_000_000):
        nc = ctypes.c_int32()
        st = load().lbmx_batch_run_to_steady(self._h, tol, int(every), int(max_steps),
                                             ctypes.byref(nc))
        _check(st, ok=(0, 4, 5))
        return int(nc.value)

    def info(self, k):
        s, t, nu = ctypes.c_int32(), ctypes.c_int64(), lbmx_nu()
        _check(load().lbmx_batch_info(self._h, int(k), ctypes.byref(s), ctypes.byref(t),
                                      ctypes.byref(nu)))
        return {"state": BATCH_STATE[s.value], "t": int(t.value), "nu3d": nu.nu3d,
                "nu2d": nu.nu2d, "numax": nu.numax}

    def nusselt(self, k):
        out = lbmx_nu()
        _check(load().lbmx_batch_nusselt(self._h, int(k), ctypes.byref(out)))
        return {"nu3d": out.nu3d, "nu2d": out.nu2d, "numax": out.numax, "step": out.step}

    def read_macro(self, k):
        n = self.n[k]
        arrs = [np.empty(n ** 3) for _ in range(5)]
        _check(load().lbmx_batch_read_macro(self._h, int(k), *[_dptr(a) for a in arrs]))
        return tuple(a.reshape((n,) * 3) for a in arrs)

    def resample(self, k, out_n=64):
        out = np.empty(4 * out_n ** 3, dtype=np.float32)
        _check(load().lbmx_batch_resample(self._h, int(k), int(out_n),
                                          out.ctypes.data_as(_fp)))
        return out.reshape(4, out_n, out_n, out_n)

    def set_launch(self, block=256, grid=0, graph_steps=64):
        _check(load().lbmx_batch_set_launch(self._h, int(block), int(grid), int(graph_steps)))
        return self

    def get_launch(self):
        b, g, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().lbmx_batch_get_launch(self._h, ctypes.byref(b), ctypes.byref(g),
                                            ctypes.byref(s)))
        return int(b.value), int(g.value), int(s.value)

    def autotune(self, cache_path=None):
        us = ctypes.c_double()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(load().lbmx_batch_autotune(self._h, path, ctypes.byref(us)))
        return float(us.value)

"""Host-side calls of the C-ABI, run in a subprocess against a build of the
library whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer
(tests/test_sanitizers.py builds it and preloads the sanitizer runtime).
Only calls that return before any device work are made: parameter defaults,
derivation and validation, sizes, error strings, NULL handles and rejected
network-kernel shapes.  Usage: python sanitize_abi_host.py LIBRARY.so"""
import ctypes
import math
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_1511_04633_amd.lbmx import lbmx_nu, lbmx_params  # noqa: E402  (no torch)

L = ctypes.CDLL(sys.argv[1])
P = ctypes.POINTER(lbmx_params)
vp = ctypes.c_void_p
for name, args in {"lbmx_params_default": [P], "lbmx_derive": [P, ctypes.POINTER(ctypes.c_double)],
                   "lbmx_workspace_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
                   "lbmx_bytes_per_cell": [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
                   "lbmx_create": [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
                   "lbmx_batch_create": [P, ctypes.c_int32, vp, ctypes.POINTER(vp)]}.items():
    getattr(L, name).argtypes = args
L.lbmx_strerror.restype = ctypes.c_char_p
L.lbmx_last_error.restype = ctypes.c_char_p

fails = []


def check(cond, what):
    if not cond:
        fails.append(what)


def params(**kw):
    p = lbmx_params()
    check(L.lbmx_params_default(ctypes.byref(p)) == 0, "params_default")
    for k, v in kw.items():
        if k in ("s", "tau", "aniso"):
            getattr(p, k)[:] = v
        else:
            setattr(p, k, v)
    return p


out = (ctypes.c_double * 6)()
for n, ra in ((4, 1e3), (16, 1e3), (256, 1e6), (1024, 1e7)):
    for st in range(7):
        p = params(n=n, ra=ra, storage=st)
        check(L.lbmx_derive(ctypes.byref(p), out) == 0, f"derive {n} {ra} {st}")
        ws = ctypes.c_size_t()
        check(L.lbmx_workspace_bytes(ctypes.byref(p), ctypes.byref(ws)) == 0 and ws.value > 0, "ws")
bad = [dict(n=3), dict(n=2048), dict(wall_type=0), dict(wall_type=4), dict(ra=0.0),
       dict(ra=float("inf")), dict(ra=float("nan")), dict(pr=0.0), dict(ma=0.0), dict(ma=0.9),
       dict(storage=-1), dict(storage=7), dict(theta_hot=float("nan")), dict(force_model=3),
       dict(nu_stencil=-1), dict(aniso=[1, 1, 1, 2, 0, 0]), dict(aniso=[1, 1, float("inf"), 0, 0, 0]),
       dict(custom_rates=1, s=[3.0] * 19, tau=[1.0] * 7),
       dict(custom_rates=1, s=[1.0] * 19, tau=[0.4] * 7),
       dict(custom_rates=1, s=[1.0] * 19, tau=[1.0] * 7, aniso=[1, 1, 1, 0, 0, 0]),
       dict(ra=1e300, pr=1e-300)]  # nu underflows to 0: s_nu = 2
for kw in bad:
    p = params(**kw)
    check(L.lbmx_derive(ctypes.byref(p), out) == 1, f"derive rejects {kw}")
    h = vp()
    check(L.lbmx_create(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == 1 and not h.value,
          f"create rejects {kw}")
    check(len(L.lbmx_last_error()) > 0, "last_error")
check(L.lbmx_derive(None, out) == 1 and L.lbmx_derive(ctypes.byref(params()), None) == 1, "NULL")
bpc = ctypes.c_double()
for st, want in enumerate((416, 208, 104, 104, 132, 132, 104)):
    check(L.lbmx_bytes_per_cell(st, ctypes.byref(bpc)) == 0 and bpc.value == want, f"bpc {st}")
check(L.lbmx_bytes_per_cell(9, ctypes.byref(bpc)) == 1, "bpc invalid")
arr = (lbmx_params * 3)(params(n=8), params(n=8, storage=2), params(n=8))
h = vp()
check(L.lbmx_batch_create(arr, 3, None, ctypes.byref(h)) == 1, "batch mixed storage")
arr = (lbmx_params * 2)(params(n=8), params(n=300))
check(L.lbmx_batch_create(arr, 2, None, ctypes.byref(h)) == 1, "batch n > 255")
check(L.lbmx_batch_create(arr, 0, None, ctypes.byref(h)) == 1, "batch count 0")
# NULL handles: EINVAL, no crash
nu = lbmx_nu()
check(L.lbmx_step(None, ctypes.c_int64(1)) == 1, "step NULL")
check(L.lbmx_nusselt(None, ctypes.byref(nu), None) == 1, "nusselt NULL")
check(L.lbmx_nusselt_noalloc(None, ctypes.byref(nu), None) == 1, "nusselt_noalloc NULL")
check(L.lbmx_read_macro(None, None, None, None, None, None) == 1, "read_macro NULL")
check(L.lbmx_set_launch(None, 64, 1) == 1, "set_launch NULL")
check(L.lbmx_batch_step(None, ctypes.c_int64(1)) == 1, "batch_step NULL")
check(L.lbmx_batch_info(None, 0, None, None, None) == 1, "batch_info NULL")
L.lbmx_destroy(None)
L.lbmx_batch_destroy(None)
for s in list(range(8)) + [99]:
    check(len(L.lbmx_strerror(s)) > 0, "strerror")
# network kernels: rejected shapes return before any launch
i32 = ctypes.c_int32
check(L.lbmx_nn_conv3d_fwd(None, None, None, None, i32(0), i32(1), i32(4), i32(4), i32(4), i32(8),
                           i32(16), None) == 1, "conv Ci 8")
check(L.lbmx_nn_conv3d_wgrad(None, None, None, None, i32(1), i32(4), i32(4), i32(4), i32(16),
                             i32(2048), None) == 1, "wgrad Co 2048")
if fails:
    print("FAILED:", fails)
    sys.exit(1)
print("sanitize_abi_host: host paths ran clean")

"""The C-ABI library loads and exports what include/lbmx.h declares; the
host-only calls (parameter derivation and validation, sizes, error strings)
work without a GPU."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from oracle import oracle as O
from paper_1511_04633_amd import lbmx as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbmx_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(L.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lbmx_\w+)", out))
    assert set(declared_functions()) <= exported


def test_params_struct_layout_matches_header():
    """The ctypes mirror has the C struct's size: 4+4 + 7*8 + 4+4 + 19*8 + 7*8
    + 4+4 + 6*8 (no padding anywhere)."""
    assert ctypes.sizeof(L.lbmx_params) == 8 + 56 + 8 + 152 + 56 + 8 + 48
    assert ctypes.sizeof(L.lbmx_nu) == 40


def test_derived_parameters_match_the_oracle():
    """Host derivation in the library (Eq. 38, 26, 36) equals the oracle's."""
    for n, ra in ((16, 1e3), (50, 1e4), (60, 1e5), (128, 1e5), (256, 1e6), (32, 1e6)):
        got = L.derive(L.make_params(n=n, ra=ra))
        want = O.derive(n, ra)
        for k in want:
            assert math.isclose(got[k], want[k], rel_tol=1e-15), (k, got[k], want[k])


def test_invalid_parameters_rejected_on_host():
    bad = [dict(n=3), dict(n=2048), dict(wall_type=0), dict(wall_type=4), dict(ra=0.0),
           dict(ra=-1.0), dict(pr=0.0), dict(ma=0.0), dict(ma=0.9), dict(storage=7), dict(storage=-1),
           dict(ra=float("inf")), dict(theta_hot=float("nan"))]
    for kw in bad:
        p = L.make_params(**kw)
        with pytest.raises(L.LbmxError) as e:
            L.derive(p)
        assert e.value.status == 1, kw
    with pytest.raises(L.LbmxError):
        L.derive(L.make_params(s=[1.0] * 19, tau=[1.0, 0.4, 1, 1, 1, 1, 1]))
    with pytest.raises(L.LbmxError):
        L.derive(L.make_params(s=[2.5] + [1.0] * 18, tau=[1.0] * 7))


def test_sizes():
    assert L.bytes_per_cell("f64") == 416.0
    assert L.bytes_per_cell("f32") == 208.0
    assert L.bytes_per_cell("f16") == 104.0 and L.bytes_per_cell("bf16") == 104.0
    assert L.bytes_per_cell("f16_f32") == 132.0 and L.bytes_per_cell("bf16_f32") == 132.0
    assert L.bytes_per_cell("f16_i16") == 104.0
    p = L.make_params(n=256, ra=1e6, storage="f32")
    ws = L.workspace_bytes(p)
    assert ws >= 2 * 26 * 256 ** 3 * 4
    assert ws < 2 * 26 * 256 ** 3 * 4 * 1.01


def test_error_strings():
    lib = L.load()
    for s in range(8):
        assert lib.lbmx_strerror(s) and lib.lbmx_strerror(s) != b"unknown status"
    assert lib.lbmx_strerror(99) == b"unknown status"


def test_null_arguments():
    lib = L.load()
    assert lib.lbmx_derive(None, None) == 1
    assert lib.lbmx_step(None, 1) == 1
    assert lib.lbmx_nusselt(None, None, None) == 1
    assert lib.lbmx_init_from_cavity(None, None) == 1
    assert lib.lbmx_init_from_cavities(None, None, 1.0, None, 0.0) == 1
    assert lib.lbmx_batch_init_from(None, 0, None, 0) == 1
    lib.lbmx_destroy(None)


def test_batch_create_rejects_sizes_before_any_device_call():
    """lbmx_batch_create validates sizes on the host: n > 255 fails with
    LBMX_EINVAL and no handle.  The largest admitted lattice (FP64, n = 255)
    stays under 4 GiB, which the batch kernel's 32-bit byte offsets need."""
    lib = L.load()
    arr = (L.lbmx_params * 2)()
    arr[0] = L.make_params(n=16, storage="f32")
    arr[1] = L.make_params(n=256, storage="f32")
    h = ctypes.c_void_p(123)
    assert lib.lbmx_batch_create(arr, 2, None, ctypes.byref(h)) == 1
    assert not h.value
    assert b"cavity 1" in lib.lbmx_last_error()
    for storage in ("f64", "f32", "f16_f32"):
        ws = L.workspace_bytes(L.make_params(n=255, storage=storage))
        assert ws // 2 < 2 ** 32, storage


def test_variant_parameters_validated():
    """Force model, Nu stencil and the anisotropy tensor are checked on the
    host: unknown values, a tensor that is not positive definite and aniso
    together with custom rates are EINVAL; valid sets derive."""
    L.derive(L.make_params(force_model="guo", nu_stencil="wall_flux",
                           aniso=[1.0, 0.6, 0.8, 0.3, 0.2, -0.25]))
    for kw in (dict(force_model=3), dict(force_model=-1), dict(nu_stencil=3),
               dict(aniso=[1, 1, 1, 1.5, 0, 0]), dict(aniso=[-1, 1, 1, 0, 0, 0]),
               dict(aniso=[1, 1, 0, 0, 0, 0]), dict(aniso=[1, 1, 1, 0, 0, float("nan")]),
               dict(aniso=[1, 1, 1, 0, 0, 0], s=[1.0] * 19, tau=[1.0] * 7)):
        with pytest.raises(L.LbmxError) as e:
            L.derive(L.make_params(**kw))
        assert e.value.status == 1, kw


def test_batch_rejects_mixed_force_models():
    lib = L.load()
    arr = (L.lbmx_params * 2)()
    arr[0] = L.make_params(n=16, force_model=0)
    arr[1] = L.make_params(n=16, force_model=2)
    h = ctypes.c_void_p()
    assert lib.lbmx_batch_create(arr, 2, None, ctypes.byref(h)) == 1
    assert b"force model" in lib.lbmx_last_error()


def test_convolution_plane_limits_rejected_on_host():
    """The convolution launchers reject, before any device call, shapes whose
    32-bit brick-relative offsets (a few H x W planes of C channels) would
    overflow although the voxel count fits: one 8192 x 8192 plane of 16
    channels.  The pointers are never dereferenced."""
    from paper_1511_04633_amd import unet
    lib = unet.nn()
    p = ctypes.c_void_p(256)
    shape = (1, 1, 8192, 8192, 16, 16)
    assert lib.lbmx_nn_conv3d_fwd(p, p, None, p, 0, *shape, None) == 1
    assert b"brick offsets" in lib.lbmx_last_error()
    assert lib.lbmx_nn_conv3d_wgrad(p, p, p, None, *shape, None) == 1
    assert b"brick offsets" in lib.lbmx_last_error()
    assert lib.lbmx_nn_conv3d_mse(p, p, None, p, 4, p, p, 64, None, *shape, None) == 1
    assert b"brick offsets" in lib.lbmx_last_error()
    assert lib.lbmx_nn_conv3d_fwd(p, p, None, p, 0, 1, 1, 8192, 8192, 16, 1040, None) == 1
    assert b"multiples of 16" in lib.lbmx_last_error()

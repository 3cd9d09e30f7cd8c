"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/smsm.h, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1901_01893_amd as pkg
from paper_1901_01893_amd import smsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smsm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smsm_[a-z_A-Z0-9]+)\s*\(", text)))


needs_lib = pytest.mark.skipif(not os.path.exists(smsm.LIB_PATH), reason="libsmsm.so not built")


def test_binding_lists_every_declared_symbol():
    assert sorted(smsm.ABI_SYMBOLS) == declared_symbols()


def test_binding_has_a_function_per_declared_symbol():
    # the thin binding mirrors every C entry point under the same name
    for name in declared_symbols():
        assert callable(getattr(smsm, name, None)), name


def test_flat_names_are_the_marshalling_methods():
    # each flat name is the class method (or constructor) that marshals the
    # call, so no name can drift from what the class does
    owners = {"plan": smsm.Plan, "batch": smsm.Batch, "learned": smsm.Learned, "al": smsm.AL}
    for name in declared_symbols():
        f = getattr(smsm, name)
        if name == "smsm_status_string":
            assert f is smsm.status_string
            continue
        kind = next((k for k in ("batch", "learned", "al") if name.startswith(f"smsm_{k}_")), "plan")
        cls = owners[kind]
        assert f is cls or any(f is getattr(v, "fget", v) for v in vars(cls).values()), name


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(smsm.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


@needs_lib
def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert pkg.status_string(code) != "unknown status"
    assert pkg.status_string(-99) == "unknown status"


def _create(geom, params, coil_ptr, masks, out):
    lib = smsm.lib()
    return lib.smsm_plan_create(
        ctypes.byref(geom) if geom is not None else None,
        ctypes.byref(params) if params is not None else None,
        coil_ptr, masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if masks is not None else None,
        None, None, out)


@needs_lib
def test_plan_create_rejects_bad_arguments_without_a_device():
    geom = smsm.Geometry(64, 64, 2, 4, 8, 5)
    params = smsm.make_params()
    masks = np.stack([(np.arange(64) % 4 == i) for i in range(4)]).astype(np.uint8)
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    out = ctypes.c_void_p()
    assert _create(geom, params, fake, masks, None) == pkg.SMSM_E_INVALID
    assert _create(None, params, fake, masks, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert _create(geom, None, fake, masks, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert _create(geom, params, None, masks, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    bad = smsm.make_params(lam=-1.0)
    assert _create(geom, bad, fake, masks, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    bad = smsm.make_params(n_irls=0)
    assert _create(geom, bad, fake, masks, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert _create(smsm.Geometry(60, 64, 2, 4, 8, 5), params, fake, masks, ctypes.byref(out)) == \
        pkg.SMSM_E_UNSUPPORTED                       # not a power of two
    assert _create(smsm.Geometry(64, 64, 2, 4, 8, 40), params, fake, masks, ctypes.byref(out)) == \
        pkg.SMSM_E_UNSUPPORTED                       # filter wider than the grid allows
    other = masks.copy()
    other[0, 1] = 1                                   # not the interleaved pattern
    assert _create(geom, params, fake, other, ctypes.byref(out)) == pkg.SMSM_E_UNSUPPORTED
    assert out.value is None


@needs_lib
def test_entry_points_reject_null_plan():
    lib = smsm.lib()
    for name in ("smsm_apply_A", "smsm_apply_AH", "smsm_apply_AHA", "smsm_gram", "smsm_lambda_max",
                 "smsm_apply_reg", "smsm_apply_normal", "smsm_solve"):
        assert getattr(lib, name)(None, None, None, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_set_weights(None, None, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_plan_destroy(None) == pkg.SMSM_OK
    assert lib.smsm_plan_device_bytes(None) == 0
    assert lib.smsm_workspace_bytes(None) == 0
    assert lib.smsm_set_workspace(None, None, 0) == pkg.SMSM_E_INVALID
    shape = (ctypes.c_int * 2)()
    assert lib.smsm_plan_autotune(None, 10, shape, None) == pkg.SMSM_E_INVALID


@needs_lib
def test_batch_timer_and_image_entry_points_reject_bad_arguments():
    lib = smsm.lib()
    vp = ctypes.c_void_p
    assert lib.smsm_images_sos(None, None, None, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_kernel_timer_start(None, 0, 1, 1) == pkg.SMSM_E_INVALID
    ms, n = ctypes.c_double(), ctypes.c_int()
    assert lib.smsm_kernel_timer_read(None, ctypes.byref(ms), ctypes.byref(n)) == pkg.SMSM_E_INVALID
    out = vp()
    arr = (vp * 1)(vp(0x1000))              # never dereferenced: validation fails first
    null = (vp * 1)(None)
    assert lib.smsm_batch_create(None, 1, arr, arr, 1, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_batch_create(null, 1, arr, arr, 1, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_batch_create(arr, 0, arr, arr, 1, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_batch_create(arr, 1, arr, arr, -1, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_batch_create(arr, 1, arr, arr, 65, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_batch_create(arr, 1, arr, arr, 1, None) == pkg.SMSM_E_INVALID
    assert out.value is None
    assert lib.smsm_batch_launch(None, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_batch_destroy(None) == pkg.SMSM_OK
    assert lib.smsm_batch_streams(None) == 0


@needs_lib
def test_learned_entry_points_reject_bad_arguments():
    lib = smsm.lib()
    out = ctypes.c_void_p()
    params = np.zeros(16, np.float32)
    pf = params.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    assert lib.smsm_learned_create(None, 64, 5, 10, 1.0, pf, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    fake = ctypes.c_void_p(0x1000)            # never dereferenced: validation fails first
    assert lib.smsm_learned_create(fake, 64, 5, 10, 1.0, None, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_create(fake, 60, 5, 10, 1.0, pf, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_create(fake, 64, 0, 10, 1.0, pf, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_create(fake, 64, 5, 10, 0.0, pf, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_create(fake, 64, 5, 10, 1.0, pf, None) == pkg.SMSM_E_INVALID
    assert out.value is None
    assert lib.smsm_learned_destroy(None) == pkg.SMSM_OK
    assert lib.smsm_learned_param_count(None) == 0
    assert lib.smsm_learned_get_params(None, pf) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_set_params(None, pf) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_cnn_forward(None, None, None, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_cnn_backward(None, None, None, None, pf, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_solve(None, None, None, None) == pkg.SMSM_E_INVALID
    d = ctypes.c_double()
    assert lib.smsm_learned_gradients(None, None, None, ctypes.byref(d), pf, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_train_step(None, None, None, 1e-3, ctypes.byref(d), None) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_residual(None, None, None, ctypes.byref(d), None) == pkg.SMSM_E_INVALID
    assert lib.smsm_learned_set_bf16(None, 1) == pkg.SMSM_E_INVALID
    r2 = (ctypes.c_double * 2)()
    fb = ctypes.c_int()
    assert lib.smsm_learned_solve_fallback(None, None, None, 1.5, 0.0, r2, ctypes.byref(fb), None) == \
        pkg.SMSM_E_INVALID


@needs_lib
def test_al_entry_points_reject_bad_arguments():
    lib = smsm.lib()
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)            # never dereferenced: validation fails first
    good = smsm.ALParams(1e-3, 1e-4, 10, 5, 0, 0)
    assert lib.smsm_al_create(None, ctypes.byref(good), ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_al_create(fake, None, ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert lib.smsm_al_create(fake, ctypes.byref(good), None) == pkg.SMSM_E_INVALID
    for bad in (smsm.ALParams(0.0, 1e-4, 10, 5, 0, 0), smsm.ALParams(1e-3, 0.0, 10, 5, 0, 0),
                smsm.ALParams(1e-3, float("nan"), 10, 5, 0, 0), smsm.ALParams(1e-3, 1e-4, 0, 5, 0, 0),
                smsm.ALParams(1e-3, 1e-4, 10, -1, 0, 0), smsm.ALParams(1e-3, 1e-4, 10, 5, -1, 0),
                smsm.ALParams(1e-3, 1e-4, 10, 5, 201, 0), smsm.ALParams(1e-3, 1e-4, 10, 5, 0, 0x2)):
        assert lib.smsm_al_create(fake, ctypes.byref(bad), ctypes.byref(out)) == pkg.SMSM_E_INVALID
    assert out.value is None
    assert lib.smsm_al_destroy(None) == pkg.SMSM_OK
    assert lib.smsm_al_device_bytes(None) == 0
    assert lib.smsm_al_dual_stride(None) == 0
    assert lib.smsm_al_solve(None, None, None, None) == pkg.SMSM_E_INVALID
    assert lib.smsm_al_dual(None, None, None) == pkg.SMSM_E_INVALID


def test_learned_parameter_layout_round_trip():
    import smsm_inputs as si
    params = si.cnn_init(1, 8, width=16)
    flat = smsm.flatten_params(params)
    assert flat.size == 8 * 16 * 9 + 16 + 3 * (16 * 16 * 9 + 16) + 16 * 8 * 9 + 8
    back = smsm.unflatten_params(flat, 8, 16)
    for (w, b), (w2, b2) in zip(params, back):
        assert np.array_equal(w, w2) and np.array_equal(b, b2)

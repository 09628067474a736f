"""C-ABI checks that need no GPU: the shared library loads, exports every
symbol include/mps_lbm.h declares, and rejects bad arguments before it
touches a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lib():
    from paper_2512_07615_amd import mps_lbm as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    return L


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mps_lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mps_lbm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    for need in ["mps_lbm_init_from_field", "mps_lbm_step", "mps_lbm_to_dense",
                 "mps_lbm_observables", "mps_lbm_destroy", "mps_lbm_last_error"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    L = lib()
    so = C.CDLL(L.LIB_PATH)
    for name in declared_functions():
        getattr(so, name)  # raises AttributeError if missing
    assert sorted(L.EXPORTED) == declared_functions()


def test_config_struct_layout_matches_header():
    L = lib()
    # field order/sizes of mps_lbm_config as declared in the header
    c = L.Config
    assert c.n.offset == 0
    assert c.tol.offset % 8 == 0
    assert c.rank_predictor.offset == c.seed.offset + 8
    assert C.sizeof(c) == c.rank_oversample.offset + 4


def test_default_config_values():
    L = lib()
    c = L.mps_lbm_default_config()
    assert c.lattice == L.D3Q19 and c.chi_max == 16 and c.sweeps == 2
    assert c.tol == 1e-10 and c.tau == 0.8 and c.precision == L.FP64


@pytest.mark.parametrize("field,value,code", [
    ("tau", 0.5, -1), ("tau", 0.3, -1), ("n", 1, -1), ("n", 11, -1), ("chi_max", 0, -1),
    ("lattice", 15, -1), ("precision", 7, -1), ("inv_rho_mode", 9, -1), ("sweeps", 0, -1),
    ("chi_max", 4096, -5), ("rank_predictor", 3, -1), ("rank_predictor", 1, -5),
])
def test_invalid_config_rejected_before_device_use(field, value, code):
    L = lib()
    c = L.mps_lbm_default_config()
    setattr(c, field, value)
    h = C.c_void_p()
    so = L.load()
    rc = so.mps_lbm_init_from_field(C.byref(c), None, None, None, None, None, C.byref(h))
    assert rc == code
    assert so.mps_lbm_last_error().decode() != ""
    assert not h.value


def test_bc_on_periodic_axis_and_missing_fields_rejected():
    L = lib()
    so = L.load()
    c = L.mps_lbm_default_config()
    c.face_bc[0] = L.BC_PRESSURE
    c.face_val[0][0] = 1.0
    h = C.c_void_p()
    assert so.mps_lbm_init_from_field(C.byref(c), None, None, None, None, None,
                                      C.byref(h)) == L.EINVAL
    c = L.mps_lbm_default_config()
    c.axis_open[0] = 1
    c.face_bc[1] = L.BC_PRESSURE
    c.face_val[1][0] = 0.0   # rho_b must be positive
    assert so.mps_lbm_init_from_field(C.byref(c), None, None, None, None, None,
                                      C.byref(h)) == L.EINVAL
    c = L.mps_lbm_default_config()
    rho = np.ones((16, 16, 16))
    # u missing and f missing
    assert so.mps_lbm_init_from_field(C.byref(c), rho.ctypes.data_as(C.POINTER(C.c_double)),
                                      None, None, None, None, C.byref(h)) == L.EINVAL


def test_tensor_mask_init_validates_its_parts_before_device_use():
    L = lib()
    so = L.load()
    c = L.mps_lbm_default_config()
    c.n = 5
    rho = np.ones((32, 32, 32))
    u = np.zeros((3, 32, 32, 32))
    outer = np.zeros((8, 8, 8), dtype=np.uint8)
    inner = np.zeros((4, 4, 4), dtype=np.uint8)
    DP = C.POINTER(C.c_double)
    U8 = C.POINTER(C.c_uint8)
    h = C.c_void_p()
    args = (rho.ctypes.data_as(DP), u.ctypes.data_as(DP), None)
    # NULL parts
    assert so.mps_lbm_init_tensor_mask(C.byref(c), *args, None, 3, inner.ctypes.data_as(U8),
                                       None, C.byref(h)) == L.EINVAL
    assert so.mps_lbm_init_tensor_mask(C.byref(c), *args, outer.ctypes.data_as(U8), 3, None,
                                       None, C.byref(h)) == L.EINVAL
    # each part needs at least two sites
    for l in (1, 4, 0, 7):
        assert so.mps_lbm_init_tensor_mask(C.byref(c), *args, outer.ctypes.data_as(U8), l,
                                           inner.ctypes.data_as(U8), None,
                                           C.byref(h)) == L.EINVAL
    assert not h.value
    # the binding checks the shapes of the parts
    with pytest.raises(ValueError):
        L.mps_lbm_init_tensor_mask(c, outer, np.zeros((8, 8, 8), np.uint8), rho=rho, u=u)


def test_profile_and_region_entry_points_validate_without_gpu():
    L = lib()
    so = L.load()
    coef = (C.c_double * 6)(0, 1, 1.5, 0, 0, 0)
    lo = (C.c_int * 3)(0, 0, 0)
    hi = (C.c_int * 3)(2, 2, 2)
    assert so.mps_lbm_set_face_profile(None, 0, 0, coef, 0.1) == L.EINVAL
    assert so.mps_lbm_set_face_profile(None, 0, 0, None, 0.0) == L.EINVAL
    assert so.mps_lbm_set_region(None, 0, lo, hi, 1.0) == L.EINVAL
    with pytest.raises(ValueError):
        L.mps_lbm_set_face_profile(None, 0, (1, 2, 3), 0.1)
    with pytest.raises(ValueError):
        L.mps_lbm_set_region(None, (0, 0), (1, 1, 1), 1.0)


def test_null_handle_calls_fail_cleanly():
    L = lib()
    so = L.load()
    assert so.mps_lbm_step(None, 1) == L.EINVAL
    out = np.zeros(8)
    assert so.mps_lbm_to_dense(None, 0, out.ctypes.data_as(C.POINTER(C.c_double)), 8) == L.EINVAL
    o = L.Obs()
    assert so.mps_lbm_observables(None, C.byref(o)) == L.EINVAL
    so.mps_lbm_destroy(None)
    assert so.mps_lbm_version().decode().startswith("mps-lbm")


def test_batch_init_validation_before_device_use():
    L = lib()
    so = L.load()
    h = C.c_void_p()
    c0 = L.mps_lbm_default_config()
    c1 = L.mps_lbm_default_config()
    arr = (L.Config * 2)(c0, c1)
    rho = np.ones((16, 16, 16))
    u = np.zeros((3, 16, 16, 16))
    dp = C.POINTER(C.c_double)
    R = (dp * 2)(rho.ctypes.data_as(dp), rho.ctypes.data_as(dp))
    U = (dp * 2)(u.ctypes.data_as(dp), u.ctypes.data_as(dp))
    # count < 1, NULL fields
    assert so.mps_lbm_init_batch(arr, 0, R, U, None, None, C.byref(h)) == L.EINVAL
    assert so.mps_lbm_init_batch(arr, 2, None, U, None, None, C.byref(h)) == L.EINVAL
    # an invalid member configuration (domains may otherwise differ: they
    # then form groups)
    arr = (L.Config * 2)(L.mps_lbm_default_config(), L.mps_lbm_default_config())
    arr[1].tau = 0.4
    assert so.mps_lbm_init_batch(arr, 2, R, U, None, None, C.byref(h)) == L.EINVAL
    assert not h.value
    assert so.mps_lbm_domains(None) == L.EINVAL
    o = L.Obs()
    assert so.mps_lbm_observables_domain(None, 0, C.byref(o)) == L.EINVAL


def test_predictor_entry_points_validate_without_gpu():
    """The learned-predictor entry points reject bad arguments before any
    device call."""
    L = lib()
    so = L.load()
    fp = C.POINTER(C.c_float)
    z = (C.c_float * 64)()
    zp = C.cast(z, fp)
    loss = C.c_float()
    big = (C.c_float * L.MLP_NPARAM)()
    assert so.mps_lbm_mlp_gradient(C.cast(big, fp), zp, zp, 0, C.byref(loss), C.cast(big, fp)) == -1
    assert so.mps_lbm_mlp_gradient(C.cast(big, fp), zp, zp, 2000, C.byref(loss), C.cast(big, fp)) == -1
    assert so.mps_lbm_mlp_gradient(None, zp, zp, 1, C.byref(loss), C.cast(big, fp)) == -1
    assert so.mps_lbm_train_rank_predictor(None, 1, 1e-3, None) == -1
    info = L.PredictorInfo()
    assert so.mps_lbm_rank_predictor_info(None, C.byref(info)) == -1


def test_allocator_registration_validates_and_resets():
    """mps_lbm_set_allocator takes both callbacks or neither."""
    L = lib()
    so = L.load()
    a = L.ALLOC_FN(lambda size, stream, ctx: None)
    f = L.FREE_FN(lambda ptr, stream, ctx: None)
    assert so.mps_lbm_set_allocator(a, L.FREE_FN(), None) == L.EINVAL
    assert so.mps_lbm_set_allocator(L.ALLOC_FN(), f, None) == L.EINVAL
    assert so.mps_lbm_set_allocator(a, f, None) == L.OK
    assert so.mps_lbm_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None) == L.OK


def test_model_and_debug_entry_points_validate_without_gpu():
    L = lib()
    so = L.load()
    fp = C.POINTER(C.c_float)
    w = (C.c_float * L.MLP_NPARAM)()
    assert so.mps_lbm_load_rank_model(None, C.cast(w, fp), L.MLP_NPARAM) == L.EINVAL
    assert so.mps_lbm_get_rank_model(None, C.cast(w, fp), L.MLP_NPARAM) == L.EINVAL
    assert so.mps_lbm_debug_raise_flags(None, 1, 0) == L.EINVAL


def test_every_entry_point_that_reaches_the_engine_is_guarded():
    """No C++ exception may cross the C ABI: every exported function whose
    body calls into a handle's simulation (or creates one) runs that call
    inside guarded(), which catches Error, std::bad_alloc, std::exception
    and anything else."""
    src = open(os.path.join(ROOT, "paper_2512_07615_amd", "csrc", "mps_lbm.hip")).read()
    body_of = {}
    start = src.index('extern "C" {')
    for m in re.finditer(r"\n(?:int|void|const char\*) (mps_lbm_[a-z_]+)\([^)]*\)[^{;]*\{", src[start:]):
        i = start + m.end()
        depth = 1
        j = i
        while depth:
            depth += {"{": 1, "}": -1}.get(src[j], 0)
            j += 1
        body_of[m.group(1)] = src[i:j]
    assert len(body_of) >= 24
    no_engine = ("->domains()", "->cells()", "->fatal_seen()")
    for name, body in body_of.items():
        calls = re.findall(r"->sim->[a-z_]+\(\)?", body)
        calls = [c for c in calls if not any(c.startswith("->sim" + x[:-2]) for x in no_engine)]
        if calls or "new " in body or "hipMemcpy" in body:
            assert "guarded(" in body or name == "mps_lbm_destroy", name
    # create(), which the init entry points call, runs inside guarded()
    c0 = src.index("static int create(")
    assert "return guarded(" in src[c0:src.index("int mps_lbm_init_from_field", c0)]
    assert "catch (...)" in src[src.index("static int guarded"):start]
    assert "catch (...)" in body_of["mps_lbm_destroy"]

"""Thin ctypes binding of the gfx950 MPS lattice Boltzmann library.

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  The names follow the C ABI declared in
include/mps_lbm.h.  Loading fails loudly when the shared library has not
been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmps_lbm.so")

MAX_SITES = 10

OK, EINVAL, ENOMEM, EHIP, ENUMERIC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
D3Q19 = 19
D3Q15 = 15
FP64, FP32, BF16, BF16X3 = 0, 1, 2, 3
INV_TAYLOR2, INV_NEWTON = 0, 1
BC_NONE, BC_VELOCITY, BC_PRESSURE = 0, 1, 2
POPS, RHO, J, VEL = 0, 1, 2, 3

K_NONE, K_JACOBI, K_HOUSEHOLDER, K_PRODGEMM, K_CHOLESKY = 0, 1, 2, 3, 4
MPS_MASK = 19

EXPORTED = sorted(["mps_lbm_default_config", "mps_lbm_init_from_field", "mps_lbm_step",
                   "mps_lbm_to_dense", "mps_lbm_observables", "mps_lbm_destroy",
                   "mps_lbm_last_error", "mps_lbm_version", "mps_lbm_kernel_timing",
                   "mps_lbm_kernel_stats", "mps_lbm_get_mps", "mps_lbm_init_batch",
                   "mps_lbm_domains", "mps_lbm_to_dense_domain",
                   "mps_lbm_observables_domain", "mps_lbm_capture_step",
                   "mps_lbm_train_rank_predictor", "mps_lbm_rank_predictor_info",
                   "mps_lbm_mlp_gradient", "mps_lbm_autotune", "mps_lbm_set_allocator",
                   "mps_lbm_load_rank_model", "mps_lbm_get_rank_model",
                   "mps_lbm_debug_raise_flags", "mps_lbm_mlp_gradient_device",
                   "mps_lbm_init_tensor_mask", "mps_lbm_set_face_profile",
                   "mps_lbm_set_region", "mps_lbm_kinetic_energy"])


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("lattice", C.c_int), ("chi_max", C.c_int), ("chi_mask_max", C.c_int),
        ("tol", C.c_double), ("tol_mask", C.c_double), ("tau", C.c_double),
        ("g", C.c_double * 3), ("inv_rho_mode", C.c_int), ("inv_rho_iters", C.c_int),
        ("precision", C.c_int), ("sweeps", C.c_int), ("axis_open", C.c_int * 3),
        ("face_bc", C.c_int * 6), ("face_val", (C.c_double * 3) * 6),
        ("seed", C.c_ulonglong), ("rank_predictor", C.c_int), ("rank_oversample", C.c_int),
    ]


class Obs(C.Structure):
    _fields_ = [
        ("step", C.c_longlong), ("mass", C.c_double), ("momentum", C.c_double * 3),
        ("rho0", C.c_double), ("n_fluid", C.c_double), ("max_bond", C.c_int),
        ("bonds", (C.c_int * MAX_SITES) * 19), ("nvps", C.c_double),
        ("compression", C.c_double), ("max_discarded", C.c_double), ("mask_bond", C.c_int),
        ("mask_trunc_err", C.c_double), ("roundings", C.c_longlong),
        ("products", C.c_longlong), ("svd_failures", C.c_int), ("nonfinite", C.c_int),
        ("jacobi_sweeps", C.c_double), ("lds_bytes", C.c_int),
        ("rs_attempted", C.c_longlong), ("rs_accepted", C.c_longlong),
        ("jacobi_sweeps_wide", C.c_double), ("jacobi_cols_wide", C.c_double),
        ("face_trunc_err", C.c_double),
        ("dp_p0", C.c_double),
        ("region_cells", C.c_double),
        ("region_trunc_err", C.c_double),
    ]


class PredictorInfo(C.Structure):
    _fields_ = [("samples", C.c_longlong), ("trained", C.c_int), ("first_loss", C.c_double),
                ("last_loss", C.c_double), ("predictions", C.c_longlong),
                ("mlp_abs_err", C.c_double), ("prev_abs_err", C.c_double)]


MLP_IN, MLP_H = 33, 128
MLP_NPARAM = MLP_IN * MLP_H + MLP_H + 2 * (MLP_H * MLP_H + MLP_H) + MLP_H + 1


class KStats(C.Structure):
    _fields_ = [("launches", C.c_longlong), ("total_ms", C.c_double), ("flops", C.c_double)]


_lib = None

# device allocator callbacks: alloc(bytes, stream, ctx) -> ptr, free(ptr, stream, ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_callbacks = []  # registered callbacks stay referenced while the library may call them


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P = C.c_void_p
    DP = C.POINTER(C.c_double)
    lib.mps_lbm_default_config.argtypes = [C.POINTER(Config)]
    lib.mps_lbm_default_config.restype = None
    lib.mps_lbm_init_from_field.argtypes = [C.POINTER(Config), DP, DP, DP,
                                            C.POINTER(C.c_uint8), P, C.POINTER(P)]
    lib.mps_lbm_init_from_field.restype = C.c_int
    lib.mps_lbm_init_tensor_mask.argtypes = [C.POINTER(Config), DP, DP, DP,
                                             C.POINTER(C.c_uint8), C.c_int,
                                             C.POINTER(C.c_uint8), P, C.POINTER(P)]
    lib.mps_lbm_init_tensor_mask.restype = C.c_int
    lib.mps_lbm_set_face_profile.argtypes = [P, C.c_int, C.c_int, DP, C.c_double]
    lib.mps_lbm_set_face_profile.restype = C.c_int
    lib.mps_lbm_set_region.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.c_double]
    lib.mps_lbm_set_region.restype = C.c_int
    lib.mps_lbm_kinetic_energy.argtypes = [P, C.c_int, DP]
    lib.mps_lbm_kinetic_energy.restype = C.c_int
    lib.mps_lbm_step.argtypes = [P, C.c_int]
    lib.mps_lbm_step.restype = C.c_int
    lib.mps_lbm_to_dense.argtypes = [P, C.c_int, DP, C.c_size_t]
    lib.mps_lbm_to_dense.restype = C.c_int
    lib.mps_lbm_observables.argtypes = [P, C.POINTER(Obs)]
    lib.mps_lbm_observables.restype = C.c_int
    lib.mps_lbm_destroy.argtypes = [P]
    lib.mps_lbm_destroy.restype = None
    lib.mps_lbm_last_error.argtypes = []
    lib.mps_lbm_last_error.restype = C.c_char_p
    lib.mps_lbm_version.argtypes = []
    lib.mps_lbm_version.restype = C.c_char_p
    lib.mps_lbm_kernel_timing.argtypes = [P, C.c_int]
    lib.mps_lbm_kernel_timing.restype = C.c_int
    lib.mps_lbm_kernel_stats.argtypes = [P, C.POINTER(KStats)]
    lib.mps_lbm_kernel_stats.restype = C.c_int
    lib.mps_lbm_get_mps.argtypes = [P, C.c_int, DP, C.c_size_t, C.POINTER(C.c_int)]
    lib.mps_lbm_get_mps.restype = C.c_int
    lib.mps_lbm_init_batch.argtypes = [C.POINTER(Config), C.c_int, C.POINTER(DP), C.POINTER(DP),
                                       C.POINTER(C.POINTER(C.c_uint8)), P, C.POINTER(P)]
    lib.mps_lbm_init_batch.restype = C.c_int
    lib.mps_lbm_capture_step.argtypes = [P]
    lib.mps_lbm_capture_step.restype = C.c_int
    lib.mps_lbm_domains.argtypes = [P]
    lib.mps_lbm_domains.restype = C.c_int
    lib.mps_lbm_to_dense_domain.argtypes = [P, C.c_int, C.c_int, DP, C.c_size_t]
    lib.mps_lbm_to_dense_domain.restype = C.c_int
    lib.mps_lbm_observables_domain.argtypes = [P, C.c_int, C.POINTER(Obs)]
    lib.mps_lbm_observables_domain.restype = C.c_int
    FP = C.POINTER(C.c_float)
    lib.mps_lbm_train_rank_predictor.argtypes = [P, C.c_int, C.c_double, DP]
    lib.mps_lbm_train_rank_predictor.restype = C.c_int
    lib.mps_lbm_rank_predictor_info.argtypes = [P, C.POINTER(PredictorInfo)]
    lib.mps_lbm_rank_predictor_info.restype = C.c_int
    lib.mps_lbm_mlp_gradient.argtypes = [FP, FP, FP, C.c_int, FP, FP]
    lib.mps_lbm_mlp_gradient.restype = C.c_int
    lib.mps_lbm_autotune.argtypes = [P, C.POINTER(C.c_int)]
    lib.mps_lbm_autotune.restype = C.c_int
    lib.mps_lbm_set_allocator.argtypes = [ALLOC_FN, FREE_FN, P]
    lib.mps_lbm_set_allocator.restype = C.c_int
    lib.mps_lbm_load_rank_model.argtypes = [P, FP, C.c_size_t]
    lib.mps_lbm_load_rank_model.restype = C.c_int
    lib.mps_lbm_get_rank_model.argtypes = [P, FP, C.c_size_t]
    lib.mps_lbm_get_rank_model.restype = C.c_int
    lib.mps_lbm_debug_raise_flags.argtypes = [P, C.c_int, C.c_int]
    lib.mps_lbm_debug_raise_flags.restype = C.c_int
    lib.mps_lbm_mlp_gradient_device.argtypes = [P, P, P, C.c_int, P, P, P]
    lib.mps_lbm_mlp_gradient_device.restype = C.c_int
    _lib = lib
    return lib


class MpsLbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mps_lbm error {code}: {msg}")
        self.code = code


def _check(code):
    if code != OK:
        raise MpsLbmError(code, load().mps_lbm_last_error().decode())


def mps_lbm_default_config() -> Config:
    c = Config()
    load().mps_lbm_default_config(C.byref(c))
    return c


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def mps_lbm_init_from_field(cfg: Config, rho=None, u=None, f=None, solid=None,
                            hip_stream: Optional[int] = None):
    """Create a simulation handle; arrays are C-order FP64 ([x][y][z])."""
    lib = load()
    rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    s = None
    if solid is not None:
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        s = solid.ctypes.data_as(C.POINTER(C.c_uint8))
    h = C.c_void_p()
    _check(lib.mps_lbm_init_from_field(C.byref(cfg), _dp(rho), _dp(u), _dp(f), s,
                                       C.c_void_p(hip_stream or 0), C.byref(h)))
    return h


def mps_lbm_init_tensor_mask(cfg: Config, solid_outer, solid_inner, rho=None, u=None, f=None,
                             hip_stream: Optional[int] = None):
    """Create a simulation whose obstacle mask is solid_outer (x) solid_inner
    (cubic uint8 arrays of sides 2**l and 2**(n - l))."""
    lib = load()
    rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    outer = np.ascontiguousarray(solid_outer, dtype=np.uint8)
    inner = np.ascontiguousarray(solid_inner, dtype=np.uint8)
    L = outer.shape[0] if outer.ndim == 3 else 0
    if L < 1 or outer.shape != (L, L, L) or L & (L - 1):
        raise ValueError("solid_outer must be a cube of side 2**l")
    K = (1 << cfg.n) // L
    if inner.shape != (K, K, K):
        raise ValueError("solid_inner must be a cube of side 2**(n - l)")
    h = C.c_void_p()
    _check(lib.mps_lbm_init_tensor_mask(
        C.byref(cfg), _dp(rho), _dp(u), _dp(f), outer.ctypes.data_as(C.POINTER(C.c_uint8)),
        int(L).bit_length() - 1, inner.ctypes.data_as(C.POINTER(C.c_uint8)),
        C.c_void_p(hip_stream or 0), C.byref(h)))
    return h


def mps_lbm_set_face_profile(h, face: int, coef=None, dt: float = 0.0, domain: int = 0):
    """Time profile u_b(t) = u_b phi(t) of a velocity face; coef = (c0..c5)
    of phi = c0 + c1 (1 - e^(-c2 t)) + c3 t^c4 e^(-c5 t), t = steps x dt;
    None restores the constant face."""
    c = None
    if coef is not None:
        if len(coef) != 6:
            raise ValueError("coef needs six entries")
        c = (C.c_double * 6)(*[float(v) for v in coef])
    _check(load().mps_lbm_set_face_profile(h, int(domain), int(face), c, float(dt)))


def mps_lbm_set_region(h, lo, hi, rho_ref: float, domain: int = 0):
    """Region (fluid cells of the box lo <= x < hi) of the Delta p / p_0
    observable, with p_0 = c_s^2 rho_ref."""
    if len(lo) != 3 or len(hi) != 3:
        raise ValueError("lo and hi need three entries")
    a = (C.c_int * 3)(*[int(v) for v in lo])
    b = (C.c_int * 3)(*[int(v) for v in hi])
    _check(load().mps_lbm_set_region(h, int(domain), a, b, float(rho_ref)))


def mps_lbm_kinetic_energy(h, domain: int = 0) -> float:
    """(1 / (2 N^3)) sum_x |j / rho|^2 of the state, lattice units."""
    e = C.c_double()
    _check(load().mps_lbm_kinetic_energy(h, int(domain), C.byref(e)))
    return e.value


def mps_lbm_train_rank_predictor(h, epochs: int, lr: float) -> float:
    loss = C.c_double()
    _check(load().mps_lbm_train_rank_predictor(h, int(epochs), float(lr), C.byref(loss)))
    return loss.value


def mps_lbm_autotune(h) -> int:
    n = C.c_int()
    _check(load().mps_lbm_autotune(h, C.byref(n)))
    return n.value


def mps_lbm_rank_predictor_info(h) -> PredictorInfo:
    o = PredictorInfo()
    _check(load().mps_lbm_rank_predictor_info(h, C.byref(o)))
    return o


def mps_lbm_mlp_gradient(params, x, t):
    """Loss and gradient of the predictor network (FP32 arrays: params of
    MLP_NPARAM, x of batch x 33, t of batch)."""
    fp = C.POINTER(C.c_float)
    params = np.ascontiguousarray(params, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    grad = np.zeros(MLP_NPARAM, dtype=np.float32)
    loss = C.c_float()
    _check(load().mps_lbm_mlp_gradient(params.ctypes.data_as(fp), x.ctypes.data_as(fp),
                                       t.ctypes.data_as(fp), int(len(t)), C.byref(loss),
                                       grad.ctypes.data_as(fp)))
    return float(loss.value), grad


def mps_lbm_set_allocator(alloc=None, free=None):
    """Register device allocator callbacks (Python callables or ctypes
    function pointers); both None restore hipMalloc / hipFree."""
    lib = load()
    if alloc is None and free is None:
        _check(lib.mps_lbm_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return
    a = alloc if isinstance(alloc, ALLOC_FN) else (ALLOC_FN(alloc) if alloc else ALLOC_FN())
    f = free if isinstance(free, FREE_FN) else (FREE_FN(free) if free else FREE_FN())
    _callbacks.extend([a, f])
    _check(lib.mps_lbm_set_allocator(a, f, None))


def use_torch_allocator():
    """Take the library's device memory from PyTorch's caching allocator,
    on the stream each handle runs on."""
    import torch

    def alloc(size, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(size), stream=int(stream or 0))
        except Exception:
            return None

    def free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    mps_lbm_set_allocator(alloc, free)


def mps_lbm_load_rank_model(h, weights):
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(load().mps_lbm_load_rank_model(h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))


def mps_lbm_get_rank_model(h) -> np.ndarray:
    w = np.empty(MLP_NPARAM, dtype=np.float32)
    _check(load().mps_lbm_get_rank_model(h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))
    return w


def mps_lbm_debug_raise_flags(h, nonfinite: int = 0, sweep_limit: int = 0):
    _check(load().mps_lbm_debug_raise_flags(h, int(nonfinite), int(sweep_limit)))


def mps_lbm_mlp_gradient_device(params_ptr, x_ptr, t_ptr, batch, loss_ptr, grad_ptr,
                                hip_stream=None):
    """The network's loss and gradient on device buffers (pointers as ints),
    enqueued on hip_stream without allocating."""
    _check(load().mps_lbm_mlp_gradient_device(
        C.c_void_p(params_ptr), C.c_void_p(x_ptr), C.c_void_p(t_ptr), int(batch),
        C.c_void_p(loss_ptr), C.c_void_p(grad_ptr), C.c_void_p(hip_stream or 0)))


def mps_lbm_step(h, nsteps: int = 1):
    _check(load().mps_lbm_step(h, int(nsteps)))


def mps_lbm_to_dense(h, what: int, N: int, q: int = D3Q19) -> np.ndarray:
    shape = {POPS: (q, N, N, N), RHO: (N, N, N), J: (3, N, N, N), VEL: (3, N, N, N)}[what]
    out = np.empty(shape, dtype=np.float64)
    _check(load().mps_lbm_to_dense(h, int(what), _dp(out), out.size))
    return out


def mps_lbm_observables(h) -> Obs:
    o = Obs()
    _check(load().mps_lbm_observables(h, C.byref(o)))
    return o


def mps_lbm_kernel_timing(h, kind: int):
    _check(load().mps_lbm_kernel_timing(h, int(kind)))


def mps_lbm_kernel_stats(h) -> KStats:
    k = KStats()
    _check(load().mps_lbm_kernel_stats(h, C.byref(k)))
    return k


def mps_lbm_init_batch(cfgs, rhos, us, solids=None, hip_stream: Optional[int] = None):
    """One handle advancing len(cfgs) domains together (see the C header)."""
    lib = load()
    cnt = len(cfgs)
    carr = (Config * cnt)(*cfgs)
    keep = []
    def darr(fields):
        out = (C.POINTER(C.c_double) * cnt)()
        for d, a in enumerate(fields):
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            out[d] = a.ctypes.data_as(C.POINTER(C.c_double))
        return out
    r, u = darr(rhos), darr(us)
    sarr = None
    if solids is not None:
        sarr = (C.POINTER(C.c_uint8) * cnt)()
        for d, m in enumerate(solids):
            if m is None:
                sarr[d] = None
            else:
                m = np.ascontiguousarray(m, dtype=np.uint8)
                keep.append(m)
                sarr[d] = m.ctypes.data_as(C.POINTER(C.c_uint8))
    h = C.c_void_p()
    _check(lib.mps_lbm_init_batch(carr, cnt, r, u, sarr, C.c_void_p(hip_stream or 0), C.byref(h)))
    return h


def mps_lbm_capture_step(h):
    _check(load().mps_lbm_capture_step(h))


def mps_lbm_domains(h) -> int:
    v = load().mps_lbm_domains(h)
    if v < 0:
        _check(v)
    return v


def mps_lbm_to_dense_domain(h, domain: int, what: int, N: int, q: int = D3Q19) -> np.ndarray:
    shape = {POPS: (q, N, N, N), RHO: (N, N, N), J: (3, N, N, N), VEL: (3, N, N, N)}[what]
    out = np.empty(shape, dtype=np.float64)
    _check(load().mps_lbm_to_dense_domain(h, int(domain), int(what), _dp(out), out.size))
    return out


def mps_lbm_observables_domain(h, domain: int) -> Obs:
    o = Obs()
    _check(load().mps_lbm_observables_domain(h, int(domain), C.byref(o)))
    return o


def mps_lbm_get_mps(h, which: int, n: int):
    """One MPS of the state as a list of FP64 cores [r_k][8][r_{k+1}]."""
    lib = load()
    bonds = (C.c_int * (n + 1))()
    _check(lib.mps_lbm_get_mps(h, int(which), None, 0, bonds))
    b = [int(bonds[k]) for k in range(n + 1)]
    sizes = [b[k] * 8 * b[k + 1] for k in range(n)]
    out = np.empty(sum(sizes), dtype=np.float64)
    _check(lib.mps_lbm_get_mps(h, int(which), _dp(out), out.size, bonds))
    cores, pos = [], 0
    for k in range(n):
        cores.append(out[pos:pos + sizes[k]].reshape(b[k], 8, b[k + 1]).copy())
        pos += sizes[k]
    return cores


def mps_lbm_destroy(h):
    if h:
        load().mps_lbm_destroy(h)


def config_from_case(case, precision=None, sweeps: int = 2, inv_mode: int = INV_TAYLOR2,
                     inv_iters: int = 2, seed: int = 2512, rank_predictor: int = 0,
                     rank_oversample: int = 16) -> Config:
    """Config from a workloads.Case."""
    c = mps_lbm_default_config()
    c.n = case.n
    c.lattice = int(getattr(case, "lattice", D3Q19))
    c.chi_max = int(case.chi)
    c.chi_mask_max = int(case.chi_mask or 0)
    c.tol = float(case.tol)
    c.tol_mask = float(case.tol_mask)
    c.tau = float(case.tau)
    for a in range(3):
        c.g[a] = float(case.g[a])
        c.axis_open[a] = int(case.axis_open[a])
    for face in range(6):
        c.face_bc[face] = int(case.face_bc[face])
        for a in range(3):
            c.face_val[face][a] = float(case.face_val[face][a])
    prec = precision or case.precision
    c.precision = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3}[prec]
    c.sweeps = sweeps
    c.inv_rho_mode = inv_mode
    c.inv_rho_iters = inv_iters
    c.seed = seed
    c.rank_predictor = rank_predictor
    c.rank_oversample = rank_oversample
    return c


class BatchSimulation:
    """Several domains (workloads.Case) advanced together by one handle;
    domains of equal n / chi / precision / tol share batched launches."""

    def __init__(self, cases, precision=None, hip_stream=None, **kw):
        self.cases = list(cases)
        cfgs = [config_from_case(c, precision, **kw) for c in self.cases]
        self.cfgs = cfgs
        self.h = mps_lbm_init_batch(cfgs, [c.rho0_field() for c in self.cases],
                                    [c.u0_field() for c in self.cases],
                                    [c.solid for c in self.cases], hip_stream=hip_stream)

    def step(self, n=1):
        mps_lbm_step(self.h, n)

    def dense(self, domain, what=POPS):
        return mps_lbm_to_dense_domain(self.h, domain, what, self.cases[domain].N,
                                       self.cfgs[domain].lattice)

    def observables(self, domain=0):
        return mps_lbm_observables_domain(self.h, domain)

    def domains(self):
        return mps_lbm_domains(self.h)

    def capture(self):
        mps_lbm_capture_step(self.h)

    def train_predictor(self, epochs: int, lr: float) -> float:
        return mps_lbm_train_rank_predictor(self.h, epochs, lr)

    def autotune(self) -> int:
        return mps_lbm_autotune(self.h)

    def predictor_info(self) -> PredictorInfo:
        return mps_lbm_rank_predictor_info(self.h)

    def kernel_timing(self, kind):
        mps_lbm_kernel_timing(self.h, kind)

    def kernel_stats(self):
        return mps_lbm_kernel_stats(self.h)

    def load_rank_model(self, weights):
        mps_lbm_load_rank_model(self.h, weights)

    def get_rank_model(self) -> np.ndarray:
        return mps_lbm_get_rank_model(self.h)

    def debug_raise_flags(self, nonfinite=0, sweep_limit=0):
        mps_lbm_debug_raise_flags(self.h, nonfinite, sweep_limit)

    def close(self):
        if self.h:
            mps_lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation:
    """Convenience wrapper owning one handle."""

    def __init__(self, case, precision=None, hip_stream=None, **kw):
        self.case = case
        self.cfg = config_from_case(case, precision, **kw)
        if case.mask_parts is not None:
            outer, inner = case.mask_parts
            self.h = mps_lbm_init_tensor_mask(self.cfg, outer, inner, rho=case.rho0_field(),
                                              u=case.u0_field(), hip_stream=hip_stream)
        else:
            self.h = mps_lbm_init_from_field(self.cfg, rho=case.rho0_field(),
                                             u=case.u0_field(), solid=case.solid,
                                             hip_stream=hip_stream)
        for face, (coef, dt) in (case.face_profile or {}).items():
            mps_lbm_set_face_profile(self.h, face, coef, dt)

    def set_face_profile(self, face, coef=None, dt=0.0):
        mps_lbm_set_face_profile(self.h, face, coef, dt)

    def set_region(self, lo, hi, rho_ref):
        mps_lbm_set_region(self.h, lo, hi, rho_ref)

    def kinetic_energy(self):
        return mps_lbm_kinetic_energy(self.h)

    def step(self, n=1):
        mps_lbm_step(self.h, n)

    def dense(self, what=POPS):
        return mps_lbm_to_dense(self.h, what, self.case.N, self.cfg.lattice)

    def observables(self):
        return mps_lbm_observables(self.h)

    def kernel_timing(self, kind):
        mps_lbm_kernel_timing(self.h, kind)

    def kernel_stats(self):
        return mps_lbm_kernel_stats(self.h)

    def mps(self, which):
        return mps_lbm_get_mps(self.h, which, self.case.n)

    def capture(self):
        mps_lbm_capture_step(self.h)

    def train_predictor(self, epochs: int, lr: float) -> float:
        return mps_lbm_train_rank_predictor(self.h, epochs, lr)

    def autotune(self) -> int:
        return mps_lbm_autotune(self.h)

    def predictor_info(self) -> PredictorInfo:
        return mps_lbm_rank_predictor_info(self.h)

    def load_rank_model(self, weights):
        mps_lbm_load_rank_model(self.h, weights)

    def get_rank_model(self) -> np.ndarray:
        return mps_lbm_get_rank_model(self.h)

    def debug_raise_flags(self, nonfinite=0, sweep_limit=0):
        mps_lbm_debug_raise_flags(self.h, nonfinite, sweep_limit)

    def close(self):
        if self.h:
            mps_lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

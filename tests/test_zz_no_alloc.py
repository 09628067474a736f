"""The allocation-free entry point (mps_lbm_mlp_gradient_device) against
the allocating one (mps_lbm_mlp_gradient) on the same inputs, through the C
ABI: two calls in a row, the second with a smaller batch."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2  # hipMemcpyHostToDevice, hipMemcpyDeviceToHost


def _hip():
    # the HIP runtime the library itself is linked against
    from paper_2512_07615_amd import mps_lbm as L
    L.load()
    return L, C.CDLL("libamdhip64.so.7")


class DevBuf:
    def __init__(self, hip, nbytes):
        self.hip = hip
        self.p = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.p), C.c_size_t(nbytes)) == 0
        self.nbytes = nbytes

    def put(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        assert a.nbytes <= self.nbytes
        assert self.hip.hipMemcpy(self.p, a.ctypes.data_as(C.c_void_p), C.c_size_t(a.nbytes),
                                  H2D) == 0

    def get(self, n):
        out = np.empty(n, dtype=np.float32)
        assert self.hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), self.p, C.c_size_t(out.nbytes),
                                  D2H) == 0
        return out

    def free(self):
        self.hip.hipFree(self.p)


def _inputs(L, rng, batch):
    from oracle import mlp as M
    p = np.zeros(L.MLP_NPARAM)
    off = 0
    for name, shape in M.SHAPES:
        n = int(np.prod(shape))
        p[off:off + n] = (rng.uniform(-1, 1, n) * np.sqrt(6.0 / shape[0]) if name.startswith("W")
                          else rng.uniform(-0.1, 0.1, n))
        off += n
    x = rng.uniform(-2, 0, (batch, L.MLP_IN))
    t = rng.normal(0, 0.5, batch)
    return p.astype(np.float32), x.astype(np.float32), t.astype(np.float32)


def test_gradient_without_allocation_matches_the_allocating_entry_point():
    L, hip = _hip()
    rng = np.random.default_rng(21)
    bufs = {k: DevBuf(hip, n) for k, n in (("p", 4 * L.MLP_NPARAM), ("x", 4 * 1024 * L.MLP_IN),
                                           ("t", 4 * 1024), ("loss", 64),
                                           ("g", 4 * L.MLP_NPARAM))}
    try:
        for batch in (700, 96):
            p, x, t = _inputs(L, rng, batch)
            print("no-alloc gradient, batch", batch, flush=True)
            loss_ref, grad_ref = L.mps_lbm_mlp_gradient(p, x, t)
            bufs["p"].put(p)
            bufs["x"].put(x)
            bufs["t"].put(t)
            bufs["g"].put(np.full(L.MLP_NPARAM, np.nan, dtype=np.float32))
            L.mps_lbm_mlp_gradient_device(bufs["p"].p.value, bufs["x"].p.value,
                                          bufs["t"].p.value, batch, bufs["loss"].p.value,
                                          bufs["g"].p.value)
            assert hip.hipDeviceSynchronize() == 0
            loss = float(bufs["loss"].get(1)[0])
            grad = bufs["g"].get(L.MLP_NPARAM)
            rg = float(np.linalg.norm(grad - grad_ref) / np.linalg.norm(grad_ref))
            print("batch", batch, "loss", loss, loss_ref, "gradient rel L2", rg, flush=True)
            # the same kernels on the same inputs in the same order
            assert np.isfinite(grad).all()
            assert abs(loss - loss_ref) <= 1e-6 * max(1.0, abs(loss_ref))
            assert rg < 1e-6
        with pytest.raises(L.MpsLbmError) as e:
            L.mps_lbm_mlp_gradient_device(bufs["p"].p.value, bufs["x"].p.value,
                                          bufs["t"].p.value, 1025, bufs["loss"].p.value,
                                          bufs["g"].p.value)
        assert e.value.code == L.EINVAL and "1024" in str(e.value)
    finally:
        for b in bufs.values():
            b.free()

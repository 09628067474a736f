"""GPU checks of the C ABI's boundary behaviour: the caller's allocator,
numerical-failure reporting and the predictor-weights transfer."""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as WL
from oracle.dense_lbm import DenseLBM

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lib():
    from paper_2512_07615_amd import mps_lbm as L
    L.load()
    return L


def _case():
    case = WL.case_channel(n=3, chi=64, tol=1e-13)
    rho, u = WL.random_flow_state(3, 3, amp=0.01)
    case.rho_init, case.u_init = rho, u
    return case


def test_allocator_without_memory_gives_enomem():
    """An allocator that has no memory makes initialisation fail with
    ENOMEM (and nothing else is left behind); resetting it restores
    hipMalloc."""
    L = lib()
    calls = []

    def none(size, stream, ctx):
        calls.append(size)
        return None

    L.mps_lbm_set_allocator(none, lambda p, s, c: None)
    try:
        with pytest.raises(L.MpsLbmError) as e:
            L.Simulation(_case(), precision="fp64")
        assert e.value.code == L.ENOMEM and len(calls) == 1
    finally:
        L.mps_lbm_set_allocator(None, None)
    s = L.Simulation(_case(), precision="fp64")
    s.step(1)
    s.close()


_TORCH_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import torch                      # first, so that one HIP runtime serves both
import numpy as np
import workloads as WL
from oracle.dense_lbm import DenseLBM
from paper_2512_07615_amd import mps_lbm as L
case = WL.case_channel(n=3, chi=64, tol=1e-13)
rho, u = WL.random_flow_state(3, 3, amp=0.01)
case.rho_init, case.u_init = rho, u
stream = torch.cuda.Stream()
base = torch.cuda.memory_allocated()
L.use_torch_allocator()
sim = L.Simulation(case, precision="fp64", hip_stream=stream.cuda_stream)
held = torch.cuda.memory_allocated() - base
sim.step(2)
got = sim.dense(L.POPS)
sim.close()
after = torch.cuda.memory_allocated() - base
L.mps_lbm_set_allocator(None, None)
d = DenseLBM(case)
d.step(); d.step()
err = float(np.abs(got - d.f).max() / np.abs(d.f).max())
print("torch allocator: held", held, "bytes; after destroy", after, "; rel vs dense", err, flush=True)
assert held > 1 << 20 and after == 0 and err < 1e-10
print("CHILD_OK", flush=True)
"""


def test_torch_caching_allocator_serves_the_handle():
    """With PyTorch's caching allocator registered, the handle's state and
    workspaces come from PyTorch's pool on the handle's stream (its
    allocated-bytes counter rises by the handle's footprint and returns to
    zero on destroy), and the step still matches the dense oracle.  Runs
    in a child process that imports torch first, so that the library binds
    to the same HIP runtime as torch."""
    r = subprocess.run([sys.executable, "-c", _TORCH_CHILD, ROOT], capture_output=True,
                       text=True, timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "CHILD_OK" in r.stdout


def test_numerical_failures_surface_as_enumeric():
    """Flags raised on the device (here by the testing hook, so that no
    kernel computes on invalid data) are returned as ENUMERIC by the next
    synchronising read: sweep-limit hits once, a non-finite value for good
    (reads and steps), while observables keep reporting the counts."""
    L = lib()
    s = L.Simulation(_case(), precision="fp64")
    s.step(1)
    ref = s.dense()
    s.debug_raise_flags(sweep_limit=2)
    with pytest.raises(L.MpsLbmError) as e:
        s.dense()
    assert e.value.code == L.ENUMERIC and "sweep limit" in str(e.value)
    assert np.array_equal(s.dense(), ref)  # reported once
    s.debug_raise_flags(nonfinite=1)
    for _ in range(2):
        with pytest.raises(L.MpsLbmError) as e:
            s.dense()
        assert e.value.code == L.ENUMERIC
    with pytest.raises(L.MpsLbmError) as e:
        s.step(1)
    assert e.value.code == L.ENUMERIC
    o = s.observables()
    assert o.nonfinite >= 1 and o.svd_failures >= 2 and o.step == 1
    s.close()


def test_rank_model_weights_round_trip():
    """Predictor weights read out of one handle load into another, which
    then counts as trained and returns the same weights."""
    L = lib()
    case = WL.case_channel(n=4, chi=16, tol=1e-6)
    a = L.Simulation(case, precision="fp32", rank_predictor=2)
    b = L.Simulation(case, precision="fp32", rank_predictor=2, seed=99)
    wa, wb = a.get_rank_model(), b.get_rank_model()
    assert wa.shape == (L.MLP_NPARAM,) and not np.array_equal(wa, wb)
    assert b.predictor_info().trained == 0
    b.load_rank_model(wa)
    assert np.array_equal(b.get_rank_model(), wa)
    assert b.predictor_info().trained == 1
    a.step(1)
    b.step(1)
    off = L.Simulation(case, precision="fp32")
    with pytest.raises(L.MpsLbmError) as e:
        off.load_rank_model(wa)
    assert e.value.code == L.EUNSUPPORTED
    for s in (a, b, off):
        s.close()

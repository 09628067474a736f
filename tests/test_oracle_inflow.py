"""Pins for the time-dependent velocity inlet (Section 4.1 inflow profiles)
and the pressure metric Delta p / p_0 (Section 4.2)."""
import dataclasses

import numpy as np
import pytest

import workloads as WL
from oracle import mps as M
from oracle.dense_lbm import DenseLBM
from oracle.inflow import inflow_scale
from oracle.metrics import pressure_drop
from oracle.mps_lbm import MPSLBM

RAMP = (0.0, 1.0, 1.5, 0.0, 0.0, 0.0)        # u_0 (1 - exp(-1.5 t))
PULSE = (0.1, 0.0, 0.0, 18.0, 1.5, 10.0)     # 0.1 + 18 t^1.5 exp(-10 t)


def test_pulse_spans_the_velocity_range_the_paper_states():
    # Section 4.1: inflow velocities between 0.1 and 0.34 m/s over the
    # simulated part of the cycle (0 <= t <= 0.25 s)
    t = np.linspace(0.0, 0.25, 25001)
    v = np.array([inflow_scale(PULSE, x) for x in t])
    assert v[0] == 0.1 and v.min() == 0.1
    assert 0.33 < v.max() < 0.345
    # d/dt t^a e^(-b t) = 0 at t = a / b
    assert t[v.argmax()] == pytest.approx(1.5 / 10.0, abs=1e-4)


def test_ramp_closed_forms():
    assert inflow_scale(RAMP, 0.0) == 0.0
    assert inflow_scale(RAMP, 1.0 / 1.5) == pytest.approx(1.0 - np.exp(-1.0), rel=1e-15)
    v = [inflow_scale(RAMP, x) for x in np.linspace(0, 20, 201)]
    assert np.all(np.diff(v) > 0) and abs(v[-1] - 1.0) < 1e-12
    # a constant profile is the constant face
    assert inflow_scale((1.0, 0, 0, 0, 0, 0), 3.7) == 1.0


def _closed_duct(n, ub, profile, solid=None):
    """x open: velocity inlet (profiled) on x = 0, a resting velocity face
    (bounce-back wall) on x = N-1; y, z periodic; a seeded flow inside."""
    N = 1 << n
    rho, u = WL.random_flow_state(n, 11, amp=0.01)
    return WL.Case(name="closed_duct", n=n, tau=0.7, chi=10 ** 6, tol=1e-14,
                   solid=solid, axis_open=(1, 0, 0),
                   face_bc=(WL.BC_VELOCITY, WL.BC_VELOCITY, 0, 0, 0, 0),
                   face_val=((ub, 0.0, 0.0), (0.0, 0.0, 0.0)) + ((0, 0, 0),) * 4,
                   rho_init=rho, u_init=u, face_profile={0: (profile, 0.05)})


@pytest.mark.parametrize("oracle", ["dense", "mps"])
def test_inlet_adds_rho0_ub_per_face_cell_every_step(oracle):
    """Every population entering through a velocity face is the leaving one
    plus 6 w_i rho_0 c_i.u_b, and 6 sum_(entering i) w_i c_ix = 1 for D3Q19,
    so a step changes the mass by exactly N_face rho_0 u_b(t_k) through the
    inlet, whatever the state; the resting far face adds nothing.  With the
    ramp, the k-th step (t_k = k dt) adds rho_0 u_b (1 - exp(-1.5 k dt))."""
    n, ub = 3, 0.03
    case = _closed_duct(n, ub, RAMP)
    sim = DenseLBM(case) if oracle == "dense" else MPSLBM(case)
    N = 1 << n
    mass = lambda: float(sim.f.sum()) if oracle == "dense" else sim.mass()
    m0 = mass()
    for k in range(5):
        rho0 = m0 / N ** 3
        sim.step()
        m1 = mass()
        expect = N * N * rho0 * ub * (1.0 - np.exp(-1.5 * k * 0.05))
        # (the MPS oracle rounds at tol 1e-14 of a norm of about 30: 1e-12)
        assert m1 - m0 == pytest.approx(expect, rel=1e-9,
                                        abs=1e-13 if oracle == "dense" else 5e-12)
        m0 = m1


def test_profiled_face_equals_a_sequence_of_constant_faces():
    n, ub = 3, 0.04
    case = _closed_duct(n, ub, PULSE)
    a = DenseLBM(case)
    const = dataclasses.replace(case, face_profile=None)
    b = DenseLBM(const)
    for k in range(4):
        s = inflow_scale(PULSE, k * 0.05)
        b.case = dataclasses.replace(const, face_val=((s * ub, 0.0, 0.0),) + const.face_val[1:])
        a.step()
        b.step()
    assert np.abs(a.f - b.f).max() == 0.0


def test_untruncated_mps_with_a_profiled_inlet_equals_dense():
    case = WL.case_vascular(n=4, chi=64, tau=0.6, u_in=0.03, tol=1e-13, precision="fp64")
    rho, u = WL.random_flow_state(4, 5, amp=0.01)
    case.rho_init, case.u_init = rho, u
    case.face_profile = {0: (RAMP, 0.2)}
    m = MPSLBM(case)
    d = DenseLBM(case)
    for _ in range(3):
        m.step()
        d.step()
    assert np.abs(m.dense_populations() - d.f).max() < 1e-11


def test_pressure_drop_closed_forms():
    rng = np.random.default_rng(4)
    N = 16
    solid = (rng.uniform(size=(N, N, N)) < 0.3).astype(np.uint8)
    lo, hi = (2, 3, 1), (9, 14, 7)
    # uniform density (1 + delta) rho_ref: Delta p / p_0 = delta
    rho = np.full((N, N, N), 1.004 * 1.02)
    assert pressure_drop(rho, solid, lo, hi, 1.02) == pytest.approx(0.004, rel=1e-12)
    # whatever the solid cells hold, they do not count
    rho2 = rho.copy()
    rho2[solid.astype(bool)] = 7.0
    assert pressure_drop(rho2, solid, lo, hi, 1.02) == pytest.approx(0.004, rel=1e-12)
    # a density linear in x, no solid: the mean over the box is the value at
    # the mean x of its cells, (lo + hi - 1) / 2
    x = np.arange(N, dtype=float)[:, None, None] * np.ones((1, N, N))
    rho3 = 1.0 + 1e-3 * x
    xm = (lo[0] + hi[0] - 1) / 2.0
    assert pressure_drop(rho3, None, lo, hi, 1.0) == pytest.approx(1e-3 * xm, rel=1e-12)
    with pytest.raises(ValueError):
        pressure_drop(rho, np.ones((N, N, N), np.uint8), lo, hi, 1.0)


def test_mps_oracle_pressure_drop_follows_the_dense_lbm():
    case = WL.case_pinfin(n=4, l=2, chi=64, tau=0.6, u_in=0.03, tol=1e-12, precision="fp64")
    m = MPSLBM(case)
    d = DenseLBM(case)
    for _ in range(3):
        m.step()
        d.step()
    lo, hi = (0, 0, 0), (2, 8, 8)
    got = m.pressure_drop(lo, hi, 1.0)
    ref = pressure_drop(d.f.sum(axis=0), case.solid, lo, hi, 1.0)
    assert got != 0.0
    assert abs(got - ref) < 1e-3 * abs(ref) + 1e-12

"""Pins for the D3Q15 velocity set (the paper's 3D lattice, Section 4.1), the
Taylor-Green vortex initial state and the kinetic-energy metrics
(Section 4.2)."""
import numpy as np
import pytest

import workloads as WL
from oracle import mps as M
from oracle.dense_lbm import DenseLBM, equilibrium, moments
from oracle.lattice import CS2, D3Q15, D3Q19, PI_PAIRS
from oracle.metrics import dissipation, kinetic_energy
from oracle.mps_lbm import MPSLBM


@pytest.mark.parametrize("lat", [D3Q15, D3Q19], ids=["d3q15", "d3q19"])
def test_lattice_identities(lat):
    C, W, OPP = lat.c, lat.w, lat.opp
    assert len(set(map(tuple, C))) == lat.q and W.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(W @ C, 0.0, atol=1e-16)
    second = np.einsum("i,ia,ib->ab", W, C, C)
    assert np.allclose(second, CS2 * np.eye(3), atol=1e-15)
    third = np.einsum("i,ia,ib,ic->abc", W, C, C, C)
    assert np.allclose(third, 0.0, atol=1e-16)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", W, C, C, C, C)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(fourth, iso, atol=1e-15)
    for i in range(lat.q):
        assert np.array_equal(C[OPP[i]], -C[i])
    # D3Q15: the corners are the eight sign patterns of (1, 1, 1)
    if lat.q == 15:
        assert sorted(map(tuple, np.abs(C[7:]))) == [(1, 1, 1)] * 8


def test_d3q15_equilibrium_moments():
    rng = np.random.default_rng(1)
    shape = (4, 4, 4)
    rho = 1.0 + 0.05 * rng.standard_normal(shape)
    u = 0.05 * rng.standard_normal((3,) + shape)
    j = rho * u
    Pi = {(a, b): j[a] * u[b] for (a, b) in PI_PAIRS}
    feq = equilibrium(rho, j, Pi, D3Q15)
    r2, j2 = moments(feq)
    assert np.allclose(r2, rho, atol=1e-14) and np.allclose(j2, j, atol=1e-14)
    # second moment: rho c_s^2 delta + rho u u
    P = np.einsum("ia,ib,ixyz->abxyz", D3Q15.c.astype(float), D3Q15.c.astype(float), feq)
    for a in range(3):
        for b in range(3):
            ref = rho * u[a] * u[b] + (CS2 * rho if a == b else 0.0)
            assert np.allclose(P[a, b], ref, atol=1e-14)


def test_tgv_initial_state():
    n, U = 4, 0.1
    rho, u = WL.tgv_state(n, U)
    case = WL.case_tgv(n=n, re=100.0)
    d = DenseLBM(case)
    # mean of sin^2 x cos^2 y cos^2 z on the grid is 1/8: E_kin(0) = U^2 / 8
    assert kinetic_energy(d.f) == pytest.approx(U * U / 8.0, rel=1e-12)
    assert rho.mean() == pytest.approx(1.0, abs=1e-15)
    # spectral divergence of the initial velocity vanishes
    N = 1 << n
    k = np.fft.fftfreq(N, d=1.0 / N)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    div = KX * np.fft.fftn(u[0]) + KY * np.fft.fftn(u[1]) + KZ * np.fft.fftn(u[2])
    assert np.abs(div).max() < 1e-10
    # Re = U N / (2 pi nu) with nu = (tau - 1/2) / 3
    assert U * N / (2 * np.pi * (case.tau - 0.5) / 3.0) == pytest.approx(100.0, rel=1e-12)


def _decay_deviation(n, lattice):
    """Relative deviation of E_kin(t) / E_kin(0) from exp(-2 nu |k|^2 t) of
    the linear (Stokes) Taylor-Green mode, |k|^2 = 3 (2 pi / N)^2, after
    the time in which the closed form falls to exp(-1.41)."""
    N = 1 << n
    U = 0.001                   # linear regime
    nu = 0.0509                 # tau = 0.653
    case = WL.case_tgv(n=n, re=U * N / (2 * np.pi * nu), u_lat=U, lattice=lattice,
                       precision="fp64")
    d = DenseLBM(case)
    e0 = kinetic_energy(d.f)
    k2 = 3 * (2 * np.pi / N) ** 2
    steps = int(round(1.41 / (2 * nu * k2)))
    for _ in range(steps):
        d.step()
    return kinetic_energy(d.f) / e0 / np.exp(-2 * nu * k2 * steps) - 1.0


@pytest.mark.parametrize("lattice", [15, 19])
def test_tgv_linear_decay_converges_to_the_viscous_closed_form(lattice):
    """The Stokes limit of the vortex decays as exp(-2 nu |k|^2 t) with
    nu = c_s^2 (tau - 1/2); the lattice Boltzmann error is second order in
    the grid spacing, so doubling N cuts the deviation about fourfold
    (measured: D3Q15 -5.6 % -> -1.4 %, D3Q19 -11.7 % -> -3.0 %)."""
    d16 = _decay_deviation(4, lattice)
    d32 = _decay_deviation(5, lattice)
    assert abs(d32) < 0.05
    assert 3.0 < d16 / d32 < 5.0


def test_dissipation_is_second_order():
    a = 0.7
    for dt, tol in ((0.01, 2e-4), (0.005, 5e-5)):
        t = np.arange(0.0, 2.0 + dt / 2, dt)
        e = np.exp(-a * t)
        err = np.abs(dissipation(e, dt) - a * np.exp(-a * t)).max()
        assert err < tol


@pytest.mark.parametrize("which", ["tgv", "porous"])
def test_untruncated_mps_d3q15_equals_dense(which):
    if which == "tgv":
        case = WL.case_tgv(n=3, chi=64, re=50.0, tol=1e-14, precision="fp64")
    else:
        case = WL.case_porous(n=4, chi=64, tau=0.6, tol=1e-13, precision="fp64")
        case.lattice = 15
        rho, u = WL.random_flow_state(4, 5, amp=0.01)
        case.rho_init, case.u_init = rho, u
    m = MPSLBM(case)
    d = DenseLBM(case)
    assert len(m.f) == 15 and d.f.shape[0] == 15
    for _ in range(3):
        m.step()
        d.step()
    assert np.abs(m.dense_populations() - d.f).max() < 1e-11


@pytest.mark.parametrize("oracle", ["dense", "mps"])
def test_d3q15_velocity_inlet_pressure_outlet_keep_a_uniform_equilibrium(oracle):
    """As for D3Q19: the face terms are exact at equilibrium, so a uniform
    flow (rho_b, u_b) with a velocity inlet and a pressure outlet at rho_b
    is a fixed point; the corner velocities exercise every cross term."""
    n, N, rho_b = 3, 8, 1.02
    u = np.array([0.05, 0.02, -0.03])
    case = WL.Case(name="uniform_duct15", n=n, tau=0.7, chi=10 ** 6, tol=1e-14,
                   axis_open=(1, 0, 0), face_bc=(WL.BC_VELOCITY, WL.BC_PRESSURE, 0, 0, 0, 0),
                   face_val=(tuple(u), (rho_b, 0, 0)) + ((0, 0, 0),) * 4,
                   rho_init=np.full((N,) * 3, rho_b),
                   u_init=np.broadcast_to(u[:, None, None, None], (3, N, N, N)).copy(),
                   lattice=15)
    sim = DenseLBM(case) if oracle == "dense" else MPSLBM(case)
    ref = np.empty((15, N, N, N))
    for i in range(15):
        cu = float(D3Q15.c[i] @ u)
        ref[i] = D3Q15.w[i] * rho_b * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * float(u @ u))
    for _ in range(2):
        sim.step()
    f = sim.f if oracle == "dense" else sim.dense_populations()
    assert np.abs(f - ref).max() < 1e-13


def test_d3q15_dense_mass_conservation_with_obstacles():
    case = WL.case_porous(n=4, chi=64, tau=0.6, tol=1e-13, precision="fp64")
    case.lattice = 15
    case.axis_open = (0, 0, 0)
    case.face_bc = (0,) * 6
    rho, u = WL.random_flow_state(4, 6, amp=0.02)
    case.rho_init, case.u_init = rho, u
    d = DenseLBM(case)
    m0 = d.f.sum()
    for _ in range(50):
        d.step()
    assert abs(d.f.sum() - m0) < 1e-11 * m0
    assert np.abs(d.f[:, case.solid.astype(bool)]).max() == 0.0

"""Pins for the dense D3Q19 oracle and the CPU MPS-LBM step: lattice
identities, equilibrium moments, the inverse-density closed forms, mass
conservation, the obstacle rule, a Poiseuille closed form, and untruncated
MPS-LBM == dense LBM."""
import numpy as np
import pytest

import workloads as WL
from oracle import mps as M
from oracle.dense_lbm import (DenseLBM, equilibrium, inverse_density, INV_EXACT,
                              INV_TAYLOR2, INV_NEWTON)
from oracle.lattice import C, W, OPP, Q, CS2, PI_PAIRS
from oracle.mps_lbm import MPSLBM


def test_d3q19_lattice_identities():
    assert Q == 19 and len(set(map(tuple, C))) == 19
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(W @ C, 0.0)
    second = np.einsum("i,ia,ib->ab", W, C, C)
    assert np.allclose(second, CS2 * np.eye(3), atol=1e-15)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", W, C, C, C, C)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(fourth, iso, atol=1e-15)
    for i in range(Q):
        assert np.array_equal(C[OPP[i]], -C[i])


def test_equilibrium_moments_and_literal_form():
    rng = np.random.default_rng(0)
    shape = (4, 4, 4)
    rho = 1.0 + 0.05 * rng.standard_normal(shape)
    u = 0.05 * rng.standard_normal((3,) + shape)
    j = rho * u
    Pi = {(a, b): j[a] * u[b] for (a, b) in PI_PAIRS}
    feq = equilibrium(rho, j, Pi)
    assert np.allclose(feq.sum(0), rho, rtol=0, atol=1e-14)
    assert np.allclose(np.einsum("ia,ixyz->axyz", C.astype(float), feq), j, atol=1e-14)
    # the equilibrium equation as printed: w rho (1 + cu/cs2 + (cu)^2/2cs4 - uu/2cs2)
    for i in range(Q):
        cu = np.einsum("a,axyz->xyz", C[i].astype(float), u)
        lit = W[i] * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2)
                            - (u ** 2).sum(0) / (2 * CS2))
        assert np.allclose(feq[i], lit, atol=1e-15)


def test_inverse_density_closed_forms():
    rho0 = 1.1
    e = np.linspace(-0.3, 0.3, 41)
    rho = rho0 * (1 + e)
    r2 = inverse_density(rho, rho0, INV_TAYLOR2)
    # |1/rho - r_T2| = |e|^3 / (rho0 |1+e|)
    assert np.allclose(np.abs(1 / rho - r2), np.abs(e) ** 3 / (rho0 * np.abs(1 + e)),
                       rtol=1e-9, atol=1e-15)
    # k Newton-Schulz steps from 1/rho0 = Taylor order 2^k - 1
    for k in (1, 2, 3):
        y = inverse_density(rho, rho0, INV_NEWTON, iters=k)
        order = 2 ** k - 1
        taylor = sum((-e) ** p for p in range(order + 1)) / rho0
        assert np.allclose(y, taylor, rtol=1e-13)


def _obstacle_case(n=4, seed=7):
    case = WL.case_channel(n=n, chi=10 ** 6, tol=0.0)
    N = 1 << n
    rng = np.random.default_rng(seed)
    solid = case.solid.copy()
    for _ in range(3):
        c = rng.integers(2, N - 2, size=3)
        solid[c[0] - 1:c[0] + 1, c[1] - 1:c[1] + 1, c[2] - 1:c[2] + 1] = 1
    case.solid = solid
    rho, u = WL.random_flow_state(n, seed, amp=0.03)
    case.rho_init, case.u_init = rho, u
    return case


def test_dense_mass_conservation_and_solid_zero():
    case = _obstacle_case()
    d = DenseLBM(case)
    m0 = d.f.sum()
    for _ in range(300):
        d.step()
    assert abs(d.f.sum() - m0) / m0 < 1e-12
    assert np.all(d.f[:, case.solid.astype(bool)] == 0.0)


def test_dense_obstacle_rule_is_halfway_bounce_back():
    """(1 - m) f_i + S(c_i)(m f_ihat) after streaming equals the textbook
    halfway bounce-back f_i(x_f, t+1) = f*_ihat(x_f, t) at fluid cells next
    to a wall."""
    case = _obstacle_case(n=3, seed=1)
    d = DenseLBM(case)
    fpost, _ = d.collide(d.f)
    d.step()
    solid = case.solid.astype(bool)
    N = 8
    for i in range(1, Q):
        c = C[i]
        for x in np.argwhere(~solid):
            src = (x - c) % N
            if solid[tuple(src)]:
                assert d.f[i][tuple(x)] == pytest.approx(fpost[OPP[i]][tuple(x)], abs=1e-15)
            else:
                assert d.f[i][tuple(x)] == pytest.approx(fpost[i][tuple(src)], abs=1e-15)


@pytest.mark.slow
def test_poiseuille_closed_form():
    """Body-force driven channel (D3Q19 BGK + the obstacle bounce-back +
    Shan-Chen forcing): the steady bare momentum is
    j_x(y) = g/(2 nu) (y - 1/2)(H + 1/2 - y) + g (16 tau^2 - 20 tau + 3)/(24 nu)
    with fluid rows y = 1..H (closed form derived for this scheme, not printed
    in the paper); nu = (tau - 1/2)/3."""
    tau, g, ny = 0.8, 1e-6, 32
    H = ny - 2
    shape = (2, ny, 2)
    solid = np.zeros(shape, dtype=np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    case = WL.Case(name="poiseuille", n=1, tau=tau, chi=1, tol=0.0, g=(g, 0.0, 0.0),
                   solid=solid, rho_init=np.ones(shape), u_init=np.zeros((3,) + shape))
    d = DenseLBM(case, inv_mode=INV_EXACT, shape=shape)
    for _ in range(12000):
        d.step()
    nu = (tau - 0.5) / 3.0
    y = np.arange(1, H + 1, dtype=float)
    jx_ref = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y) + g * (16 * tau ** 2 - 20 * tau + 3) / (24 * nu)
    jx = d.j()[0][0, 1:H + 1, 0]
    l2 = np.linalg.norm(jx - jx_ref) / np.linalg.norm(jx_ref)
    assert l2 < 1e-3
    assert l2 < 1e-5  # the closed form is exact for this scheme up to convergence


@pytest.mark.parametrize("which", ["channel8", "porous16", "vascular16"])
def test_untruncated_mps_equals_dense(which):
    if which == "channel8":
        case = _obstacle_case(n=3, seed=2)
    elif which == "porous16":
        case = WL.case_porous(n=4, chi=10 ** 6, tol=1e-14)
    else:
        case = WL.case_vascular(n=4, chi=10 ** 6, tol=1e-14)
    if case.rho_init is None:
        rho, u = WL.random_flow_state(case.n, 3, amp=0.01)
        case.rho_init, case.u_init = rho, u
    d = DenseLBM(case)
    m = MPSLBM(case)
    for _ in range(2):
        d.step()
        m.step()
    fm = m.dense_populations()
    assert np.abs(fm - d.f).max() / np.abs(d.f).max() < 1e-11


def test_untruncated_mps_newton_inverse_equals_dense():
    case = _obstacle_case(n=3, seed=4)
    d = DenseLBM(case, inv_mode=INV_NEWTON, inv_iters=2)
    m = MPSLBM(case, inv_mode="newton", inv_iters=2)
    d.step()
    m.step()
    assert np.abs(m.dense_populations() - d.f).max() / np.abs(d.f).max() < 1e-11


@pytest.mark.slow
def test_channel16_chi16_200_steps_vs_dense_and_mass():
    """The 16^3 channel at chi = 16, tol 1e-10, 200 steps: the MPS oracle
    follows the dense oracle and conserves mass."""
    case = WL.case_channel()
    d = DenseLBM(case)
    m = MPSLBM(case)
    mass0 = m.mass()
    for _ in range(200):
        d.step()
        m.step()
    fm = m.dense_populations()
    assert np.abs(fm - d.f).max() / np.abs(d.f).max() < 1e-9
    assert abs(m.mass() - mass0) / mass0 < 1e-12
    # the flow develops in x: momentum equals the injected tau * F per step
    assert m.momentum()[0] > 0


def _duct(shape, face_bc, face_val, walls):
    solid = np.zeros(shape, dtype=np.uint8)
    if walls:
        solid[:, 0, :] = 1
        solid[:, -1, :] = 1
    return WL.Case(name="duct", n=1, tau=0.8, chi=1, tol=0.0, solid=solid,
                   axis_open=(1, 0, 0), face_bc=face_bc, face_val=face_val,
                   rho_init=np.ones(shape), u_init=np.zeros((3,) + shape))


@pytest.mark.slow
def test_velocity_inlet_sign_plug_flow():
    """Velocity inlet (Ladd sign: + 2 w rho_b c.u_b / c_s^2 for populations
    entering the fluid) with a pressure outlet, no walls: the steady state is
    plug flow with u_x = u_b, so the mass flux through every cross-section
    is rho_0 u_b per unit area."""
    ub = 0.02
    shape = (16, 2, 2)
    case = _duct(shape, (WL.BC_VELOCITY, WL.BC_PRESSURE, 0, 0, 0, 0),
                 ((ub, 0, 0), (1.0, 0, 0)) + ((0, 0, 0),) * 4, walls=False)
    d = DenseLBM(case, inv_mode=INV_EXACT, shape=shape)
    for _ in range(6000):
        mac = d.step()
    jx = d.j()[0]
    # steady mass flux rho_0 u_b through every cross-section (a wrong sign
    # would drive it to -rho_0 u_b)
    assert np.allclose(jx, mac["rho0"] * ub, rtol=1e-3)
    assert np.abs(d.j()[1]).max() < 1e-10 and np.abs(d.j()[2]).max() < 1e-10


@pytest.mark.slow
def test_pressure_faces_drive_flow_down_the_gradient():
    """Pressure faces (anti-bounce-back) on both ends of a walled duct: the
    density near each face approaches its rho_b and the flow runs from high
    to low pressure."""
    shape = (32, 10, 2)
    case = _duct(shape, (WL.BC_PRESSURE, WL.BC_PRESSURE, 0, 0, 0, 0),
                 ((1.001, 0, 0), (0.999, 0, 0)) + ((0, 0, 0),) * 4, walls=True)
    d = DenseLBM(case, inv_mode=INV_EXACT, shape=shape)
    for _ in range(4000):
        d.step()
    rho = d.rho()[:, 1:-1, :]
    assert rho[0].mean() == pytest.approx(1.001, abs=2e-4)
    assert rho[-1].mean() == pytest.approx(0.999, abs=2e-4)
    prof = rho.mean(axis=(1, 2))
    assert np.all(np.diff(prof) < 0)
    assert d.j()[0][:, 1:-1, :].min() > 0


def _uniform_duct(face_bc, face_val, u):
    """An 8^3 duct open in x, periodic in y and z, no solid, holding the
    uniform state (rho_b, u) everywhere."""
    n = 3
    N = 1 << n
    rho_b = 1.02
    return WL.Case(name="uniform_duct", n=n, tau=0.7, chi=10 ** 6, tol=1e-14,
                   axis_open=(1, 0, 0), face_bc=face_bc, face_val=face_val,
                   rho_init=np.full((N,) * 3, rho_b),
                   u_init=np.broadcast_to(np.asarray(u, float)[:, None, None, None],
                                          (3, N, N, N)).copy()), rho_b


def _feq_uniform(rho, u, shape):
    out = np.empty((Q,) + shape)
    uu = float(np.dot(u, u))
    for i in range(Q):
        cu = float(C[i] @ u)
        out[i] = W[i] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
    return out


@pytest.mark.parametrize("oracle", ["dense", "mps"])
def test_pressure_faces_keep_a_uniform_equilibrium(oracle):
    """The pressure face term -f_ihat + 2 w_i rho_b (1 + 4.5 (c_i.u)^2 - 1.5
    u.u) is exact at equilibrium: with f_ihat = f_eq,ihat(rho_b, u) it gives
    f_eq,i(rho_b, u), since the odd terms of f_i + f_ihat cancel.  So a
    uniform flow (rho_b, u) with pressure faces at rho_b on both ends is a
    fixed point of the step.  u has three nonzero components, so every
    coefficient (4.5, 1.5 and the cross terms 9 c_a c_b u_a u_b) is
    exercised; a wrong one moves the face planes by O(u^2)."""
    u = np.array([0.06, -0.04, 0.03])
    case, rho_b = _uniform_duct((WL.BC_PRESSURE, WL.BC_PRESSURE, 0, 0, 0, 0),
                                ((1.02, 0, 0), (1.02, 0, 0)) + ((0, 0, 0),) * 4, u)
    sim = DenseLBM(case) if oracle == "dense" else MPSLBM(case)
    ref = _feq_uniform(rho_b, u, (case.N,) * 3)
    for _ in range(2):
        sim.step()
    f = sim.f if oracle == "dense" else sim.dense_populations()
    assert np.abs(f - ref).max() < 1e-13
    # a perturbed coefficient would not keep it: the face term's quadratic
    # part is not negligible at this velocity
    assert 4.5 * 0.1 ** 2 * W[7] * rho_b > 1e-5


@pytest.mark.parametrize("oracle", ["dense", "mps"])
def test_velocity_face_keeps_a_uniform_equilibrium(oracle):
    """The velocity face term f_ihat + 6 w_i rho_0 c_i.u_b is exact at
    equilibrium: with f_ihat = f_eq,ihat(rho_0, u_b) it gives
    f_eq,i(rho_0, u_b).  A uniform flow at u_b with a velocity inlet and a
    pressure outlet at rho_b = rho_0 is therefore a fixed point."""
    u = np.array([0.05, 0.02, -0.03])
    case, rho_b = _uniform_duct((WL.BC_VELOCITY, WL.BC_PRESSURE, 0, 0, 0, 0),
                                (tuple(u), (1.02, 0, 0)) + ((0, 0, 0),) * 4, u)
    sim = DenseLBM(case) if oracle == "dense" else MPSLBM(case)
    ref = _feq_uniform(rho_b, u, (case.N,) * 3)
    for _ in range(2):
        sim.step()
    f = sim.f if oracle == "dense" else sim.dense_populations()
    assert np.abs(f - ref).max() < 1e-13


def test_obstacle_mask_is_machine_precision_and_products_keep_population_bonds():
    """The obstacle mask is decomposed to machine precision (Section 5.2:
    the mask bond dimension is the one that represents it exactly), so its
    rank may exceed chi; the obstacle products take the population as the
    candidate, so every population keeps bonds <= chi.  An explicit cap
    (case.chi_mask) still applies when given."""
    case = WL.case_porous(n=4, chi=8, tol=1e-6)
    rho, u = WL.random_flow_state(4, 3, amp=0.01)
    case.rho_init, case.u_init = rho, u
    m = MPSLBM(case)
    dense = M.to_dense(m.mask)
    assert np.abs(dense - case.solid).max() < 1e-12
    assert max(M.bonds(m.mask)) > case.chi
    assert m.n_fluid == pytest.approx(float((case.solid == 0).sum()), abs=1e-8)
    m.step()
    assert all(max(b) <= case.chi for b in m.bond_dims())
    capped = WL.case_porous(n=4, chi=8, tol=1e-6, chi_mask=4)
    assert max(M.bonds(MPSLBM(capped).mask)) <= 4


def test_face_masks_are_the_fluid_cells_of_the_face_planes():
    """m_B of an open face is the indicator of the fluid cells of the face
    plane, decomposed from that definition (exact to tol_mask)."""
    case = WL.case_vascular(n=4, chi=64, tol=1e-12)
    m = MPSLBM(case)
    N = case.N
    for face, mps in m.fluid_plane.items():
        ax, side = divmod(face, 2)
        ref = np.zeros((N,) * 3)
        sl = [slice(None)] * 3
        sl[ax] = 0 if side == 0 else N - 1
        ref[tuple(sl)] = 1.0 - case.solid[tuple(sl)]
        assert np.abs(M.to_dense(mps) - ref).max() < 1e-12

"""Pins for the zip-up product, the alternative to the variational product
that Section 2.3 names, and for the right-canonical form it starts from."""
import numpy as np
import pytest

import workloads as WL
from oracle import mps as M
from oracle.mps_lbm import MPSLBM


def _rand_mps(rng, n, bonds):
    b = [1] + list(bonds) + [1]
    return [rng.standard_normal((b[k], 8, b[k + 1])) for k in range(n)]


def test_right_canonical_form():
    rng = np.random.default_rng(1)
    a = _rand_mps(rng, 4, [5, 9, 3])
    r = M.right_canonical(a)
    assert np.allclose(M.to_dense(r), M.to_dense(a), atol=1e-12 * np.abs(M.to_dense(a)).max())
    for k in range(1, 4):
        x = r[k].reshape(r[k].shape[0], -1)
        assert np.allclose(x @ x.T, np.eye(x.shape[0]), atol=1e-12)


def test_zipup_is_exact_when_nothing_is_cut():
    # chi above every bond of the exact product and tol 0: the dense Hadamard
    # product, with left-orthonormal cores 1..n-1
    rng = np.random.default_rng(2)
    a = _rand_mps(rng, 4, [3, 4, 2])
    b = _rand_mps(rng, 4, [2, 5, 3])
    z = M.hadamard_zipup(a, b, 1 << 20, 0.0)
    ex = M.to_dense(a) * M.to_dense(b)
    assert np.allclose(M.to_dense(z), ex, rtol=0, atol=1e-11 * np.abs(ex).max())
    for k in range(3):
        x = z[k].reshape(-1, z[k].shape[2])
        assert np.allclose(x.T @ x, np.eye(x.shape[1]), atol=1e-12)
    # the opposite operand order is the same field
    z2 = M.hadamard_zipup(b, a, 1 << 20, 0.0)
    assert np.allclose(M.to_dense(z2), ex, rtol=0, atol=1e-11 * np.abs(ex).max())


def test_zipup_with_the_unit_field_is_the_optimal_truncation():
    # with b = 1 the carried factor meets a's own right-orthonormal part, so
    # the cut is the SVD of a's unfolding: Eckart-Young on a two-site a
    rng = np.random.default_rng(3)
    a = _rand_mps(rng, 2, [8])
    one = M.ones(2)
    ex = M.to_dense(a)
    sv = np.linalg.svd(M.scale_order(ex, 2).reshape(8, 8), compute_uv=False)
    for chi in (2, 4, 6):
        z = M.hadamard_zipup(a, one, chi, 0.0)
        err2 = float(((M.to_dense(z) - ex) ** 2).sum())
        assert err2 == pytest.approx(float((sv[chi:] ** 2).sum()), rel=1e-9)
        assert M.bonds(z) == [chi]


def test_zipup_bonds_and_tolerance():
    rng = np.random.default_rng(4)
    rho, u = WL.random_flow_state(4, 5, amp=0.05, modes=3)
    a = M.from_dense(rho, 4, 64, 1e-12)
    b = M.from_dense(u[0], 4, 64, 1e-12)
    ex = M.to_dense(a) * M.to_dense(b)
    for chi in (2, 4, 8):
        z = M.hadamard_zipup(a, b, chi, 1e-12)
        assert max(M.bonds(z)) <= chi
    # a loose tolerance cuts ranks below the cap, and the error grows with it
    e = []
    for tol in (1e-10, 1e-6, 1e-3):
        z = M.hadamard_zipup(a, b, 64, tol)
        e.append(np.linalg.norm(M.to_dense(z) - ex) / np.linalg.norm(ex))
    assert e[0] < 1e-9 and e[0] <= e[1] <= e[2] and e[2] < 0.05


def test_step_with_zipup_products_equals_dense_when_nothing_is_cut():
    case = WL.case_porous(n=3, chi=64, tau=0.6, tol=1e-14, precision="fp64")
    rho, u = WL.random_flow_state(3, 5, amp=0.01)
    case.rho_init, case.u_init = rho, u
    from oracle.dense_lbm import DenseLBM
    m = MPSLBM(case, product="zipup")
    d = DenseLBM(case)
    for _ in range(2):
        m.step()
        d.step()
    assert np.abs(m.dense_populations() - d.f).max() < 1e-11

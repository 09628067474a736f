"""Pins for the tensor-product mask composition (Appendix D): a geometry
repeated on a coarse grid is the tensor product of the coarse layout and
the fine unit geometry, its MPS is the chain of the two MPS, and its bond
dimensions are those of the parts (so the largest is the larger of theirs)."""
import dataclasses

import numpy as np

import workloads as WL
from oracle import mps as M
from oracle.mps_lbm import MPSLBM


def _compose_by_index(outer, inner):
    """combined[x, y, z] = outer[x // K, y // K, z // K] inner[x % K, y % K, z % K],
    written out cell by cell."""
    L, K = outer.shape[0], inner.shape[0]
    N = L * K
    out = np.empty((N, N, N))
    for x in range(N):
        for y in range(N):
            for z in range(N):
                out[x, y, z] = outer[x // K, y // K, z // K] * inner[x % K, y % K, z % K]
    return out


def test_chained_cores_contract_to_the_composition():
    rng = np.random.default_rng(7)
    outer = rng.standard_normal((4, 4, 4))
    inner = rng.standard_normal((4, 4, 4))
    a = M.from_dense(outer, 2, 1 << 20, 0.0)
    b = M.from_dense(inner, 2, 1 << 20, 0.0)
    combined = M.to_dense(M.tensor_product(a, b))
    assert np.allclose(combined, _compose_by_index(outer, inner), rtol=0, atol=1e-12)
    # the opposite order of the parts is a different field (the coarse
    # sites must come first)
    swapped = M.to_dense(M.tensor_product(b, a))
    assert np.abs(swapped - combined).max() > 0.1


def test_bonds_of_the_chain_are_those_of_the_parts():
    rng = np.random.default_rng(8)
    outer = (rng.uniform(size=(8, 8, 8)) < 0.4).astype(np.float64)
    inner = (rng.uniform(size=(4, 4, 4)) < 0.5).astype(np.float64)
    a = M.from_dense(outer, 3, 1 << 20, 1e-12)
    b = M.from_dense(inner, 2, 1 << 20, 1e-12)
    c = M.tensor_product(a, b)
    assert M.bonds(c) == M.bonds(a) + [1] + M.bonds(b)
    assert M.max_bond(c) == max(M.max_bond(a), M.max_bond(b))


def test_chain_has_the_minimal_ranks_of_the_dense_composite():
    # every unfolding of outer (x) inner has the rank of the matching
    # unfolding of one part, so the machine-precision TT-SVD of the dense
    # composite finds exactly the bonds of the chain
    rng = np.random.default_rng(9)
    outer = (rng.uniform(size=(4, 4, 4)) < 0.5).astype(np.float64)
    inner = (rng.uniform(size=(8, 8, 8)) < 0.3).astype(np.float64)
    chain = M.tensor_product(M.from_dense(outer, 2, 1 << 20, 1e-12),
                             M.from_dense(inner, 3, 1 << 20, 1e-12))
    direct = M.from_dense(_compose_by_index(outer, inner), 5, 1 << 20, 1e-12)
    assert M.bonds(direct) == M.bonds(chain)
    assert np.allclose(M.to_dense(direct), M.to_dense(chain), rtol=0, atol=1e-10)


def test_pin_fin_parts_compose_to_the_drawn_array():
    outer, inner, solid = WL.pin_fin_parts(5, 3)
    assert outer.shape == (8, 8, 8) and inner.shape == (4, 4, 4)
    assert np.array_equal(_compose_by_index(outer, inner).astype(np.uint8), solid)
    assert 0 < solid.mean() < 0.5
    m = M.tensor_product(M.from_dense(outer.astype(float), 3, 1 << 20, 1e-12),
                         M.from_dense(inner.astype(float), 2, 1 << 20, 1e-12))
    assert np.allclose(M.to_dense(m), solid, rtol=0, atol=1e-10)


def test_step_with_the_chained_mask_equals_the_step_with_the_dense_mask():
    case = WL.case_pinfin(n=4, l=2, chi=64, tau=0.6, u_in=0.03, tol=1e-12,
                          precision="fp64")
    dense_case = dataclasses.replace(case, mask_parts=None)
    a = MPSLBM(case)
    b = MPSLBM(dense_case)
    assert M.bonds(a.mask) == M.bonds(b.mask)
    assert np.allclose(M.to_dense(a.mask), M.to_dense(b.mask), rtol=0, atol=1e-12)
    assert abs(a.n_fluid - b.n_fluid) < 1e-9
    assert abs(a.n_fluid - float((1 - case.solid).sum())) < 1e-9
    for _ in range(2):
        a.step()
        b.step()
    fa = np.stack([M.to_dense(x) for x in a.f])
    fb = np.stack([M.to_dense(x) for x in b.f])
    assert np.abs(fa - fb).max() < 1e-10

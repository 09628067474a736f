"""Pins for the CPU MPS algebra (oracle) against what the paper and the
mathematics fix: printed values, brute-force dense contraction on small
grids, closed forms and invariants."""
import os

import numpy as np
import pytest

from oracle import mps as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_mps(rng, n, bonds):
    r = [1] + list(bonds) + [1]
    return [rng.standard_normal((r[k], 8, r[k + 1])) for k in range(n)]


# ---------------------------------------------------------------- scale order

def test_scale_order_hand_example():
    # n = 4: x = 5 = 0101, y = 3 = 0011, z = 12 = 1100 (x most significant
    # in each 3-bit group): sigma = (0,0,1)=1, (1,0,1)=5, (0,1,0)=2, (1,1,0)=6
    n, N = 4, 16
    f = np.zeros((N, N, N))
    f[5, 3, 12] = 7.0
    t = M.scale_order(f, n)
    assert t[1, 5, 2, 6] == 7.0
    assert np.count_nonzero(t) == 1
    assert np.array_equal(M.scale_unorder(t, n), f)


def test_scale_order_roundtrip_random():
    rng = np.random.default_rng(0)
    f = rng.standard_normal((8, 8, 8))
    assert np.array_equal(M.scale_unorder(M.scale_order(f, 3), 3), f)


# -------------------------------------------------------------- TT-SVD, NVPS

@pytest.mark.parametrize("n", [3, 4])
def test_tt_svd_exact_full_rank(n):
    rng = np.random.default_rng(n)
    N = 1 << n
    f = rng.standard_normal((N, N, N))
    X = M.from_dense(f, n, 10 ** 6, 0.0)
    # full bond ranks are min(8^k, 8^(n-k))
    assert M.bonds(X) == [min(8 ** k, 8 ** (n - k)) for k in range(1, n)]
    assert np.abs(M.to_dense(X) - f).max() < 1e-12 * np.abs(f).max() * 10
    # left-orthogonal cores (lorg equation)
    for c in X[:-1]:
        m = c.reshape(-1, c.shape[2])
        assert np.abs(m.T @ m - np.eye(m.shape[1])).max() < 1e-12


def test_tt_svd_truncation_bound():
    rng = np.random.default_rng(3)
    n, N = 4, 16
    x = np.linspace(0, 1, N)
    f = (np.sin(3 * x)[:, None, None] * np.cos(2 * x)[None, :, None] * x[None, None, :]
         + 1e-3 * rng.standard_normal((N, N, N)))
    for tol in (1e-1, 1e-2, 1e-3):
        X = M.from_dense(f, n, 10 ** 6, tol)
        err = np.linalg.norm(M.to_dense(X) - f) / np.linalg.norm(f)
        assert err <= tol * (1 + 1e-12)


def test_nvps_printed_compression_ratios():
    rows = []
    for line in open(os.path.join(GOLD, "compression_ratios.txt")):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split())
    assert len(rows) == 7
    for dim, n, chi, cr, dec in rows:
        got = M.compression_ratio(int(n), int(chi), int(dim))
        assert round(got, int(dec)) == pytest.approx(float(cr)), (dim, n, chi, got)


def test_nvps_exact_at_chi64_for_8_4_and_8_5():
    # the paper notes that MPS of N = 8^4 and 8^5 cells are exact at chi = 64:
    # the full bond profiles are [8,64,8] and [8,64,64,8]
    for n in (4, 5):
        assert M.nvps(n, 64) == M.nvps(n, 10 ** 6)
        assert M.nvps(n, 63) < M.nvps(n, 64)


# ------------------------------------------------- add, exact product, ones

def test_add_and_scale_brute_force():
    rng = np.random.default_rng(1)
    a = rand_mps(rng, 3, [3, 5])
    b = rand_mps(rng, 3, [2, 4])
    s = M.add(M.scale(a, 2.5), b)
    assert M.bonds(s) == [5, 9]
    assert np.allclose(M.contract(s), 2.5 * M.contract(a) + M.contract(b), atol=1e-12)


def test_hadamard_exact_brute_force():
    rng = np.random.default_rng(2)
    a = rand_mps(rng, 3, [3, 5])
    b = rand_mps(rng, 3, [2, 4])
    p = M.hadamard_exact(a, b)
    assert M.bonds(p) == [6, 20]
    assert np.allclose(M.contract(p), M.contract(a) * M.contract(b), atol=1e-12)


def test_inner_ones_and_plane_slice():
    rng = np.random.default_rng(4)
    n = 4
    a = rand_mps(rng, n, [5, 7, 3])
    d = M.to_dense(a)
    assert M.inner_ones(a) == pytest.approx(d.sum(), rel=1e-12)
    assert M.inner_ones(M.ones(n)) == 16 ** 3
    for ax in range(3):
        for idx in (0, 15, 6):
            s = M.to_dense(M.plane_slice(a, ax, idx))
            ref = np.zeros_like(d)
            sl = [slice(None)] * 3
            sl[ax] = idx
            ref[tuple(sl)] = d[tuple(sl)]
            assert np.allclose(s, ref, atol=1e-12)


# ------------------------------------------------------------------ rounding

def test_rounding_bound_orthogonality_and_spectra():
    rng = np.random.default_rng(5)
    n = 4
    a = rand_mps(rng, n, [6, 20, 6])
    b = rand_mps(rng, n, [6, 20, 6])
    s = M.add(a, M.scale(b, 0.3))
    dense = M.contract(s)
    nrm = np.linalg.norm(dense)
    for tol in (1e-1, 1e-3, 1e-12):
        r = M.round_mps(s, 10 ** 6, tol)
        err = np.linalg.norm(M.contract(r) - dense) / nrm
        assert err <= tol * (1 + 1e-9)
        # right-orthogonal cores k >= 2 (centre at site 1)
        for c in r[1:]:
            m = c.reshape(c.shape[0], -1)
            assert np.abs(m @ m.T - np.eye(m.shape[0])).max() < 1e-12
    # untruncated: singular values at each bond equal those of the unfolding
    info = M.RoundInfo()
    M.round_mps(s, 10 ** 6, 0.0, info)
    for j, k in enumerate(range(n - 1, 0, -1)):
        unf = dense.reshape(8 ** k, -1)
        sv = np.linalg.svd(unf, compute_uv=False)
        got = info.spectra[j]
        m = len(got)
        assert np.allclose(got, sv[:m], atol=1e-10 * sv[0])
        assert np.all(sv[m:] < 1e-10 * sv[0])


def test_rounding_chi_cap_is_optimal_at_one_bond():
    # for n = 2 rounding to chi is the truncated SVD (Eckart-Young)
    rng = np.random.default_rng(6)
    a = rand_mps(rng, 2, [8])
    full = M.contract(a).reshape(8, 8)
    sv = np.linalg.svd(full, compute_uv=False)
    r = M.round_mps(a, 3, 0.0)
    err = np.linalg.norm(M.contract(r).reshape(8, 8) - full)
    assert err == pytest.approx(np.sqrt(np.sum(sv[3:] ** 2)), rel=1e-10)


def test_rank_rule_is_minimal_and_meets_the_tail_bound():
    """The rank kept is the smallest one whose discarded tail is within
    delta^2: a rule that keeps one rank too many (or too few) fails here.
    The tails are summed independently of the rule, by a sorted cumulative
    sum of exact squares."""
    rng = np.random.default_rng(12)
    for trial in range(400):
        m = int(rng.integers(1, 40))
        s = np.sort(np.abs(rng.standard_normal(m)) * 10.0 ** rng.uniform(-8, 0, m))[::-1]
        tot = float(np.sum(s * s))
        delta2 = tot * 10.0 ** rng.uniform(-12, 0)
        chi = int(rng.integers(1, 45))
        r = M.rank_rule(s, delta2, chi)
        tail = lambda k: float(np.sum(s[k:] ** 2))  # weight discarded at rank k
        assert 1 <= r <= min(chi, m)
        if r < chi:
            assert tail(r) <= delta2
            # one rank fewer would discard too much
            if r > 1:
                assert tail(r - 1) > delta2
        else:
            # capped at chi: the uncapped rule needs at least chi
            assert chi == 1 or tail(chi - 1) > delta2 or chi > m


def test_rounding_keeps_the_exact_minimal_ranks_of_a_known_spectrum():
    """An n = 2 MPS built as U diag(s) V^T with orthonormal U, V has the
    bond spectrum s exactly; at a tolerance whose threshold falls between
    two known tails the rounding must keep exactly the rank in between."""
    rng = np.random.default_rng(13)
    s = np.array([1.0, 0.5, 0.2, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6])
    U, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    V, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    a = [U.reshape(1, 8, 8), (np.diag(s) @ V.T).reshape(8, 8, 1)]
    tot = float(np.sum(s * s))
    for keep in range(1, 8):
        lo, hi = float(np.sum(s[keep:] ** 2)), float(np.sum(s[keep - 1:] ** 2))
        delta2 = np.sqrt(lo * hi)  # strictly between the two tails
        tol = np.sqrt(delta2 / tot)  # n - 1 = 1 bond
        r = M.round_mps(a, 10 ** 6, tol)
        assert M.bonds(r) == [keep]


# ------------------------------------------------------- variational product

def test_variational_product_exact_at_full_bonds():
    rng = np.random.default_rng(7)
    n = 3
    # B at full rank [8, 8]: every product is representable
    B = M.from_dense(rng.standard_normal((8, 8, 8)), n, 10 ** 6, 0.0)
    Cm = rand_mps(rng, n, [3, 4])
    A = M.hadamard_variational(B, Cm)
    assert np.allclose(M.contract(A), M.contract(B) * M.contract(Cm), atol=1e-11)


def _residual_trace(B, Cm, sweeps):
    """Residual after each local update (instrumented copy of the sweep
    using the oracle's own contractions)."""
    target = M.contract(B) * M.contract(Cm)
    out = []
    for s in range(1, sweeps + 1):
        A = M.hadamard_variational(B, Cm, sweeps=s)
        out.append(np.linalg.norm(M.contract(A) - target))
    return out


def test_variational_product_residual_non_increasing_and_near_optimal():
    rng = np.random.default_rng(8)
    n = 4
    x = np.linspace(0, 1, 16)
    f1 = np.exp(-x[:, None, None] - 2 * x[None, :, None] * x[None, None, :])
    f2 = np.cos(4 * x[:, None, None] + x[None, :, None]) + x[None, None, :] ** 2
    B = M.from_dense(f1, n, 6, 0.0)
    Cm = M.from_dense(f2, n, 6, 0.0)
    res = _residual_trace(B, Cm, 4)
    assert all(res[i + 1] <= res[i] * (1 + 1e-10) for i in range(len(res) - 1))
    # compare with SVD truncation of the exact product at the same bonds
    exact = M.hadamard_exact(B, Cm)
    target = M.contract(exact)
    best = M.round_mps(exact, 6, 0.0)
    err_svd = np.linalg.norm(M.contract(best) - target)
    A = M.hadamard_variational(B, Cm)
    err_var = np.linalg.norm(M.contract(A) - target)
    assert err_var <= 3.0 * err_svd + 1e-12 * np.linalg.norm(target)


def test_variational_product_keeps_the_first_factors_bonds():
    """hadamard_variational takes the first factor as the candidate
    (Section 2.3): the result has its bonds whatever the second factor's
    rank, and where the exact product fits those bonds it is reproduced."""
    rng = np.random.default_rng(10)
    hi = M.from_dense(rng.standard_normal((8, 8, 8)), 3, 10 ** 6, 0.0)
    one_like = [np.ones((1, 8, 1)) * 1.5 for _ in range(3)]
    A = M.hadamard_variational(one_like, hi)
    assert M.bonds(A) == [1, 1]
    # a rank-1 second factor times a full-rank first factor is exact
    B = M.hadamard_variational(hi, one_like)
    assert M.bonds(B) == M.bonds(hi)
    assert np.allclose(M.contract(B), 1.5 ** 3 * M.contract(hi), atol=1e-11)


def test_product_puts_higher_rank_first():
    rng = np.random.default_rng(9)
    lo = rand_mps(rng, 3, [1, 1])
    hi = M.from_dense(rng.standard_normal((8, 8, 8)), 3, 10 ** 6, 0.0)
    A = M.product(lo, hi)
    assert M.bonds(A) == [8, 8]
    assert np.allclose(M.contract(A), M.contract(lo) * M.contract(hi), atol=1e-11)


# ---------------------------------------------------------------- shift MPOs

def _read_shift_golden():
    mats, cur = {}, None
    for line in open(os.path.join(GOLD, "shift_matrices_n2.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("S", "SHAT"):
            cur = line
            mats[cur] = []
        else:
            mats[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in mats.items()}


def test_shift_matrices_match_printed_n2():
    g = _read_shift_golden()
    assert np.array_equal(M.shift_matrix(2, True), g["S"])
    assert np.array_equal(M.shift_matrix(2, False), g["SHAT"])


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_shift_recursion_is_cyclic_and_noncyclic_shift(n):
    N = 1 << n
    v = np.arange(N, dtype=float) + 1.0
    S = M.shift_matrix(n, True)
    Sh = M.shift_matrix(n, False)
    assert np.array_equal(S @ v, np.roll(v, -1))          # (S f)(x) = f(x+1)
    ref = np.roll(v, -1)
    ref[-1] = 0.0
    assert np.array_equal(Sh @ v, ref)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_shift_mpo_cores_reproduce_recursion(n):
    """The rank-core-product factors A, B..B, C multiply out to S^(n)."""
    for cyclic in (True, False):
        cores = M.shift_cores_1d(n, True, cyclic)
        # contract block matrices: entries are 2x2 operators, combine by kron
        T = None
        for core in cores:
            rl, rr = core.shape[:2]
            if T is None:
                T = [[core[0, b] for b in range(rr)]]
                T = T[0]
            else:
                T = [sum(np.kron(T[a], core[a, b]) for a in range(rl)) for b in range(rr)]
        assert len(T) == 1
        assert np.array_equal(T[0], M.shift_matrix(n, cyclic))


D3Q19_DIRS = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
              (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


@pytest.mark.parametrize("n", [3, 4])
def test_streaming_mpo_equals_roll_all_18_directions(n):
    rng = np.random.default_rng(10 + n)
    N = 1 << n
    f = rng.standard_normal((N, N, N))
    X = M.from_dense(f, n, 10 ** 6, 0.0)
    for c in D3Q19_DIRS:
        for open_axes in [(0, 0, 0), (1, 0, 0), (1, 1, 1)]:
            Y = X
            for ax in range(3):
                if c[ax]:
                    Y = M.apply_mpo(M.stream_mpo(n, ax, c[ax], not open_axes[ax]), Y)
            ref = np.roll(f, c, axis=(0, 1, 2))
            for ax in range(3):
                if open_axes[ax] and c[ax]:
                    sl = [slice(None)] * 3
                    sl[ax] = 0 if c[ax] > 0 else N - 1
                    ref[tuple(sl)] = 0.0
            assert np.abs(M.to_dense(Y) - ref).max() < 1e-12 * np.abs(f).max() * 10


def test_shift_mpo_bond_dimensions():
    n = 5
    X = M.from_dense(np.random.default_rng(0).standard_normal((32, 32, 32)), n, 8, 0.0)
    Y = M.apply_mpo(M.stream_mpo(n, 0, 1, True), X)
    assert M.bonds(Y) == [2 * b for b in M.bonds(X)]
    # after rounding an axis shift of a smooth field keeps a low rank: the
    # shift MPO itself has rank 2 at every bond
    mpo = M.stream_mpo(n, 1, -1, True)
    assert [o.shape[3] for o in mpo[:-1]] == [2] * (n - 1)

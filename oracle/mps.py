"""Matrix product state algebra in plain numpy/LAPACK, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An MPS is a Python list of cores; core k has shape (r_{k-1}, 8, r_k) with
r_0 = r_n = 1 (Section 2.1, MPS equation).  Every routine follows the
paper's definition of the operation:

* scale ordering of a 3D field (Section 2.4, scale-ordering equation):
  site k carries the k-th most significant bit of x, y and z, grouped as
  sigma_k = 4 x_k + 2 y_k + z_k;
* TT-SVD construction (Section 2.1, svd-comp equation) and the centre
  shift by SVD with truncation (svd-move equation);
* the tensor-product composition of a coarse and a fine mask (Appendix D);
* elementwise addition by block-diagonal cores (Section 2.2, add equation),
  the exact Hadamard product (mul equation), MPO application (applympo
  equation);
* the variational compressed Hadamard product (Section 2.3, minimization
  equation), single-site, candidate = first factor, sweeping 1 -> n -> 1
  twice with QR centre shifts; the zip-up product, the alternative that
  Section 2.3 names;
* the cyclic / non-cyclic shift MPOs assembled from the 2x2 matrices
  I, J, J', P and the rank core product (Section 2.5), padded with
  identities to act on one spatial bit of each site.
"""
from __future__ import annotations

import numpy as np

D = 8  # physical dimension of a site: one bit of each of x, y, z


# --------------------------------------------------------------------------
# scale ordering and dense <-> MPS
# --------------------------------------------------------------------------

def scale_order(field: np.ndarray, n: int) -> np.ndarray:
    """[x][y][z] field of side 2**n -> order-n tensor with 8-valued indices."""
    t = np.asarray(field, dtype=np.float64).reshape([2] * (3 * n))
    perm = []
    for k in range(n):
        perm += [k, n + k, 2 * n + k]
    return t.transpose(perm).reshape([D] * n)


def scale_unorder(t: np.ndarray, n: int) -> np.ndarray:
    N = 1 << n
    t = np.asarray(t).reshape([2] * (3 * n))
    perm = [0] * (3 * n)
    for k in range(n):
        perm[k] = 3 * k
        perm[n + k] = 3 * k + 1
        perm[2 * n + k] = 3 * k + 2
    return t.transpose(perm).reshape(N, N, N)


def rank_rule(s: np.ndarray, delta2: float, chi: int) -> int:
    """Smallest r >= 1 whose discarded tail sum_{j>r} s_j^2 is <= delta2,
    capped at chi.  (The paper leaves the rule open; this is the standard
    TT-rounding choice that bounds the total error by tol * ||X||.)"""
    s2 = np.asarray(s, dtype=np.float64) ** 2
    m = len(s2)
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])  # tail[r] = sum_{j>=r}
    r = m
    for cand in range(1, m + 1):
        if tail[cand] <= delta2:
            r = cand
            break
    return max(1, min(r, chi))


def tt_svd(t: np.ndarray, n: int, chi: int, tol: float):
    """Dense order-n tensor -> MPS by successive truncated SVDs."""
    norm2 = float(np.sum(np.asarray(t, dtype=np.float64) ** 2))
    delta2 = (tol * tol * norm2 / (n - 1)) if n > 1 else 0.0
    cores = []
    M = np.asarray(t, dtype=np.float64).reshape(D, -1)
    r_prev = 1
    for k in range(n - 1):
        M = M.reshape(r_prev * D, -1)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        r = rank_rule(S, delta2, chi)
        cores.append(U[:, :r].reshape(r_prev, D, r))
        M = S[:r, None] * Vt[:r]
        r_prev = r
    cores.append(M.reshape(r_prev, D, 1))
    return cores


def from_dense(field: np.ndarray, n: int, chi: int, tol: float):
    return tt_svd(scale_order(field, n), n, chi, tol)


def contract(cores) -> np.ndarray:
    """Full contraction of an MPS to its order-n tensor."""
    t = cores[0].reshape(D, -1)
    for c in cores[1:]:
        rl, d, rr = c.shape
        t = (t.reshape(-1, rl) @ c.reshape(rl, d * rr)).reshape(-1, rr)
    return t.reshape([D] * len(cores))


def to_dense(cores) -> np.ndarray:
    n = len(cores)
    return scale_unorder(contract(cores), n)


def bonds(cores):
    return [c.shape[2] for c in cores[:-1]]


def tensor_product(outer, inner):
    """MPS of the composition m(x) = outer(x >> k) inner(x mod 2^k) per axis
    (Appendix D): with scale ordering the l sites of the coarse grid come
    first and the k sites of the fine grid after them, so the cores of the
    two MPS are simply chained; the bond between them is 1 (outer's last
    and inner's first bond)."""
    assert outer[-1].shape[2] == 1 and inner[0].shape[0] == 1
    return [c.copy() for c in outer] + [c.copy() for c in inner]


def ones(n: int):
    """Rank-1 all-ones MPS."""
    return [np.ones((1, D, 1)) for _ in range(n)]


def zeros(n: int):
    return [np.zeros((1, D, 1)) for _ in range(n)]


def scale(cores, a: float):
    out = [c.copy() for c in cores]
    out[0] = out[0] * a
    return out


def inner_ones(cores) -> float:
    """<1, X>: contraction with the rank-1 unit MPS (chain of matvecs)."""
    v = np.ones(1)
    for c in cores:
        v = v @ c.sum(axis=1)
    return float(v[0])


# --------------------------------------------------------------------------
# addition, rounding
# --------------------------------------------------------------------------

def add(a, b):
    """Block-diagonal cores: bonds add (add equation)."""
    n = len(a)
    if n == 1:
        return [a[0] + b[0]]
    out = []
    for k in range(n):
        x, y = a[k], b[k]
        if k == 0:
            out.append(np.concatenate([x, y], axis=2))
        elif k == n - 1:
            out.append(np.concatenate([x, y], axis=0))
        else:
            rl = x.shape[0] + y.shape[0]
            rr = x.shape[2] + y.shape[2]
            c = np.zeros((rl, D, rr))
            c[:x.shape[0], :, :x.shape[2]] = x
            c[x.shape[0]:, :, x.shape[2]:] = y
            out.append(c)
    return out


class RoundInfo:
    def __init__(self):
        self.spectra = []      # singular values per bond (right-to-left order)
        self.discarded = 0.0   # total discarded squared weight / ||X||^2


def round_mps(cores, chi: int, tol: float, info: RoundInfo | None = None):
    """Restore bond dimension <= chi: QR orthogonalisation from the left
    (centre moves to site n), then the centre is shifted back to site 1 by
    truncated SVDs (svd-move equation), truncating only at the centre.
    Per-bond threshold delta^2 = tol^2 ||X||^2 / (n-1)."""
    n = len(cores)
    c = [x.copy() for x in cores]
    if n == 1:
        return c
    for k in range(n - 1):
        rl, d, rr = c[k].shape
        Q, R = np.linalg.qr(c[k].reshape(rl * d, rr))
        c[k] = Q.reshape(rl, d, Q.shape[1])
        c[k + 1] = np.einsum("ab,bsc->asc", R, c[k + 1])
    norm2 = float(np.sum(c[n - 1] ** 2))
    delta2 = tol * tol * norm2 / (n - 1)
    disc = 0.0
    for k in range(n - 1, 0, -1):
        rl, d, rr = c[k].shape
        U, S, Vt = np.linalg.svd(c[k].reshape(rl, d * rr), full_matrices=False)
        r = rank_rule(S, delta2, chi)
        disc += float(np.sum(S[r:] ** 2))
        if info is not None:
            info.spectra.append(S.copy())
        c[k] = Vt[:r].reshape(r, d, rr)
        c[k - 1] = np.einsum("asb,bc->asc", c[k - 1], U[:, :r] * S[:r])
    if info is not None:
        info.discarded = max(info.discarded, disc / norm2 if norm2 > 0 else 0.0)
    return c


# --------------------------------------------------------------------------
# Hadamard products
# --------------------------------------------------------------------------

def hadamard_exact(a, b):
    """Cores joined by a Kronecker delta on the physical index; bonds
    multiply (mul equation)."""
    out = []
    for x, y in zip(a, b):
        t = np.einsum("asb,csd->acsbd", x, y)
        out.append(t.reshape(x.shape[0] * y.shape[0], D, x.shape[2] * y.shape[2]))
    return out


def sweep_positions(n: int, sweeps: int = 2):
    """Centre positions of the variational product: 1 -> n -> 1, twice
    (0-based, consecutive repeats dropped)."""
    one = list(range(n)) + list(range(n - 2, -1, -1))
    pos = list(one)
    for _ in range(sweeps - 1):
        pos += one[1:]
    return pos


def _lbc(L, b, c):
    """T[s, a, y, z] = sum_{b,c} L[a,b,c] B[b,s,y] C[c,s,z] (delta on s)."""
    T1 = np.tensordot(L, b, axes=([1], [0]))            # [a, c, s, y]
    a, cc, s, y = T1.shape
    T1 = T1.transpose(2, 0, 3, 1).reshape(s, a * y, cc)  # [s, (a y), c]
    T2 = np.matmul(T1, c.transpose(1, 0, 2))            # [s, (a y), z]
    return T2.reshape(s, a, y, c.shape[2])


def env_local(L, b, c, R):
    """Local optimum at the centre: A[a,s,x] = L[a,b,c] B[b,s,y] C[c,s,z] R[x,y,z]."""
    T = _lbc(L, b, c)                                   # [s, a, y, z]
    A = np.tensordot(T, R, axes=([2, 3], [1, 2]))       # [s, a, x]
    return np.ascontiguousarray(A.transpose(1, 0, 2))


def env_left(L, a_core, b, c):
    """L'[x,y,z] = L[a,b,c] A[a,s,x] B[b,s,y] C[c,s,z]."""
    T = _lbc(L, b, c)                                   # [s, a, y, z]
    return np.tensordot(a_core, T, axes=([0, 1], [1, 0]))


def env_right(a_core, b, c, R):
    """R'[a,b,c] = A[a,s,x] B[b,s,y] C[c,s,z] R[x,y,z]."""
    U1 = np.tensordot(a_core, R, axes=([2], [0]))       # [a, s, y, z]
    a, s, y, z = U1.shape
    U1 = U1.transpose(1, 0, 3, 2).reshape(s, a * z, y)  # [s, (a z), y]
    U2 = np.matmul(U1, b.transpose(1, 2, 0))            # [s, (a z), b]
    U2 = U2.reshape(s, a, z, b.shape[0])
    return np.tensordot(U2, c, axes=([0, 2], [1, 2]))   # [a, b, c]


def hadamard_variational(b, c, sweeps: int = 2):
    """Single-site variational fit of A ~ B (.) C (Section 2.3).
    Candidate A = B; environments L, R hold the partial contractions of
    A, B and C (joined by the delta on the physical index); the local
    optimum at the centre is the contraction L B C R; the centre moves
    by QR."""
    n = len(b)
    A = [x.copy() for x in b]
    # right-canonicalise the candidate (LQ from the right)
    for k in range(n - 1, 0, -1):
        rl, d, rr = A[k].shape
        Q, R = np.linalg.qr(A[k].reshape(rl, d * rr).T)
        A[k] = Q.T.reshape(Q.shape[1], d, rr)
        A[k - 1] = np.einsum("asb,bc->asc", A[k - 1], R.T)
    Renv = [None] * (n + 1)
    Lenv = [None] * (n + 1)
    Renv[n] = np.ones((1, 1, 1))
    Lenv[0] = np.ones((1, 1, 1))
    for k in range(n - 1, 0, -1):
        Renv[k] = env_right(A[k], b[k], c[k], Renv[k + 1])
    pos = sweep_positions(n, sweeps)
    for idx, p in enumerate(pos):
        A[p] = env_local(Lenv[p], b[p], c[p], Renv[p + 1])
        if idx + 1 == len(pos):
            break
        nxt = pos[idx + 1]
        rl, d, rr = A[p].shape
        if nxt > p:
            Q, _ = np.linalg.qr(A[p].reshape(rl * d, rr))
            assert Q.shape[1] == rr
            A[p] = Q.reshape(rl, d, rr)
            Lenv[p + 1] = env_left(Lenv[p], A[p], b[p], c[p])
        else:
            Q, _ = np.linalg.qr(A[p].reshape(rl, d * rr).T)
            assert Q.shape[1] == rl
            A[p] = Q.T.reshape(rl, d, rr)
            Renv[p] = env_right(A[p], b[p], c[p], Renv[p + 1])
    return A


def max_bond(a) -> int:
    return max([x.shape[2] for x in a[:-1]] + [1])


def right_canonical(a):
    """The same tensor with cores 2..n right-orthonormal (sum over the
    physical index and right bond of A A^T = I), by QR of the transposed
    unfoldings from the right; the norm ends in the first core."""
    out = [x.copy() for x in a]
    for k in range(len(out) - 1, 0, -1):
        rl, d, rr = out[k].shape
        Q, R = np.linalg.qr(out[k].reshape(rl, d * rr).T)
        out[k] = Q.T.reshape(Q.shape[1], d, rr)
        out[k - 1] = np.einsum("asb,cb->asc", out[k - 1], R)
    return out


def hadamard_zipup(b, c, chi: int, tol: float):
    """Zip-up product, the alternative to the variational product that
    Section 2.3 names (after Stoudenmire and White).  From the left, the
    carried factor L (r x r_b r_c) meets the next pair of cores,
    Z[a, s, b', c'] = sum_{b,c} L[a, (b, c)] b_k[b, s, b'] c_k[c, s, c'],
    and a truncated SVD of Z as an (8 r) x (r_b' r_c') matrix gives the
    output core U (orthonormal columns) and the next carry S V^T; the rank at
    each cut is the rounding rule with delta^2 = tol^2 ||Z||_F^2 / (n - 1),
    capped at chi.  The last site keeps Z.  The matrices factored have at most
    8 chi rows; the exact product (bond r_b r_c) is never formed.  Both
    factors are first brought to right-canonical form (QR from the right),
    so that each local SVD sees an orthonormal right part of each factor."""
    n = len(b)
    b, c = right_canonical(b), right_canonical(c)
    L = np.ones((1, 1))
    out = []
    for k in range(n):
        x, y = b[k], c[k]
        rb, rb1 = x.shape[0], x.shape[2]
        rc, rc1 = y.shape[0], y.shape[2]
        r = L.shape[0]
        Z = np.einsum("abc,bsd,cse->asde", L.reshape(r, rb, rc), x, y)
        Z = Z.reshape(r * D, rb1 * rc1)
        if k == n - 1:
            out.append(Z.reshape(r, D, 1))
            break
        U, S, Vt = np.linalg.svd(Z, full_matrices=False)
        delta2 = tol * tol * float(np.sum(S ** 2)) / (n - 1)
        rk = rank_rule(S, delta2, chi)
        out.append(U[:, :rk].reshape(r, D, rk))
        L = S[:rk, None] * Vt[:rk]
    return out


def product(x, y, sweeps: int = 2):
    """Variational product with the higher-rank factor as the candidate
    (ties keep the written order)."""
    if max_bond(y) > max_bond(x):
        x, y = y, x
    return hadamard_variational(x, y, sweeps)


# --------------------------------------------------------------------------
# shift MPOs (Section 2.5)
# --------------------------------------------------------------------------

I2 = np.eye(2)
J = np.array([[0.0, 1.0], [0.0, 0.0]])
Jp = np.array([[0.0, 0.0], [1.0, 0.0]])
P = np.array([[0.0, 1.0], [1.0, 0.0]])
Z2 = np.zeros((2, 2))


def shift_matrix(n: int, cyclic: bool) -> np.ndarray:
    """Dense S^(n) / S-hat^(n) from the recursion (recursive equation)."""
    if n == 1:
        return P.copy() if cyclic else J.copy()
    Sh = J.copy()
    for m in range(2, n):
        Jpm = Jp
        for _ in range(m - 2):
            Jpm = np.kron(Jpm, Jp)
        Sh = np.kron(I2, Sh) + np.kron(J, Jpm)
    Jpn = Jp
    for _ in range(n - 2):
        Jpn = np.kron(Jpn, Jp)
    return np.kron(I2, Sh) + np.kron(P if cyclic else J, Jpn)


def shift_cores_1d(n: int, forward: bool, cyclic: bool):
    """Rank-core-product factors of the 1D shift: A (or A-hat), B, ..., B, C.
    Each core is a block matrix of 2x2 blocks, array [row, col, nu, omega].
    forward: (S f)(x) = f(x+1) as printed; otherwise J and J' are swapped,
    which reverses the direction."""
    j, jp = (J, Jp) if forward else (Jp, J)
    if n == 1:
        return [((P if cyclic else j))[None, None]]
    first = np.stack([I2, P if cyclic else j])[None]            # (1, 2, 2, 2)
    mid = np.array([[I2, j], [Z2, jp]])                         # (2, 2, 2, 2)
    last = np.array([[j], [jp]])                                # (2, 1, 2, 2)
    return [first] + [mid] * (n - 2) + [last]


def pad_axis(m2: np.ndarray, axis: int) -> np.ndarray:
    """Embed a 2x2 operator on one spatial bit into the 8x8 site space
    (bits ordered x, y, z with x most significant)."""
    mats = [I2, I2, I2]
    mats[axis] = m2
    return np.kron(np.kron(mats[0], mats[1]), mats[2])


def shift_mpo(n: int, axis: int, forward: bool, cyclic: bool):
    """MPO cores (l, nu, omega, r) shifting along one axis of the 3D grid."""
    out = []
    for core in shift_cores_1d(n, forward, cyclic):
        rl, rr = core.shape[:2]
        o = np.zeros((rl, D, D, rr))
        for a in range(rl):
            for b in range(rr):
                o[a, :, :, b] = pad_axis(core[a, b], axis)
        out.append(o)
    return out


def apply_mpo(mpo, a):
    """Site-wise contraction of MPO and MPS physical indices; bonds
    multiply (applympo equation)."""
    out = []
    for o, x in zip(mpo, a):
        t = np.einsum("lnwr,awb->lanrb", o, x)
        out.append(t.reshape(o.shape[0] * x.shape[0], D, o.shape[3] * x.shape[2]))
    return out


def stream_mpo(n: int, axis: int, c: int, cyclic: bool):
    """Streaming f_new(x) = f_old(x - c) along one axis: c = -1 is the
    printed S (f(x+1)), c = +1 the J<->J' swapped one."""
    return shift_mpo(n, axis, forward=(c < 0), cyclic=cyclic)


# --------------------------------------------------------------------------
# rank-1 plane masks
# --------------------------------------------------------------------------

def plane_slice(a, axis: int, index: int):
    """m_B (.) X for m_B = indicator of the plane x_axis = index: a rank-1
    mask, applied exactly by zeroing the physical slices whose bit differs."""
    n = len(a)
    out = []
    for k in range(n):
        bit = (index >> (n - 1 - k)) & 1
        keep = np.array([((s >> (2 - axis)) & 1) == bit for s in range(D)], dtype=np.float64)
        out.append(a[k] * keep[None, :, None])
    return out


# --------------------------------------------------------------------------
# compression metrics (Section 4.2)
# --------------------------------------------------------------------------

def nvps(n: int, chi: int, dim: int = 3) -> int:
    """Number of variables parametrising one MPS component at bond chi."""
    d = 2 ** dim
    tot = 0
    for i in range(1, n + 1):
        left = min(d ** (i - 1), d ** (n - i + 1), chi)
        right = min(d ** i, d ** (n - i), chi)
        tot += left * d * right
    return tot


def compression_ratio(n: int, chi: int, dim: int = 3) -> float:
    return (2 ** n) ** dim / nvps(n, chi, dim)

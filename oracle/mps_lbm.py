"""The MPS lattice Boltzmann step on the CPU, FP64 (the method, step by step).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each of the Q populations (D3Q19, or the paper's D3Q15) is an MPS over
scale-ordered sites (Section 3.2).  One step is, in this order:

1. moments rho = sum_i f_i, j_a = sum_i c_ia f_i (macro equation), each a
   sum with rounding after every pairwise addition;
2. rho_0 = <1, rho> / N_fluid (contraction with the rank-1 unit MPS,
   normalised by the fluid cell count);
3. 1/rho by the second-order Taylor expansion about rho_0 (Section 3.2),
   r = (1/rho_0)(1 - e + e (.) e) with e = rho/rho_0 - 1 (or k Newton-Schulz
   steps y <- y (.) (2 - rho (.) y) from y = 1/rho_0);
4. j_eq = j + tau g rho (Shan-Chen forcing, Appendix A), u_a = j_eq,a (.) r,
   Pi_ab = j_eq,a (.) u_b by variational products (Section 2.3);
5. f_i <- (1 - 1/tau) f_i + (1/tau) w_i [S0 + 3 c_i.j_eq + 4.5 c_i c_i : Pi]
   with S0 = rho - 1.5 tr Pi (BGK with the equilibrium equation);
6. streaming by shift MPOs, one axis at a time with rounding after each
   (Section 2.5); open axes use the non-cyclic shift;
7. open faces add m_B (.) b(f_ihat, rho_b, u_b) (boundaries equation) with
   rank-1 plane masks;
8. immersed objects: f_i <- f_i - m_O (.) f_i + S(c_i)(m_O (.) f_ihat)
   (objects equation).

A "sum" of several terms is a pairwise tree (adjacent pairs, left to
right, an odd last term carried up), rounded after each addition.
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .inflow import face_velocity
from .lattice import PI_PAIRS, get as get_lattice
from .metrics import pressure_drop

INV_TAYLOR2 = "taylor2"
INV_NEWTON = "newton"


class Counters:
    def __init__(self):
        self.roundings = 0
        self.products = 0
        self.max_discarded = 0.0


class MPSLBM:
    """CPU MPS-LBM state.  `case` is a workloads.Case."""

    def __init__(self, case, inv_mode=INV_TAYLOR2, inv_iters=2, sweeps=2,
                 f_init=None, product="variational"):
        self.case = case
        self.lat = get_lattice(int(case.lattice))
        self.n = case.n
        self.N = case.N
        self.chi = int(case.chi)
        self.tol = float(case.tol)
        self.tau = float(case.tau)
        self.omega = 1.0 / self.tau
        self.g = np.array(case.g, dtype=np.float64)
        self.inv_mode = inv_mode
        self.inv_iters = inv_iters
        self.sweeps = sweeps
        # "variational" (Section 2.3, the method) or "zipup" (the named
        # alternative, truncated at chi and the rounding tolerance)
        self.product = product
        self.axis_open = tuple(case.axis_open)
        self.cnt = Counters()
        n = self.n
        self.one = M.ones(n)
        # obstacle mask (objects equation): TT-SVD of the binary solid field
        # at tol_mask.  By default no rank cap applies, so the mask is
        # represented to machine precision, which is how Section 5.2 fixes
        # the mask bond dimension; case.chi_mask caps it explicitly.
        chi_mask = int(case.chi_mask) if case.chi_mask else 1 << 30
        fluid = None
        if case.solid is not None and case.mask_parts is not None:
            # a geometry repeated on a coarse grid (Appendix D): each part is
            # decomposed on its own grid and the two MPS are chained
            outer, inner = case.mask_parts
            l = int(round(np.log2(outer.shape[0])))
            self.mask = M.tensor_product(
                M.from_dense(outer.astype(np.float64), l, chi_mask, case.tol_mask),
                M.from_dense(inner.astype(np.float64), n - l, chi_mask, case.tol_mask))
            self.n_fluid = float(self.N ** 3) - M.inner_ones(self.mask)
            fluid = 1.0 - case.solid.astype(np.float64)
        elif case.solid is not None:
            self.mask = M.from_dense(case.solid.astype(np.float64), n, chi_mask,
                                     case.tol_mask)
            self.n_fluid = float(self.N ** 3) - M.inner_ones(self.mask)
            fluid = 1.0 - case.solid.astype(np.float64)
        else:
            self.mask = None
            self.n_fluid = float(self.N ** 3)
        # face masks m_B (boundaries equations): the fluid cells of each open
        # face plane, decomposed from that dense definition at tol_mask; they
        # are added into population sums, so their rank is capped at chi
        self.fluid_plane = {}
        for ax in range(3):
            if not self.axis_open[ax]:
                continue
            for side in (0, 1):
                face = 2 * ax + side
                if case.face_bc[face]:
                    idx = 0 if side == 0 else self.N - 1
                    plane = np.zeros((self.N,) * 3)
                    sl = [slice(None)] * 3
                    sl[ax] = idx
                    plane[tuple(sl)] = 1.0
                    if fluid is not None:
                        plane *= fluid
                    self.fluid_plane[face] = M.from_dense(plane, n, self.chi,
                                                          case.tol_mask)
        if f_init is None:
            f_init = self.initial_dense(case)
        self.f = [M.from_dense(f_init[i], n, self.chi, self.tol)
                  for i in range(self.lat.q)]
        self.step_count = 0
        self.last = {}

    @staticmethod
    def initial_dense(case):
        lat = get_lattice(int(case.lattice))
        C, W, Q = lat.c, lat.w, lat.q
        """f_i = (1 - m_O) f_eq,i(rho, u) evaluated densely (the initial
        state is given as fields, then decomposed)."""
        rho = case.rho0_field().astype(np.float64)
        u = case.u0_field().astype(np.float64)
        fluid = 1.0 if case.solid is None else (1.0 - case.solid.astype(np.float64))
        uu = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        out = np.empty((Q,) + rho.shape)
        for i in range(Q):
            cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
            out[i] = fluid * W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
        return out

    # ---- building blocks --------------------------------------------------
    def rnd(self, x):
        info = M.RoundInfo()
        y = M.round_mps(x, self.chi, self.tol, info)
        self.cnt.roundings += 1
        self.cnt.max_discarded = max(self.cnt.max_discarded, info.discarded)
        return y

    def lin_sum(self, terms):
        items = [M.scale(x, a) for (a, x) in terms if a != 0.0]
        if not items:
            return M.zeros(self.n)
        while len(items) > 1:
            nxt = []
            for i in range(0, len(items) - 1, 2):
                nxt.append(self.rnd(M.add(items[i], items[i + 1])))
            if len(items) % 2:
                nxt.append(items[-1])
            items = nxt
        return items[0]

    def prod(self, x, y):
        self.cnt.products += 1
        if self.product == "zipup":
            return M.hadamard_zipup(x, y, self.chi, self.tol)
        return M.product(x, y, self.sweeps)

    def prod_first(self, x, y):
        """Variational product with the first factor as the candidate (the
        zip-up product when chosen)."""
        self.cnt.products += 1
        if self.product == "zipup":
            return M.hadamard_zipup(x, y, self.chi, self.tol)
        return M.hadamard_variational(x, y, self.sweeps)

    def stream(self, x, c):
        for ax in range(3):
            if c[ax] != 0:
                mpo = M.stream_mpo(self.n, ax, int(c[ax]), not self.axis_open[ax])
                x = self.rnd(M.apply_mpo(mpo, x))
        return x

    def inverse_density(self, rho, rho0):
        if self.inv_mode == INV_TAYLOR2:
            e = self.lin_sum([(1.0 / rho0, rho), (-1.0, self.one)])
            ee = self.prod(e, e)
            return self.lin_sum([(1.0 / rho0, self.one), (-1.0 / rho0, e),
                                 (1.0 / rho0, ee)])
        if self.inv_mode == INV_NEWTON:
            # y1 = 2/rho0 - rho/rho0^2 is linear in rho (no product)
            y = self.lin_sum([(2.0 / rho0, self.one), (-1.0 / rho0 ** 2, rho)])
            for _ in range(self.inv_iters - 1):
                ry = self.prod(rho, y)
                t = self.lin_sum([(2.0, self.one), (-1.0, ry)])
                y = self.prod(y, t)
            return y
        raise ValueError(self.inv_mode)

    # ---- the step ---------------------------------------------------------
    def collide(self):
        f = self.f
        C, W, Q = self.lat.c, self.lat.w, self.lat.q
        rho = self.lin_sum([(1.0, f[i]) for i in range(Q)])
        j = [self.lin_sum([(float(C[i, a]), f[i]) for i in range(Q) if C[i, a] != 0])
             for a in range(3)]
        rho0 = M.inner_ones(rho) / self.n_fluid
        r = self.inverse_density(rho, rho0)
        jeq = []
        for a in range(3):
            if self.g[a] != 0.0:
                jeq.append(self.lin_sum([(1.0, j[a]), (self.tau * self.g[a], rho)]))
            else:
                jeq.append(j[a])
        u = [self.prod(jeq[a], r) for a in range(3)]
        Pi = {(a, b): self.prod(jeq[a], u[b]) for (a, b) in PI_PAIRS}
        S0 = self.lin_sum([(1.0, rho), (-1.5, Pi[(0, 0)]), (-1.5, Pi[(1, 1)]),
                           (-1.5, Pi[(2, 2)])])
        om = self.omega
        fpost = []
        for i in range(Q):
            w = W[i]
            terms = [(1.0 - om, f[i]), (om * w, S0)]
            for a in range(3):
                if C[i, a]:
                    terms.append((3.0 * om * w * C[i, a], jeq[a]))
            for (a, b) in PI_PAIRS:
                coef = C[i, a] * C[i, b] * (1 if a == b else 2)
                if coef:
                    terms.append((4.5 * om * w * coef, Pi[(a, b)]))
            fpost.append(self.lin_sum(terms))
        return fpost, dict(rho=rho, j=j, jeq=jeq, u=u, Pi=Pi, r=r, rho0=rho0)

    def boundary_terms(self, fpost, mac):
        """Terms of m_B (.) b for every population entering an open face."""
        case = self.case
        C, W, OPP, Q = self.lat.c, self.lat.w, self.lat.opp, self.lat.q
        out = {}
        for ax in range(3):
            if not self.axis_open[ax]:
                continue
            for side in (0, 1):
                face = 2 * ax + side
                typ = case.face_bc[face]
                if not typ:
                    continue
                idx = 0 if side == 0 else self.N - 1
                entering = 1 if side == 0 else -1
                fp = self.fluid_plane[face]
                if typ == 2:
                    uB = [self.rnd(M.plane_slice(mac["u"][a], ax, idx)) for a in range(3)]
                    uu = {(a, b): self.prod(uB[a], uB[b]) for (a, b) in PI_PAIRS}
                for i in range(Q):
                    if C[i, ax] != entering:
                        continue
                    c = C[i].astype(np.float64)
                    fo = M.plane_slice(fpost[OPP[i]], ax, idx)
                    if typ == 1:
                        ub = np.array(face_velocity(case, face, self.step_count))
                        terms = [(1.0, fo), (6.0 * W[i] * mac["rho0"] * float(c @ ub), fp)]
                    else:
                        rho_b = float(case.face_val[face][0])
                        k = 2.0 * W[i] * rho_b
                        terms = [(-1.0, fo), (k, fp)]
                        for (a, b) in PI_PAIRS:
                            if a == b:
                                coef = k * (4.5 * c[a] * c[a] - 1.5)
                            else:
                                coef = k * 9.0 * c[a] * c[b]
                            if coef != 0.0:
                                terms.append((coef, uu[(a, b)]))
                    out.setdefault(i, []).extend(terms)
        return out

    def step(self):
        C, OPP, Q = self.lat.c, self.lat.opp, self.lat.q
        fpost, mac = self.collide()
        bterms = self.boundary_terms(fpost, mac)
        fs = [fpost[0]] + [self.stream(fpost[i], C[i]) for i in range(1, Q)]
        for i, terms in sorted(bterms.items()):
            fs[i] = self.lin_sum([(1.0, fs[i])] + terms)
        if self.mask is not None:
            # the candidate of each obstacle product is the population, the
            # factor whose bond dimension the result keeps (Section 2.3)
            g = [None] + [self.prod_first(fs[i], self.mask) for i in range(1, Q)]
            fn = [fs[0]]
            for i in range(1, Q):
                h = self.stream(g[OPP[i]], C[i])
                fn.append(self.lin_sum([(1.0, fs[i]), (-1.0, g[i]), (1.0, h)]))
            fs = fn
        self.f = fs
        self.last = mac
        self.step_count += 1
        return mac

    # ---- observables -------------------------------------------------------
    def dense_populations(self):
        return np.stack([M.to_dense(x) for x in self.f])

    def pressure_drop(self, lo, hi, rho_ref: float) -> float:
        """Delta p / p_0 over the fluid cells of a box (Section 4.2), from the
        dense density sum_i f_i."""
        rho = sum(M.to_dense(x) for x in self.f)
        return pressure_drop(rho, self.case.solid, lo, hi, rho_ref)

    def mass(self):
        return sum(M.inner_ones(x) for x in self.f)

    def momentum(self):
        s = [M.inner_ones(x) for x in self.f]
        C, Q = self.lat.c, self.lat.q
        return np.array([sum(C[i, a] * s[i] for i in range(Q)) for a in range(3)],
                        dtype=np.float64)

    def bond_dims(self):
        return [M.bonds(x) for x in self.f]

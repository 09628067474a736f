"""Dense FP64 D3Q19 lattice Boltzmann solver: the plain definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One time step is collide-then-stream (Section 3.1, evolution equation) with
the BGK operator (collision equation) relaxing towards the equilibrium
(equilibrium equation).  The equilibrium is assembled in the form the MPS
method evaluates it, from the density rho, the momentum j_eq and the second
moment Pi_ab = j_eq,a u_b:

    f_eq,i = w_i [ rho + 3 c_i.j_eq + 4.5 c_i c_i : Pi - 1.5 tr(Pi) ]

which equals w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u) when u = j_eq / rho.
The inverse density follows Section 3.2: exactly, by the second-order
Taylor expansion about the global mean rho_0 (the paper's choice), or by k
Newton-Schulz steps started at 1/rho_0.  Forcing follows the Shan-Chen
velocity shift of Appendix A (j_eq = j + tau F, F = rho g).  Non-periodic
axes stream with the non-cyclic shift and add the boundary function on the
boundary cells (Section 3.2.1, boundaries equation); immersed solids use the
masked bounce-back rule of the objects equation.
"""
from __future__ import annotations

import numpy as np

from .inflow import face_velocity
from .lattice import D3Q19, PI_PAIRS, get as get_lattice

INV_EXACT = "exact"
INV_TAYLOR2 = "taylor2"
INV_NEWTON = "newton"


def shift_field(a: np.ndarray, c, axis_open) -> np.ndarray:
    """Streaming shift of one population: out(x) = a(x - c).  Periodic axes
    wrap; open axes fill the cells entering through the face with zero."""
    out = np.roll(a, shift=tuple(int(v) for v in c), axis=(0, 1, 2))
    for ax in range(3):
        if axis_open[ax] and c[ax] != 0:
            sl = [slice(None)] * 3
            sl[ax] = 0 if c[ax] > 0 else a.shape[ax] - 1
            out[tuple(sl)] = 0.0
    return out


def inverse_density(rho, rho0, mode=INV_TAYLOR2, iters=2, fluid=None):
    """Approximate 1/rho (Section 3.2, the Taylor expansion about rho_0)."""
    if mode == INV_EXACT:
        out = np.zeros_like(rho)
        nz = rho != 0
        out[nz] = 1.0 / rho[nz]
        return out
    if mode == INV_TAYLOR2:
        e = rho / rho0 - 1.0
        return (1.0 - e + e * e) / rho0
    if mode == INV_NEWTON:
        y = np.full_like(rho, 1.0 / rho0)
        for _ in range(iters):
            y = y * (2.0 - rho * y)
        return y
    raise ValueError(mode)


def moments(f):
    """rho and j of populations of any of the velocity sets (by their count)."""
    lat = get_lattice(f.shape[0])
    rho = f.sum(axis=0)
    j = np.einsum("ia,ixyz->axyz", lat.c.astype(np.float64), f)
    return rho, j


def equilibrium(rho, jeq, Pi, lat=D3Q19):
    """j-form equilibrium; Pi is a dict {(a,b): field} with a <= b."""
    trPi = Pi[(0, 0)] + Pi[(1, 1)] + Pi[(2, 2)]
    S0 = rho - 1.5 * trPi
    feq = np.empty((lat.q,) + rho.shape)
    for i in range(lat.q):
        c = lat.c[i]
        acc = S0.copy()
        for a in range(3):
            if c[a]:
                acc += 3.0 * c[a] * jeq[a]
        for (a, b) in PI_PAIRS:
            coef = c[a] * c[b] * (1 if a == b else 2)
            if coef:
                acc += 4.5 * coef * Pi[(a, b)]
        feq[i] = lat.w[i] * acc
    return feq


class DenseLBM:
    """Dense solver state + step.  `case` is a workloads.Case; `shape`
    overrides the cubic N^3 grid (the dense definition needs no cube)."""

    def __init__(self, case, inv_mode=INV_TAYLOR2, inv_iters=2, shape=None):
        self.case = case
        self.lat = get_lattice(int(case.lattice))
        self.tau = float(case.tau)
        self.g = np.array(case.g, dtype=np.float64)
        self.inv_mode = inv_mode
        self.inv_iters = inv_iters
        if shape is None:
            shape = (case.N,) * 3 if case.solid is None else case.solid.shape
        self.shape = tuple(shape)
        self.solid = (np.zeros(self.shape) if case.solid is None
                      else case.solid.astype(np.float64))
        self.fluid = 1.0 - self.solid
        self.n_fluid = float(self.fluid.sum())
        self.axis_open = tuple(case.axis_open)
        rho = (case.rho_init if case.rho_init is not None
               else np.ones(self.shape)).astype(np.float64)
        u = (case.u_init if case.u_init is not None
             else np.zeros((3,) + self.shape)).astype(np.float64)
        self.f = self.initial_populations(rho, u)
        self.last_u = None
        self.step_count = 0

    def initial_populations(self, rho, u):
        """f_i = (1 - m) f_eq,i(rho, u) with the exact velocity/Pi."""
        j = rho[None] * u
        Pi = {(a, b): rho * u[a] * u[b] for (a, b) in PI_PAIRS}
        return self.fluid[None] * equilibrium(rho, j, Pi, self.lat)

    def collide(self, f):
        rho, j = moments(f)
        rho0 = rho.sum() / self.n_fluid
        r = inverse_density(rho, rho0, self.inv_mode, self.inv_iters)
        jeq = j + self.tau * self.g[:, None, None, None] * rho[None]
        u = jeq * r[None]
        Pi = {(a, b): jeq[a] * u[b] for (a, b) in PI_PAIRS}
        feq = equilibrium(rho, jeq, Pi, self.lat)
        fpost = f + (feq - f) / self.tau
        return fpost, dict(rho=rho, j=j, jeq=jeq, u=u, rho0=rho0, r=r)

    def boundary_terms(self, fpost, mac):
        """Open faces: m_B * b(f_ihat, rho_b, u_b) for every population
        entering through the face (boundaries equation).  Returns a list of
        (i, face_index_tuple, values) to add after streaming."""
        case = self.case
        C, W, OPP = self.lat.c, self.lat.w, self.lat.opp
        out = []
        for ax in range(3):
            if not self.axis_open[ax]:
                continue
            for side in (0, 1):
                face = 2 * ax + side
                typ = case.face_bc[face]
                if typ == 0:
                    continue
                idx = 0 if side == 0 else self.shape[ax] - 1
                sl = [slice(None)] * 3
                sl[ax] = idx
                sl = tuple(sl)
                entering = 1 if side == 0 else -1
                fl = self.fluid[sl]
                for i in range(self.lat.q):
                    if C[i][ax] != entering:
                        continue
                    c = C[i].astype(np.float64)
                    fo = fpost[OPP[i]][sl]
                    if typ == 1:  # velocity: Ladd bounce-back with rho_b = rho_0
                        ub = np.array(face_velocity(case, face, self.step_count))
                        b = fo + 6.0 * W[i] * mac["rho0"] * float(c @ ub) * fl
                    elif typ == 2:  # pressure: anti-bounce-back, u_b = local u
                        rho_b = float(case.face_val[face][0])
                        u = mac["u"][(slice(None),) + sl]
                        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
                        uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
                        b = -fo + 2.0 * W[i] * rho_b * (fl + 4.5 * cu * cu - 1.5 * uu)
                    else:
                        raise ValueError(typ)
                    out.append((i, sl, b))
        return out

    def step(self):
        f = self.f
        fpost, mac = self.collide(f)
        bterms = self.boundary_terms(fpost, mac)
        C, OPP, Q = self.lat.c, self.lat.opp, self.lat.q
        fs = np.empty_like(fpost)
        for i in range(Q):
            fs[i] = shift_field(fpost[i], C[i], self.axis_open)
        for (i, sl, b) in bterms:
            fs[i][sl] += b
        if self.case.solid is not None:
            m = self.solid
            fn = np.empty_like(fs)
            for i in range(Q):
                fn[i] = (1.0 - m) * fs[i] + shift_field(m * fs[OPP[i]], C[i],
                                                         self.axis_open)
            fs = fn
        self.f = fs
        self.last_u = mac["u"]
        self.step_count += 1
        return mac

    # observables ------------------------------------------------------
    def rho(self):
        return self.f.sum(axis=0)

    def j(self):
        return moments(self.f)[1]

    def velocity(self):
        """u = j / rho on fluid cells (exact), 0 in solid."""
        rho, j = moments(self.f)
        u = np.zeros_like(j)
        nz = rho != 0
        u[:, nz] = j[:, nz] / rho[nz]
        return u

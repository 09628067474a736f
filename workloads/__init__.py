"""Seeded synthetic workloads for the MPS lattice Boltzmann step.

This module only produces inputs: solid masks, initial density and velocity
fields and the physical/numerical parameters of each case.  It holds none of
the method's arithmetic, so both the HIP library and the CPU oracle can take
their inputs from here without sharing any code of the method itself.

The paper's own geometries (an idealised aneurysm and a pin-fin heat sink,
Section 4.1) are not available; the generators below stand in for them with
seeded shapes of the same kind: a porous medium of random spheres, a
branching tube tree with Murray's-law radii and an array of cylindrical pins.

Conventions: a field on an N^3 grid is a C-order array indexed [x][y][z];
solid masks are uint8 with 1 = solid; N = 2**n.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# Boundary-condition face types (per face of an open axis).
BC_NONE = 0
BC_VELOCITY = 1
BC_PRESSURE = 2


@dataclass
class Case:
    """One simulation case: geometry + parameters + initial macroscopic state."""
    name: str
    n: int                                   # N = 2**n cells per axis
    tau: float
    chi: int
    tol: float
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # body acceleration (F = rho g)
    solid: Optional[np.ndarray] = None       # uint8 [N][N][N], 1 = solid
    axis_open: Tuple[int, int, int] = (0, 0, 0)
    # face order: (x-low, x-high, y-low, y-high, z-low, z-high)
    face_bc: Tuple[int, ...] = (0, 0, 0, 0, 0, 0)
    # velocity faces: u_b vector; pressure faces: (rho_b, 0, 0)
    face_val: Tuple[Tuple[float, float, float], ...] = ((0.0, 0.0, 0.0),) * 6
    rho_init: Optional[np.ndarray] = None    # [N][N][N]; None = 1
    u_init: Optional[np.ndarray] = None      # [3][N][N][N]; None = 0
    steps: int = 1
    precision: str = "fp64"
    chi_mask: Optional[int] = None
    tol_mask: float = 1e-12
    # (outer [L][L][L], inner [K][K][K]) uint8 with L K = N: the solid is the
    # inner geometry placed in every solid cell of the coarse outer grid
    mask_parts: Optional[Tuple[np.ndarray, np.ndarray]] = None
    # velocity faces with a time-dependent inflow: face -> (c0..c5, dt), the
    # face velocity scaled by c0 + c1 (1 - e^(-c2 t)) + c3 t^c4 e^(-c5 t)
    # with t = (steps taken) dt
    face_profile: Optional[dict] = None
    lattice: int = 19                        # 19 (D3Q19) or 15 (D3Q15)
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return 1 << self.n

    def rho0_field(self) -> np.ndarray:
        if self.rho_init is not None:
            return self.rho_init
        return np.ones((self.N,) * 3)

    def u0_field(self) -> np.ndarray:
        if self.u_init is not None:
            return self.u_init
        return np.zeros((3,) + (self.N,) * 3)


# --------------------------------------------------------------------------
# geometry generators
# --------------------------------------------------------------------------

def channel_mask(n: int) -> np.ndarray:
    """Plane channel: solid rows y = 0 and y = N-1, fluid elsewhere."""
    N = 1 << n
    m = np.zeros((N, N, N), dtype=np.uint8)
    m[:, 0, :] = 1
    m[:, N - 1, :] = 1
    return m


def sphere_pack_mask(n: int, solid_fraction: float, rmin: float, rmax: float,
                     seed: int, wrap_axes=(1, 2)) -> np.ndarray:
    """Random spheres (radius U[rmin, rmax], centre U[0,N)^3) added until the
    solid fraction reaches `solid_fraction`.  Distances wrap periodically on
    `wrap_axes` so the medium is periodic there."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    m = np.zeros((N, N, N), dtype=np.uint8)
    ax = np.arange(N, dtype=np.float64)
    target = solid_fraction * N ** 3
    count = 0
    while m.sum() < target:
        c = rng.uniform(0.0, N, size=3)
        r = rng.uniform(rmin, rmax)
        d2 = []
        for a in range(3):
            d = ax - c[a]
            if a in wrap_axes:
                d = (d + N / 2.0) % N - N / 2.0
            d2.append(d * d)
        dist2 = d2[0][:, None, None] + d2[1][None, :, None] + d2[2][None, None, :]
        m[dist2 <= r * r] = 1
        count += 1
        if count > 100000:
            break
    return m


def _capsule_dist2(px, py, pz, a, b):
    """Squared distance from grid points to the segment a-b."""
    ab = b - a
    L2 = float(ab @ ab)
    dx, dy, dz = px - a[0], py - a[1], pz - a[2]
    if L2 == 0.0:
        return dx * dx + dy * dy + dz * dz
    t = (dx * ab[0] + dy * ab[1] + dz * ab[2]) / L2
    t = np.clip(t, 0.0, 1.0)
    qx = dx - t * ab[0]
    qy = dy - t * ab[1]
    qz = dz - t * ab[2]
    return qx * qx + qy * qy + qz * qz


def vascular_tree_mask(n: int, seed: int, generations: int = 3,
                       r_root_frac: float = 12.0 / 128.0) -> Tuple[np.ndarray, list]:
    """Branching tube tree along +x.  The root tube (radius r_root_frac * N)
    starts on the x = 0 face; each generation splits symmetrically into two
    children of radius r / 2**(1/3) (Murray's law), opening at an angle
    U[20, 40] degrees about a random azimuth; after `generations` splits the
    leaves run straight to the x = N-1 face.  Solid = outside every tube.
    Returns (mask, segments) with segments = [(a, b, radius), ...]."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    r0 = max(1.5, r_root_frac * N)
    seg_len = N / float(generations + 1)
    segments = []
    centre = np.array([0.0, (N - 1) / 2.0, (N - 1) / 2.0])
    a = centre.copy()
    b = np.array([seg_len, centre[1], centre[2]])
    segments.append((a, b, r0))
    tips = [(b, r0)]
    for gen in range(1, generations + 1):
        new_tips = []
        for (p, r) in tips:
            rc = max(1.2, r / 2.0 ** (1.0 / 3.0))
            theta = math.radians(rng.uniform(20.0, 40.0))
            phi = rng.uniform(0.0, 2.0 * math.pi)
            for sgn in (+1.0, -1.0):
                d = np.array([math.cos(theta),
                              sgn * math.sin(theta) * math.cos(phi),
                              sgn * math.sin(theta) * math.sin(phi)])
                q = p + d * (seg_len / math.cos(theta))
                lo, hi = rc + 1.0, N - 2.0 - rc
                q[1] = min(max(q[1], lo), hi)
                q[2] = min(max(q[2], lo), hi)
                q[0] = p[0] + seg_len
                segments.append((p.copy(), q, rc))
                new_tips.append((q, rc))
        tips = new_tips
    for (p, r) in tips:
        q = np.array([N - 1.0 + r, p[1], p[2]])
        segments.append((p.copy(), q, r))
    ax = np.arange(N, dtype=np.float64)
    px = ax[:, None, None]
    py = ax[None, :, None]
    pz = ax[None, None, :]
    fluid = np.zeros((N, N, N), dtype=bool)
    for (a, b, r) in segments:
        fluid |= _capsule_dist2(px, py, pz, a, b) <= r * r
    return (~fluid).astype(np.uint8), segments


def pin_fin_parts(n: int, l: int = 3, seed: int = 2512 + 6, radius_frac: float = 0.25,
                  x_range: Tuple[int, int] = (1, 7), z_cells: Optional[int] = None,
                  missing: float = 0.2) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Array of vertical (z) cylindrical pins on a coarse grid of 2**l cells
    per axis, each coarse cell of side K = 2**(n - l) holding one pin of
    radius radius_frac * K about its centre line.  Pins stand in the coarse
    columns x_range[0] <= X < x_range[1] (every Y), over the lower z_cells
    coarse layers (default half the height); each (X, Y) column is left
    empty with probability `missing` (seeded).  Returns (outer [L]^3,
    inner [K]^3, solid [N]^3), all uint8; solid is drawn directly from the
    pin axes on the fine grid."""
    N, L, K = 1 << n, 1 << l, 1 << (n - l)
    zc = L // 2 if z_cells is None else z_cells
    rng = np.random.default_rng(seed)
    present = rng.uniform(size=(L, L)) >= missing
    present[:x_range[0], :] = False
    present[x_range[1]:, :] = False
    outer = np.zeros((L, L, L), dtype=np.uint8)
    outer[:, :, :zc] = present[:, :, None]
    c = (K - 1) / 2.0
    r2 = (radius_frac * K) ** 2
    a = np.arange(K, dtype=np.float64) - c
    disk = (a[:, None] ** 2 + a[None, :] ** 2) <= r2
    inner = np.repeat(disk[:, :, None], K, axis=2).astype(np.uint8)
    ax = np.arange(N, dtype=np.float64)
    solid = np.zeros((N, N, N), dtype=np.uint8)
    for X in range(L):
        for Y in range(L):
            if not present[X, Y]:
                continue
            d2 = ((ax[:, None] - (X * K + c)) ** 2 + (ax[None, :] - (Y * K + c)) ** 2)
            solid[:, :, :zc * K] |= (d2 <= r2)[:, :, None].astype(np.uint8)
    return outer, inner, solid


# --------------------------------------------------------------------------
# the benchmark / parity cases (synthetic stand-ins with the paper's shapes)
# --------------------------------------------------------------------------

def case_channel(n: int = 4, chi: int = 16, tau: float = 0.8, g: float = 1e-6,
                 tol: float = 1e-10, steps: int = 200, precision: str = "fp64") -> Case:
    """Plane channel driven by a uniform body force in x (walls y=0, N-1)."""
    return Case(name=f"channel{1 << n}", n=n, tau=tau, chi=chi, tol=tol,
                g=(g, 0.0, 0.0), solid=channel_mask(n), steps=steps,
                precision=precision)


def case_porous(n: int = 6, chi: int = 64, tau: float = 0.6,
                solid_fraction: float = 0.30, seed: int = 2512 + 2,
                drho: float = 5e-4, tol: float = 1e-8, steps: int = 1000,
                precision: str = "fp32", rmin: float = 4.0, rmax: float = 8.0,
                chi_mask: Optional[int] = None) -> Case:
    """Pressure-driven flow through random spheres (x open, y/z periodic)."""
    N = 1 << n
    scale = N / 64.0
    solid = sphere_pack_mask(n, solid_fraction, max(1.0, rmin * scale),
                             max(1.5, rmax * scale), seed)
    return Case(name=f"porous{N}", n=n, tau=tau, chi=chi, tol=tol, solid=solid,
                axis_open=(1, 0, 0),
                face_bc=(BC_PRESSURE, BC_PRESSURE, 0, 0, 0, 0),
                face_val=((1.0 + drho, 0, 0), (1.0 - drho, 0, 0)) + ((0, 0, 0),) * 4,
                steps=steps, precision=precision, chi_mask=chi_mask,
                meta={"seed": seed, "solid_fraction": float(solid.mean())})


def case_vascular(n: int = 7, chi: int = 128, tau: float = 0.55,
                  u_in: float = 0.02, seed: int = 2512 + 3, tol: float = 1e-8,
                  steps: int = 500, precision: str = "bf16") -> Case:
    """Velocity inlet on x=0, pressure outlet on x=N-1, tube-tree geometry."""
    solid, segs = vascular_tree_mask(n, seed)
    return Case(name=f"vascular{1 << n}", n=n, tau=tau, chi=chi, tol=tol,
                solid=solid, axis_open=(1, 0, 0),
                face_bc=(BC_VELOCITY, BC_PRESSURE, 0, 0, 0, 0),
                face_val=((u_in, 0, 0), (1.0, 0, 0)) + ((0, 0, 0),) * 4,
                steps=steps, precision=precision,
                meta={"seed": seed, "solid_fraction": float(solid.mean()),
                      "segments": len(segs)})


def case_pinfin(n: int = 7, l: int = 3, chi: int = 64, tau: float = 0.56,
                u_in: float = 0.02, seed: int = 2512 + 6, tol: float = 1e-8,
                steps: int = 100, precision: str = "fp32") -> Case:
    """Pin-fin array (Section 4.1 stand-in): velocity inlet on x = 0, pressure
    outlet on x = N-1, y and z periodic; pins on a 2**l coarse grid
    (layer spacing L / 2**l), the mask given as its two parts."""
    outer, inner, solid = pin_fin_parts(n, l, seed)
    return Case(name=f"pinfin{1 << n}", n=n, tau=tau, chi=chi, tol=tol,
                solid=solid, axis_open=(1, 0, 0),
                face_bc=(BC_VELOCITY, BC_PRESSURE, 0, 0, 0, 0),
                face_val=((u_in, 0, 0), (1.0, 0, 0)) + ((0, 0, 0),) * 4,
                steps=steps, precision=precision, mask_parts=(outer, inner),
                meta={"seed": seed, "solid_fraction": float(solid.mean()), "l": l})


def tgv_state(n: int, u_lat: float = 0.1) -> Tuple[np.ndarray, np.ndarray]:
    """3D Taylor-Green vortex initial state of Section 4.1 in lattice units
    on the 2 pi periodic cube (x_i = 2 pi i / N): u = -U sin x cos y cos z,
    v = U cos x sin y cos z, w = 0 and the density as printed there,
    rho = 1 + (cos 2x + cos 2y) cos 2z / (16 du^2).  U = u_lat = Ma c_s is the
    lattice velocity of u_0 = 1 (Ma = 0.1 / c_s gives 0.1) and du = 1 / U
    the velocity conversion factor."""
    N = 1 << n
    x = 2.0 * np.pi * np.arange(N) / N
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    u = np.stack([-u_lat * np.sin(X) * np.cos(Y) * np.cos(Z),
                  u_lat * np.cos(X) * np.sin(Y) * np.cos(Z),
                  np.zeros_like(X)])
    rho = 1.0 + (u_lat ** 2 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * np.cos(2 * Z)
    return rho, u


def case_tgv(n: int = 5, chi: int = 32, re: float = 800.0, u_lat: float = 0.1,
             lattice: int = 15, tol: float = 1e-8, steps: int = 100,
             precision: str = "fp32") -> Case:
    """Taylor-Green vortex (Section 4.1): periodic cube, Re = u_0 L / (2 pi nu)
    = U N / (2 pi nu) in lattice units, so nu = U N / (2 pi Re) and
    tau = 3 nu + 1/2; D3Q15 as in the paper by default."""
    N = 1 << n
    nu = u_lat * N / (2.0 * np.pi * re)
    rho, u = tgv_state(n, u_lat)
    return Case(name=f"tgv{N}", n=n, tau=3.0 * nu + 0.5, chi=chi, tol=tol,
                rho_init=rho, u_init=u, steps=steps, precision=precision,
                lattice=lattice, meta={"re": re, "nu": nu, "u_lat": u_lat,
                                       "steps_per_T0": 2.0 * np.pi * N / (2.0 * np.pi * u_lat)})


def c4_cases(count: int = 48, seed: int = 2512 + 4) -> List[Case]:
    """Many independent domains of mixed size and bond dimension (seeded):
    N in {32, 64, 128}, chi in {32, 64, 128} capped at the full bond of the
    grid, tau ~ U[0.55, 0.9], half body-forced channels, half pressure-driven
    porous media (the porous geometry seeded per case); FP32 storage with
    BF16X3 contractions at chi 128, FP32 otherwise."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice([5, 6, 7]))
        full = max(min(8 ** k, 8 ** (n - k)) for k in range(1, n))
        chi = min(int(rng.choice([32, 64, 128])), full)
        tau = float(rng.uniform(0.55, 0.9))
        prec = "bf16x3" if chi == 128 else "fp32"
        if rng.uniform() < 0.5:
            c = case_channel(n=n, chi=chi, tau=tau, tol=1e-8, precision=prec)
        else:
            c = case_porous(n=n, chi=chi, tau=tau, tol=1e-8, precision=prec,
                            seed=int(rng.integers(1 << 30)))
        c.name = f"c4_{i}_{c.name}_chi{chi}"
        out.append(c)
    return out


def random_flow_state(n: int, seed: int, amp: float = 0.02,
                      drho: float = 0.01, modes: int = 2) -> Tuple[np.ndarray, np.ndarray]:
    """Smooth seeded density/velocity fields (a few random Fourier modes):
    used to start parity runs from a non-trivial state."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    x = 2.0 * np.pi * np.arange(N) / N
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    def smooth():
        out = np.zeros((N, N, N))
        for _ in range(modes):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi, size=3)
            out += (np.cos(k[0] * X + ph[0]) * np.cos(k[1] * Y + ph[1])
                    * np.cos(k[2] * Z + ph[2]))
        return out / modes
    rho = 1.0 + drho * smooth()
    u = np.stack([amp * smooth() for _ in range(3)])
    return rho, u

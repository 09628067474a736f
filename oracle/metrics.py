"""Flow metrics of Section 4.2 (test infrastructure only)."""
from __future__ import annotations

import numpy as np


def pressure_drop(rho, solid, lo, hi, rho_ref: float) -> float:
    """Delta p / p_0 = (1 / (p_0 |D|)) sum_{x in D} (p_x - p_0) with
    p = c_s^2 rho and p_0 = c_s^2 rho_ref (the density prescribed at the
    outflow), D the unmasked cells of the box lo <= x < hi."""
    box = np.zeros(rho.shape, dtype=bool)
    box[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
    if solid is not None:
        box &= ~np.asarray(solid, dtype=bool)
    cells = int(box.sum())
    if cells == 0:
        raise ValueError("the region holds no fluid cell")
    return float((rho[box] - rho_ref).sum() / (rho_ref * cells))


def kinetic_energy(f, solid=None) -> float:
    """E_kin of Section 4.2 with the density normalised to total mass 1 and
    V_c = (L/N)^3: (1 / (2 N^3)) sum_x |u_x|^2, u = j / rho on fluid cells."""
    from .lattice import get
    lat = get(f.shape[0])
    rho = f.sum(axis=0)
    j = np.einsum("ia,ixyz->axyz", lat.c.astype(np.float64), f)
    fl = rho != 0.0 if solid is None else (~np.asarray(solid, dtype=bool)) & (rho != 0.0)
    u2 = np.zeros_like(rho)
    u2[fl] = (j[:, fl] ** 2).sum(axis=0) / rho[fl] ** 2
    return 0.5 * float(u2.sum()) / rho.size


def dissipation(e, dt: float):
    """-dE/dt of a sequence of E_kin values by second-order finite
    differences (central inside, one-sided second order at the ends)."""
    return -np.gradient(np.asarray(e, dtype=np.float64), dt, edge_order=2)

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

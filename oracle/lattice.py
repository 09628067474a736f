"""Velocity sets for the oracle (test infrastructure only).

D3Q19: one rest velocity (weight 1/3), six axis velocities (1/18) and
twelve edge velocities (1/36).  D3Q15, the set of the paper's 3D runs
(Section 4.1): one rest velocity (2/9), six axis velocities (1/9) and eight
corner velocities (1/72).  Both have c_s^2 = 1/3 and are isotropic to fourth
order, so the same second-order equilibrium applies.  Opposite velocities
are stored next to each other so that opp(i) is i +/- 1.  The module-level
names are the D3Q19 set.
"""
from dataclasses import dataclass

import numpy as np

Q = 19
C = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
], dtype=np.int64)
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
OPP = np.array([0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17])
CS2 = 1.0 / 3.0

# index pairs (a, b), a <= b, of the symmetric second moment Pi_ab
PI_PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


@dataclass(frozen=True)
class Lattice:
    q: int
    c: np.ndarray
    w: np.ndarray
    opp: np.ndarray


D3Q19 = Lattice(Q, C, W, OPP)

_C15 = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 1], [-1, -1, -1], [1, 1, -1], [-1, -1, 1],
    [1, -1, 1], [-1, 1, -1], [-1, 1, 1], [1, -1, -1],
], dtype=np.int64)
_W15 = np.array([2.0 / 9.0] + [1.0 / 9.0] * 6 + [1.0 / 72.0] * 8)
_OPP15 = np.array([0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13])
D3Q15 = Lattice(15, _C15, _W15, _OPP15)


def get(q: int) -> Lattice:
    if q == 19:
        return D3Q19
    if q == 15:
        return D3Q15
    raise ValueError(f"no D3Q{q} lattice")

"""D3Q19 velocity set for the oracle (test infrastructure only).

The paper's 3D runs use D3Q15 (Section 4.1); this build runs D3Q19, the
textbook set: one rest velocity (weight 1/3), six axis velocities (1/18) and
twelve edge velocities (1/36), lattice speed of sound c_s^2 = 1/3.  Opposite
velocities are stored next to each other so that opp(i) is i +/- 1.
"""
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

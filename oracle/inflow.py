"""Time-dependent inflow of a velocity face (test infrastructure only).

Section 4.1 drives its two open-boundary cases with inflow velocities that
change in time: a ramp u_0 (1 - exp(-1.5 t)) (pin-fin array, t in units of
the flow-through time) and a pulse 0.1 + 18 t^1.5 exp(-10 t) (aneurysm, t in
seconds, velocity in m/s).  Both are members of one family

    phi(t) = c0 + c1 (1 - exp(-c2 t)) + c3 t^c4 exp(-c5 t),

which scales the face's configured velocity: u_b(t) = u_b phi(t).  The step
that starts after k steps uses t = k dt.
"""
from __future__ import annotations

import math


def inflow_scale(coef, t: float) -> float:
    c0, c1, c2, c3, c4, c5 = (float(c) for c in coef)
    v = c0 + c1 * (1.0 - math.exp(-c2 * t))
    if c3 != 0.0:
        v += c3 * (t ** c4) * math.exp(-c5 * t)
    return v


def face_velocity(case, face: int, step: int):
    """u_b of a velocity face for the step that starts after `step` steps."""
    ub = [float(v) for v in case.face_val[face]]
    prof = (case.face_profile or {}).get(face)
    if prof is None:
        return ub
    coef, dt = prof
    s = inflow_scale(coef, step * float(dt))
    return [s * v for v in ub]

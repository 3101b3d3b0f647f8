"""Referee for events whose FP64 value is ill-conditioned.

The exact |M|^2 of an event is unchanged by a rotation of the frame and by permuting
identical gluons (with their momenta), but each of these equivalent inputs sends the
FP64 arithmetic down a different rounding path.  The spread of the double-precision oracle
over such equivalent evaluations, measured against the long-double oracle, estimates how
far FP64 rounding alone can move this event's value.  A GPU value beyond the 1e-12 bar is
accepted as ill-conditioned (and counted) when it is within 3x that spread of the
long-double value; otherwise it is a failure."""
import math

import numpy as np

import oracle

TOL = 1e-12


def _rotate(p, axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    out = p.copy()
    out[..., 1:] = p[..., 1:] @ R.T
    return out


def equivalent_inputs(name, p):
    n = len(p)
    out = [p]
    for axis, ang in [((1, 2, 3), 0.7), ((-2, 1, 0.5), 2.1), ((0.3, -1, 2), 4.0)]:
        out.append(_rotate(p, axis, ang))
    if name != "ee_mumu":
        out.append(p[[1, 0] + list(range(2, n))])
        if n >= 6:
            out.append(p[[0, 1, 2, 3] + list(range(n - 1, 3, -1))])
    return out


def judge(name, p, gpu_value, params):
    """(ok, rel_to_long_double, fp64_spread) for one event"""
    ld = oracle.me(name, p, params=params, precision="long double")
    spread = max(abs(oracle.me(name, q, params=params) / ld - 1) for q in equivalent_inputs(name, p))
    rel = abs(gpu_value / ld - 1)
    return rel <= max(TOL, 3 * spread), rel, spread

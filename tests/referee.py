"""Referee for events whose FP64 value is ill-conditioned.

The exact |M|^2 of an event is unchanged by a rotation of the frame and by permuting
identical gluons (with their momenta), but each of these equivalent inputs sends the
FP64 arithmetic down a different rounding path.  The spread of an FP64 evaluation over
such equivalent inputs, measured against the long-double oracle, estimates how far FP64
rounding alone can move this event's value.

Two algorithms give two such estimates, both from the oracle alone: its Berends-Giele
recursion, and (for gg -> t t~ + up to two gluons) its sum of single Feynman diagrams
(oracle/diagrams.py), the algorithm class the GPU evaluates, whose gauge cancellations
between diagrams can make it worse conditioned on soft or collinear events.  A GPU value
beyond the 1e-12 bar is accepted as ill-conditioned (and counted) when it is within 3x
the largest spread of the long-double value; otherwise it is a failure.

A third estimate covers the input itself: phase-space points conserve momentum only up to
the rounding of their generator (the massive RAMBO step stops at |f| <= 1e-14 sqrt(s), so
energy balances to ~1e-11 GeV), and |M|^2 is defined only on exactly conserving momenta.
Two valid evaluations that route a propagator's momentum through different external
legs differ by the residue; near a soft or collinear propagator (small q^2 - m^2) that
is visible at the 1e-12 level.  The spread of the long-double oracle over the points
obtained by absorbing the residue into each particle in turn measures it."""
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
    if not name.startswith("ee_"):
        out.append(p[[1, 0] + list(range(2, n))])
        if n >= 6:
            out.append(p[[0, 1, 2, 3] + list(range(n - 1, 3, -1))])
    return out


DIAGRAM_PROCESSES = ("gg_tt", "gg_ttg", "gg_ttgg")


def judge(name, p, gpu_value, params):
    """(ok, rel_to_long_double, fp64_spread) for one event"""
    ld = oracle.me(name, p, params=params, precision="long double")
    spread = max(abs(oracle.me(name, q, params=params) / ld - 1) for q in equivalent_inputs(name, p))
    rel = abs(gpu_value / ld - 1)
    if rel > max(TOL, 3 * spread):
        spread = max(spread, conservation_spread(name, p, params, ld))
    if rel > max(TOL, 3 * spread) and name in DIAGRAM_PROCESSES:
        from oracle import diagrams
        spread = max(spread, max(abs(diagrams.diagram_me(name, q, params) / ld - 1)
                                 for q in equivalent_inputs(name, p)))
    return rel <= max(TOL, 3 * spread), rel, spread


def conservation_spread(name, p, params, ld):
    """spread of the long-double |M|^2 over the exactly conserving points made by absorbing
    the momentum residue (incoming minus outgoing) into one particle at a time"""
    p = np.asarray(p, dtype=np.float64)
    delta = p[0] + p[1] - p[2:].sum(axis=0)
    out = 0.0
    for j in range(len(p)):
        q = p.copy()
        q[j] = q[j] + delta if j >= 2 else q[j] - delta
        out = max(out, abs(oracle.me(name, q, params=params, precision="long double") / ld - 1))
    return out

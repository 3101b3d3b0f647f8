"""Soft-gluon limit of the oracle's colour-ordered amplitudes at the physical top mass: the
(n+1)-point amplitudes of g g -> t t~ + k gluons (the processes of Sec. 2) against the
n-point ones, gg_tt -> gg_ttg -> gg_ttgg -> gg_ttggg.

When gluon s of momentum k becomes soft, a colour-ordered amplitude factorises onto the
amplitude with s removed, times an eikonal factor that depends only on s's two neighbours a,
b in the colour ordering (the top, a gluon or the antitop):
    A_{n+1}(..., a, s, b, ...) -> g_s (eps(k) . J) A_n(..., a, b, ...),
    J = p_a / (p_a . k) - p_b / (p_b . k)      (all momenta outgoing; J is unchanged by p -> -p).
Since J . k = 0, |eps . J|^2 = -J^2 / 2 for either helicity, whatever the polarisation
vector's phase or gauge, and massive neighbours (the tops) included:
    -J^2 / 2 = p_a.p_b / ((p_a.k)(p_b.k)) - m_a^2 / (2 (p_a.k)^2) - m_b^2 / (2 (p_b.k)^2).
The check compares moduli, ordering by ordering, over the largest helicities, at soft
energies lambda sqrt(s)/2 for lambda = 1e-4 and 1e-5: the deviation must be small and must
fall linearly with lambda, which leaves no room for a wrong constant or neighbour.
"""
import math

import numpy as np
import pytest

import oracle
from tests import workloads as W

METRIC = np.diag([1.0, -1.0, -1.0, -1.0])


def _dot(a, b):
    return a @ METRIC @ b


def add_soft_gluon(ev, lam, direction):
    """ev plus a final-state gluon of energy lam sqrt(s)/2 along `direction`; the final state is
    boosted back to its rest frame and the beams rescaled to its mass, so momentum is conserved
    exactly and every particle stays on shell"""
    rs = ev[0, 0] + ev[1, 0]
    d = np.asarray(direction, float)
    d = d / np.linalg.norm(d)
    w = lam * rs / 2
    fin = np.vstack([ev[2:], np.concatenate([[w], w * d])])
    P = fin.sum(axis=0)
    M = math.sqrt(_dot(P, P))
    b = -P[1:] / P[0]
    b2 = b @ b
    g = 1 / math.sqrt(1 - b2)
    bp = fin[:, 1:] @ b
    out = fin.copy()
    out[:, 0] = g * (fin[:, 0] + bp)
    out[:, 1:] = fin[:, 1:] + ((g - 1) * bp / b2 + g * fin[:, 0])[:, None] * b
    beams = np.array([[M / 2, 0, 0, M / 2], [M / 2, 0, 0, -M / 2]])
    return np.vstack([beams, out])


def soft_deviation(proc_n, proc_m, lam, seed, direction):
    """max over the 3 largest helicities of proc_n, both soft helicities and every ordering of
    | |A_{n+1}| - g_s sqrt(-J^2/2) |A_n| |, relative to the largest prediction"""
    n = W.n_par(proc_n)
    ev = oracle.rambo(seed, W.sqrt_s(proc_n), W.final_masses(proc_n), 1)[0]
    ev2 = add_soft_gluon(ev, lam, direction)
    out2 = [-ev2[0], -ev2[1]] + list(ev2[2:])
    k = out2[n]
    g_s = math.sqrt(4 * math.pi * W.ALPHA_S)
    glu = [0, 1] + list(range(4, n)) + [n]       # particle index of gluon label g in proc_m
    soft = len(glu) - 1
    index_n = {tuple(int(x) for x in o): i for i, o in enumerate(oracle.orderings(proc_n))}
    _, hel = oracle.me(proc_n, ev, params=W.PARAMS, per_helicity=True)
    worst = 0.0
    for h in np.argsort(hel)[-3:]:
        A = oracle.partials(proc_n, ev, int(h), params=W.PARAMS)
        for bit in (0, 1):
            A2 = oracle.partials(proc_m, ev2, (int(h) << 1) | bit, params=W.PARAMS)
            pred = np.empty(len(A2))
            for j, o in enumerate(oracle.orderings(proc_m)):
                o = [int(x) for x in o]
                chain = [2] + [glu[x] for x in o] + [3]
                pos = o.index(soft) + 1
                a, b = chain[pos - 1], chain[pos + 1]
                J = out2[a] / _dot(out2[a], k) - out2[b] / _dot(out2[b], k)
                assert -_dot(J, J) >= 0
                parent = tuple(x for x in o if x != soft)
                pred[j] = g_s * math.sqrt(-_dot(J, J) / 2) * abs(A[index_n[parent]])
            worst = max(worst, float(np.max(np.abs(np.abs(A2) - pred)) / np.max(pred)))
    return worst


@pytest.mark.parametrize("proc_n,proc_m", [("gg_tt", "gg_ttg"), ("gg_ttg", "gg_ttgg"), ("gg_ttgg", "gg_ttggg")])
@pytest.mark.parametrize("seed,direction", [(5, (0.3, -0.5, 0.8)), (9, (-0.7, 0.2, -0.1))])
def test_soft_gluon_factorisation(proc_n, proc_m, seed, direction):
    d4 = soft_deviation(proc_n, proc_m, 1e-4, seed, direction)
    d5 = soft_deviation(proc_n, proc_m, 1e-5, seed, direction)
    assert d5 < 2e-4, (d4, d5)
    assert 5 < d4 / d5 < 20, (d4, d5)          # linear approach to the eikonal limit


def test_soft_limit_tells_neighbours_apart():
    """the eikonal factor of the wrong neighbours misses the limit by O(1)"""
    proc_n, proc_m, n = "gg_ttg", "gg_ttgg", 5
    ev = oracle.rambo(5, W.sqrt_s(proc_n), W.final_masses(proc_n), 1)[0]
    ev2 = add_soft_gluon(ev, 1e-5, (0.3, -0.5, 0.8))
    out2 = [-ev2[0], -ev2[1]] + list(ev2[2:])
    k = out2[n]
    g_s = math.sqrt(4 * math.pi * W.ALPHA_S)
    h = int(np.argmax(oracle.me(proc_n, ev, params=W.PARAMS, per_helicity=True)[1]))
    A = oracle.partials(proc_n, ev, h, params=W.PARAMS)
    A2 = oracle.partials(proc_m, ev2, h << 1, params=W.PARAMS)
    o2 = [tuple(int(x) for x in o) for o in oracle.orderings(proc_m)]
    o1 = [tuple(int(x) for x in o) for o in oracle.orderings(proc_n)]
    # soft gluon (label 3) between the top and gluon label 0: ordering (3, 0, 1, 2) of (0, 1, 2)
    j, i = o2.index((3, 0, 1, 2)), o1.index((0, 1, 2))
    ratio = abs(A2[j]) / abs(A[i]) / g_s

    def eik(a, b):
        J = out2[a] / _dot(out2[a], k) - out2[b] / _dot(out2[b], k)
        return math.sqrt(-_dot(J, J) / 2)
    assert abs(ratio / eik(2, 0) - 1) < 1e-3
    assert abs(ratio / eik(0, 1) - 1) > 0.1 and abs(ratio / eik(2, 1) - 1) > 0.1

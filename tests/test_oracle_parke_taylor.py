"""Closed-form pins of the oracle's colour-ordered amplitudes for g g -> t t~ + 0..3 gluons
(the processes of Sec. 2) in the massless-quark limit m_t = 0, all particles outgoing
(incoming momenta and helicities reversed):

* tree amplitudes with fewer than two negative or fewer than two positive helicities vanish,
  and so do those whose quark pair has equal helicities (massless helicity conservation on
  the quark line);
* maximally helicity-violating amplitudes (exactly two negative helicities: one of the quark
  pair and one gluon j) have the Parke-Taylor modulus
      |A(q, g_s1, ..., g_sk, q~)| = (sqrt(2) g_s)^(n-2) |<f j>|^3 |<f' j>| / prod_cyclic |<a b>|,
  with f the negative-helicity member of the quark pair, f' the other and |<a b>| = sqrt|2 a.b|;
  their conjugates (exactly two positive helicities) have the same modulus with the roles of
  the helicities swapped.  The moduli need no phase convention, and the factor (sqrt(2) g_s)^(n-2)
  is fixed by the colour generators' normalisation Tr(T^a T^b) = delta^ab / 2.

Every MHV helicity of gg_ttgg and gg_ttggg is checked, ordering by ordering, so a dropped
diagram, a wrong vertex sign or a transposed colour ordering fails here.  At n = 7 a few
orderings cancel strongly (the long-double oracle moves them by ~1e-9), hence the tolerance
relative to the helicity's largest amplitude there.
"""
import math

import numpy as np
import pytest

import oracle
from tests import workloads as W

PARAMS_MASSLESS = (0.0, W.ALPHA_EM, W.ALPHA_S)
# absolute deviation from the closed form, relative to the largest amplitude of the helicity
TOL = {4: 1e-13, 5: 1e-13, 6: 1e-12, 7: 1e-9}


def _events(proc, seed, n_evt):
    n = W.n_par(proc)
    return oracle.rambo(seed, 1500.0, [0.0] * (n - 2), n_evt)


def _outgoing(ev):
    return [-ev[0], -ev[1]] + [ev[i] for i in range(2, len(ev))]


def _mandelstam(out):
    def s(i, j):
        a, b = out[i], out[j]
        return abs(2.0 * (a[0] * b[0] - a[1:] @ b[1:]))
    return s


@pytest.mark.parametrize("proc,seed", [("gg_tt", 3), ("gg_ttg", 3), ("gg_ttgg", 3), ("gg_ttgg", 8),
                                       ("gg_ttggg", 3), ("gg_ttggg", 8)])
def test_mhv_moduli_and_vanishing_helicities(proc, seed):
    n = W.n_par(proc)
    g_s = math.sqrt(4 * math.pi * W.ALPHA_S)
    glu = [0, 1] + list(range(4, n))            # particle index of gluon label g
    for ev in _events(proc, seed, 1):
        out = _outgoing(ev)
        s = _mandelstam(out)
        _, hel = oracle.me(proc, ev, params=PARAMS_MASSLESS, per_helicity=True)
        amp_scale = math.sqrt(hel.max())
        chains = [[2] + [glu[g] for g in sig] + [3] for sig in oracle.orderings(proc)]
        cyc = np.array([np.prod([math.sqrt(s(c[k], c[(k + 1) % n])) for k in range(n)]) for c in chains])
        n_mhv = 0
        for h in range(1 << n):
            lam = [2 * ((h >> (n - 1 - i)) & 1) - 1 for i in range(n)]
            lam_out = [-lam[0], -lam[1]] + lam[2:]
            neg = [i for i in range(n) if lam_out[i] < 0]
            pos = [i for i in range(n) if lam_out[i] > 0]
            A = oracle.partials(proc, ev, h, params=PARAMS_MASSLESS)
            if lam_out[2] == lam_out[3] or len(neg) < 2 or len(pos) < 2:
                # helicity conservation on the quark line; all-plus and one-minus amplitudes
                assert np.max(np.abs(A)) <= 1e-13 * amp_scale, (proc, h)
                continue
            odd = neg if len(neg) == 2 else (pos if len(pos) == 2 else None)
            if odd is None:
                continue                          # NMHV (n >= 6): no one-line closed form
            f = 2 if 2 in odd else 3
            j = odd[0] if odd[1] == f else odd[1]
            num = s(f, j) ** 1.5 * s(5 - f, j) ** 0.5
            pred = (math.sqrt(2.0) * g_s) ** (n - 2) * num / cyc
            amax = np.max(np.abs(A))
            assert amax > 0
            assert np.max(np.abs(np.abs(A) - pred)) <= TOL[n] * amax, (proc, h)
            n_mhv += 1
        # MHV and conjugate helicities with opposite quark helicities: 2 (quark pair) x (n-2)
        # (negative gluon) each; at n = 4 the two sets coincide
        assert n_mhv == (2 * (n - 2) if n == 4 else 4 * (n - 2))


def test_mhv_pin_catches_a_wrong_ordering():
    """the closed form tells orderings apart: compared against the orderings in reverse, it fails"""
    proc, n = "gg_ttgg", 6
    ev = _events(proc, 3, 1)[0]
    s = _mandelstam(_outgoing(ev))
    glu = [0, 1, 4, 5]
    chains = [[2] + [glu[g] for g in sig] + [3] for sig in oracle.orderings(proc)]
    cyc = np.array([np.prod([math.sqrt(s(c[k], c[(k + 1) % n])) for k in range(n)]) for c in chains])
    # helicity: gluon 0 incoming + (outgoing -), t -, the rest outgoing +: f = 2, j = 0
    lam = [1, -1, -1, 1, 1, 1]
    h = sum(((l + 1) // 2) << (n - 1 - i) for i, l in enumerate(lam))
    A = np.abs(oracle.partials(proc, ev, h, params=PARAMS_MASSLESS))
    ratio = A * cyc
    assert np.max(np.abs(ratio / ratio[0] - 1)) < 1e-12
    assert np.max(np.abs((A[::-1] * cyc) / ratio[0] - 1)) > 1e-3


@pytest.mark.parametrize("proc", ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"])
def test_helicity_filter_keeps_the_non_vanishing_configurations(proc):
    """at m_t = 0 the filter keeps opposite quark helicities with at least two of each sign
    among the all-outgoing helicities, 2 (2^(n-2) - 2) configurations, and no others"""
    n = W.n_par(proc)
    good = oracle.good_helicities(proc, 1500.0, [0.0] * (n - 2), params=PARAMS_MASSLESS,
                                  n_events=32 if n == 7 else 256)
    want = []
    for h in range(1 << n):
        lam = [2 * ((h >> (n - 1 - i)) & 1) - 1 for i in range(n)]
        lam_out = [-lam[0], -lam[1]] + lam[2:]
        if lam_out[2] != lam_out[3] and 2 <= lam_out.count(-1) <= n - 2:
            want.append(h)
    assert len(want) == 2 * (2 ** (n - 2) - 2)
    assert sorted(int(h) for h in good) == want


def _angle(p, q):
    """spinor product <p q> of two positive-energy massless momenta (one fixed phase convention;
    every particle's phase appears once in each cyclic product below, so ratios do not depend on it)"""
    pp, pm = p[0] + p[3], p[0] - p[3]
    qp, qm = q[0] + q[3], q[0] - q[3]
    ep = (p[1] + 1j * p[2]) / math.sqrt(pp * pm) if pp * pm > 0 else 1.0
    eq = (q[1] + 1j * q[2]) / math.sqrt(qp * qm) if qp * qm > 0 else 1.0
    return math.sqrt(pm * qp) * ep - math.sqrt(pp * qm) * eq


def mhv_colour_summed(proc, ev, colour):
    """{helicity index: colour-summed |M_h|^2} of every MHV and conjugate-MHV helicity at m_t = 0:
    A_sigma = c N / P_sigma with P_sigma the cyclic product of <a b> along (t, gluons of sigma, t~)
    and |c| = (sqrt(2) g_s)^(n-2), |N|^2 = s_fj^3 s_f'j, so
    |M_h|^2 = (2 g_s^2)^(n-2) |N|^2 sum_{sigma,sigma'} conj(1/P_sigma) C_{sigma sigma'} (1/P_sigma');
    the conjugate amplitudes give the complex conjugate sum, the same real number.  Crossing an
    incoming momentum multiplies its spinors by a phase, which cancels in every ratio."""
    n = len(ev)
    g_s = math.sqrt(4 * math.pi * W.ALPHA_S)
    glu = [0, 1] + list(range(4, n))
    chains = [[2] + [glu[g] for g in o] + [3] for o in oracle.orderings(proc)]
    v = 1.0 / np.array([np.prod([_angle(ev[c[k]], ev[c[(k + 1) % n]]) for k in range(n)]) for c in chains])
    colour_sum = float(np.real(np.conj(v) @ colour @ v))
    s = _mandelstam(_outgoing(ev))
    out = {}
    for h in range(1 << n):
        lam = [2 * ((h >> (n - 1 - i)) & 1) - 1 for i in range(n)]
        lam_out = [-lam[0], -lam[1]] + lam[2:]
        neg = [i for i in range(n) if lam_out[i] < 0]
        pos = [i for i in range(n) if lam_out[i] > 0]
        if lam_out[2] == lam_out[3]:
            continue
        odd = neg if len(neg) == 2 else (pos if len(pos) == 2 else None)
        if odd is None:
            continue
        f = 2 if 2 in odd else 3
        j = odd[0] if odd[1] == f else odd[1]
        out[h] = (2 * g_s ** 2) ** (n - 2) * s(f, j) ** 3 * s(5 - f, j) * colour_sum
    return out


@pytest.mark.parametrize("proc", ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"])
def test_mhv_colour_summed_closed_form(proc):
    """the colour-summed |M_h|^2 of every MHV helicity equals the Parke-Taylor closed form with
    complex spinor products and the colour matrix"""
    n = W.n_par(proc)
    C = oracle.colour_matrix(proc)
    for ev in _events(proc, 4, 2):
        _, hel = oracle.me(proc, ev, params=PARAMS_MASSLESS, per_helicity=True)
        want = mhv_colour_summed(proc, ev, C)
        assert len(want) == (2 * (n - 2) if n == 4 else 4 * (n - 2))
        for h, v in want.items():
            assert abs(hel[h] / v - 1) <= 1e-12, (proc, h, hel[h], v)

"""Pins of the oracle's per-event helicity and colour-flow choice (the two per-event records
the paper, Sec. 4, lists as missing from its event files).

* draw: against an independent formula (binary search on the running sums) and the
  frequencies of a stratified grid of uniforms;
* helicity weights of ee -> mumu: exactly four non-zero, e^4 (1 +- cos)^2 (cos between e- and
  mu-), from helicity conservation of the massless vector current;
* leading-colour weights of gg -> tt~: w_(1,2) = 8 g^4 (tau2/tau1) F and w_(2,1) =
  8 g^4 (tau1/tau2) F, F = tau1^2 + tau2^2 + rho - rho^2/(4 tau1 tau2) (the colour-ordered
  form of Combridge's result: (16/3)(w_12 + w_21) is exactly its 1/(6 tau1 tau2) term);
* Bose symmetry: swapping the incoming gluons permutes the flows' weights.
"""
import numpy as np
import pytest

import oracle
from tests import workloads as W


def test_draw_matches_binary_search_and_frequencies():
    rng = np.random.default_rng(4)
    for _ in range(200):
        n = int(rng.integers(1, 9))
        w = rng.random(n) * (rng.random(n) > 0.3)
        if w.sum() == 0:
            continue
        for r in rng.random(5):
            cum = np.cumsum(w)
            j = int(np.searchsorted(cum, r * cum[-1], side="right"))
            assert oracle.draw(w, r) == j and w[j] > 0
    w = np.array([0.1, 0.0, 0.3, 0.6, 0.0])
    N = 10000
    counts = np.bincount([oracle.draw(w, (i + 0.5) / N) for i in range(N)], minlength=5)
    assert np.all(np.abs(counts / N - w / w.sum()) <= 1.0 / N)
    assert oracle.draw(w, 0.0) == 0 and oracle.draw(w, np.nextafter(1.0, 0.0)) == 3


def test_ee_mumu_helicity_weights_closed_form():
    e4 = (4 * np.pi * W.ALPHA_EM) ** 2
    p = oracle.rambo(0, 500.0, [0.0, 0.0], 5)
    for ev in p:
        w = oracle.helicity_weights("ee_mumu", ev, params=W.PARAMS)
        pe, pm = ev[1, 1:], ev[3, 1:]
        c = pe @ pm / (np.linalg.norm(pe) * np.linalg.norm(pm))
        # bits (e+, e-, mu+, mu-), 1 = helicity +1
        want = np.zeros(16)
        for h in range(16):
            b = [(h >> (3 - i)) & 1 for i in range(4)]
            if b[0] != b[1] and b[2] != b[3]:
                want[h] = e4 * (1 + c) ** 2 if b[1] == b[3] else e4 * (1 - c) ** 2
        assert np.allclose(w, want, rtol=1e-12, atol=1e-14 * e4)


@pytest.mark.parametrize("mt", [173.0, 1e-3])
def test_gg_tt_colour_weights_closed_form(mt):
    prm = (mt, W.ALPHA_EM, W.ALPHA_S)
    g4 = (4 * np.pi * W.ALPHA_S) ** 2
    assert oracle.orderings("gg_tt") == [(0, 1), (1, 0)]
    p = oracle.rambo(1, 1500.0, [mt, mt], 6)
    mink = lambda a, b: a[0] * b[0] - a[1:] @ b[1:]
    for ev in p:
        w = oracle.colour_weights("gg_tt", ev, params=prm)
        p1, p2, p3, p4 = ev
        s, t, u = mink(p1 + p2, p1 + p2), mink(p1 - p3, p1 - p3), mink(p1 - p4, p1 - p4)
        tau1, tau2, rho = (mt * mt - t) / s, (mt * mt - u) / s, 4 * mt * mt / s
        F = tau1 ** 2 + tau2 ** 2 + rho - rho ** 2 / (4 * tau1 * tau2)
        assert w[0] == pytest.approx(8 * g4 * tau2 / tau1 * F, rel=1e-12)
        assert w[1] == pytest.approx(8 * g4 * tau1 / tau2 * F, rel=1e-12)
        # (16/3)(w_12 + w_21) = (128/3) g^4 F (1/(tau1 tau2) - 2), since tau1 + tau2 = 1: its
        # 1/(tau1 tau2) part is the 256 g^4 F / (6 tau1 tau2) term of Combridge's formula
        # (summed over colours and spins)
        lc = 16.0 / 3.0 * (w[0] + w[1])
        assert lc == pytest.approx(g4 * F * (128.0 / (3 * tau1 * tau2) - 256.0 / 3.0), rel=1e-12)


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg"])
def test_colour_weights_bose_symmetry(name):
    p = oracle.rambo(2, 1500.0, W.final_masses(name), 2)
    orders = oracle.orderings(name)
    pos = {o: k for k, o in enumerate(orders)}
    swap = {0: 1, 1: 0}
    for ev in p:
        w = oracle.colour_weights(name, ev, params=W.PARAMS)
        q = ev.copy()
        q[[0, 1]] = ev[[1, 0]]
        wq = oracle.colour_weights(name, q, params=W.PARAMS)
        for k, o in enumerate(orders):
            o2 = tuple(swap.get(int(x), int(x)) for x in o)
            assert wq[pos[o2]] == pytest.approx(w[k], rel=1e-11)

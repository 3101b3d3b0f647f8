"""Pins of the oracle's single-diagram machinery (oracle/diagrams.py), used for the
single-diagram-enhancement channel weights:

* diagram and amplitude-entry counts 3/16/123/1240 and 3/18/159/1890 (the published
  diagram counts of gg -> t t~ + 0..3 g; a four-gluon vertex has three colour structures);
* colour weights of gg -> t t~: t- and u-channel diagrams (t^a t^b)_{ij}: Tr(t^a t^b t^b t^a)
  = N C_F^2 = 16/3; s-channel f^{abc} t^c: C_A (N^2 - 1) / 2 = 12;
* completeness: the coherent sum over every diagram and colour structure, squared and
  summed over explicit colours and helicities, equals the Berends-Giele |M|^2 (an
  independent algorithm, itself pinned by the closed forms);
* the channel weights of an event sum to one.
"""
import numpy as np
import pytest

import oracle
from oracle import diagrams as Dg
from tests import workloads as W


@pytest.mark.parametrize("ng,nd,ne", [(2, 3, 3), (3, 16, 18), (4, 123, 159), (5, 1240, 1890)])
def test_diagram_counts(ng, nd, ne):
    ds = Dg.diagrams(ng)
    assert len(ds) == nd
    assert sum(len(Dg.structures(d)) for d in ds) == ne
    name = {2: "gg_tt", 3: "gg_ttg", 4: "gg_ttgg", 5: "gg_ttggg"}[ng]
    assert len({Dg.descriptor(name, d) for d in ds}) == nd     # internal lines identify a diagram


def test_gg_tt_colour_weights():
    K = Dg.colour_weights_K("gg_tt")
    by = {Dg.descriptor("gg_tt", d): k for (d, s), k in zip(Dg.entries("gg_tt"), K)}
    # particles (g0, g1, t, t~): t-channel line {1, 2}, u-channel {1, 3}, s-channel gluon {2, 3}
    assert by[(0b0110,)] == pytest.approx(16 / 3, rel=1e-14)
    assert by[(0b1010,)] == pytest.approx(16 / 3, rel=1e-14)
    assert by[(0b1100,)] == pytest.approx(12.0, rel=1e-14)


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg"])
def test_coherent_sum_of_diagrams_is_the_matrix_element(name):
    ng = oracle.n_par(name) - 2
    ents = Dg.entries(name)
    CF = np.array([Dg.colour_tensor(d, s, ng).ravel() for d, s in ents])
    p = oracle.rambo(3, 1500.0, W.final_masses(name), 1)[0]
    tot = 0.0
    for h in range(1 << oracle.n_par(name)):
        L = np.array([Dg.lorentz(name, p, h, d, s, W.PARAMS) for d, s in ents])
        tot += np.sum(np.abs(L @ CF) ** 2)
    assert tot / 256 == pytest.approx(oracle.me(name, p, params=W.PARAMS), rel=1e-12)


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg"])
def test_channel_weights_sum_to_one(name):
    p = oracle.rambo(4, 1500.0, W.final_masses(name), 1)[0]
    Wd = Dg.diagram_weights(name, p, W.PARAMS)
    assert len(Wd) == {"gg_tt": 3, "gg_ttg": 16}[name]
    f = np.array(list(Wd.values())) / sum(Wd.values())
    assert np.all(f > 0) and f.sum() == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg"])
def test_diagram_jamps_equal_berends_giele_partials(name):
    """projecting every diagram's colour tensor on the colour strings gives flow
    coefficients whose jamps sum_e c[e, sigma] L_e equal the Berends-Giele colour-ordered
    amplitudes A(sigma) flow by flow (two algorithms of the oracle); the diagram-sum |M|^2
    equals the oracle's"""
    p = oracle.rambo(7, 1500.0, W.final_masses(name), 1)[0]
    c = Dg.flow_coefficients(name)
    ents = Dg.entries(name)
    nh = 1 << oracle.n_par(name)
    scale = np.sqrt(oracle.me(name, p, params=W.PARAMS) * 256 / nh)   # typical |A| (helicities can vanish)
    for h in (0, 5, nh - 3):
        L = np.array([Dg.lorentz(name, p, h, d, s, W.PARAMS) for d, s in ents])
        J = L @ c
        A = oracle.partials(name, p, h, params=W.PARAMS)
        assert np.max(np.abs(J - A)) <= 1e-12 * scale
    assert Dg.diagram_me(name, p, W.PARAMS) == pytest.approx(oracle.me(name, p, params=W.PARAMS), rel=1e-12)


def test_golden_gg_ttggg_channel_tables_match_oracle():
    """tests/golden/gg_ttggg_channel_tables.json (the oracle's gg_ttggg colour weights and
    helicity filter, precomputed by the script beside it) against the oracle: entry order and
    internal lines, a sample of K_ds, and the filter's outcome at m_t = 173 GeV (massive tops:
    no helicity combination vanishes identically, so all 128 are kept)"""
    import json
    import os
    name = "gg_ttggg"
    tab = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "gg_ttggg_channel_tables.json")))
    ents = Dg.entries(name)
    assert len(ents) == len(tab["entries"]) == 1890
    assert [tuple(e["lines"]) for e in tab["entries"]] == [Dg.descriptor(name, d) for d, _ in ents]
    assert [tuple(e["assign"]) for e in tab["entries"]] == [tuple(s) for _, s in ents]
    for i in range(0, len(ents), 61):
        d, s = ents[i]
        assert np.sum(np.abs(Dg.colour_tensor(d, s, 5)) ** 2) == pytest.approx(tab["entries"][i]["K"], rel=1e-13)
    assert tab["good_helicities"] == list(range(128))

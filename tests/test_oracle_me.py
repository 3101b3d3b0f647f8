"""Pins of the oracle's matrix elements (CPU only).

Each check is fixed by mathematics, not by the oracle itself:
  - closed forms of the 2 -> 2 processes (textbook results, quoted in each test);
  - the colour-dressed brute force over every explicit colour assignment, which uses
    f^{abc} and t^a directly and no colour decomposition or colour matrix;
  - the decomposition identity M(colours) = sum_s (T^s)_{ij} A(s) at explicit colours;
  - gauge invariance of every colour-ordered amplitude (eps -> k gives zero);
  - Lorentz invariance, Bose symmetry and independence of the polarisation basis;
  - the long-double build agreeing with the double build.
"""
import math

import numpy as np
import pytest

import oracle
from tests import workloads as W

ALPHA = W.ALPHA_EM
GS2 = 4 * math.pi * W.ALPHA_S
E2 = 4 * math.pi * ALPHA


def two_body(rs, m, cth, phi=0.3):
    E = rs / 2
    p = math.sqrt(E * E - m * m)
    sth = math.sqrt(1 - cth * cth)
    k3 = np.array([E, p * sth * math.cos(phi), p * sth * math.sin(phi), p * cth])
    k4 = np.array([E, -k3[1], -k3[2], -k3[3]])
    return np.array([[E, 0, 0, E], [E, 0, 0, -E], k3, k4])


def mandelstam(p):
    d = lambda a: a[0] ** 2 - a[1:] @ a[1:]
    return d(p[0] + p[1]), d(p[0] - p[2]), d(p[0] - p[3])


COS = [-0.93, -0.4, 0.0, 0.5, 0.77]


@pytest.mark.parametrize("c", COS)
def test_ee_mumu_closed_form(c):
    """photon exchange, massless: <|M|^2> = 2 e^4 (t^2 + u^2) / s^2"""
    p = two_body(500.0, 0.0, c)
    s, t, u = mandelstam(p)
    assert oracle.me("ee_mumu", p) == pytest.approx(2 * E2 ** 2 * (t * t + u * u) / s ** 2, rel=1e-14)


def test_ee_mumu_worked_values():
    # e^4 at cos(theta) = 0 and (5/4) e^4 at cos(theta) = 1/2 for alpha = 1/132.507
    assert oracle.me("ee_mumu", two_body(500.0, 0, 0.0)) == pytest.approx(E2 ** 2, rel=1e-14)
    assert oracle.me("ee_mumu", two_body(500.0, 0, 0.5)) == pytest.approx(1.25 * E2 ** 2, rel=1e-14)


def test_ee_mumu_helicity_conservation():
    """massless QED: only the 4 helicity configurations with opposite e+e- and opposite
    mu+mu- helicities are non-zero"""
    p = oracle.rambo(0, 500.0, (0, 0), 3)
    for ev in p:
        v, hel = oracle.me("ee_mumu", ev, per_helicity=True)
        nz = [h for h in range(16) if hel[h] > 1e-20 * v]
        assert nz == [0b0101, 0b0110, 0b1001, 0b1010]
        assert sum(hel) / 4 == pytest.approx(v, rel=1e-15)


@pytest.mark.parametrize("c", COS)
def test_gg_gg_closed_form(c):
    """<|M|^2> = (9/2) g^4 (3 - tu/s^2 - su/t^2 - st/u^2)"""
    p = two_body(1500.0, 0.0, c)
    s, t, u = mandelstam(p)
    want = 4.5 * GS2 ** 2 * (3 - t * u / s ** 2 - s * u / t ** 2 - s * t / u ** 2)
    assert oracle.me("gg_gg", p) == pytest.approx(want, rel=1e-13)


def combridge(s, t, u, m):
    """gg -> QQbar, Combridge (1979), averaged form as in Ellis-Stirling-Webber:
    g^4 (1/(6 t1 t2) - 3/8)(t1^2 + t2^2 + rho - rho^2/(4 t1 t2))"""
    t1 = (m * m - t) / s
    t2 = (m * m - u) / s
    rho = 4 * m * m / s
    return GS2 ** 2 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 * t1 + t2 * t2 + rho - rho * rho / (4 * t1 * t2))


@pytest.mark.parametrize("c", COS)
def test_gg_tt_combridge(c):
    p = two_body(1500.0, 173.0, c)
    s, t, u = mandelstam(p)
    assert oracle.me("gg_tt", p) == pytest.approx(combridge(s, t, u, 173.0), rel=1e-13)


def test_gg_tt_threshold():
    """at threshold (beta -> 0) the averaged |M|^2 tends to 7/48 g^4"""
    m = 173.0
    p = two_body(2 * m + 1e-6, m, 0.3)
    assert oracle.me("gg_tt", p) == pytest.approx(7 / 48 * GS2 ** 2, rel=1e-6)


def test_gg_tt_massless_limit():
    """m -> 0: g^4 [(t^2+u^2)/(6tu) - 3(t^2+u^2)/(8 s^2)] (gg -> q qbar)"""
    m = 1e-4
    for c in (-0.6, 0.1, 0.8):
        p = two_body(1500.0, m, c)
        s, t, u = mandelstam(p)
        want = GS2 ** 2 * ((t * t + u * u) / (6 * t * u) - 3 * (t * t + u * u) / (8 * s * s))
        got = oracle.me("gg_tt", p, params=(m, ALPHA, W.ALPHA_S))
        assert got == pytest.approx(want, rel=1e-8)


@pytest.mark.parametrize("proc,nev", [("gg_tt", 4), ("gg_gg", 2), ("gg_ttg", 2)])
def test_brute_force_colour_sum(proc, nev):
    """colour matrix and colour-ordered recursion == explicit sum over every colour of
    the colour-dressed amplitude"""
    p = oracle.rambo(11, W.sqrt_s(proc), W.final_masses(proc), nev)
    for ev in p:
        assert oracle.me(proc, ev) == pytest.approx(oracle.me_brute_colour(proc, ev), rel=1e-13)


def nonzero_colours(proc, ev, rng, ng, n_q, scale):
    for _ in range(4000):
        h = int(rng.integers(1 << len(ev)))
        cols = list(rng.integers(0, 8, ng)) + list(rng.integers(0, 3, n_q))
        d, c = oracle.amp_explicit_colour(proc, ev, h, cols)
        if abs(d) > 1e-3 * scale:
            return d, c
    raise AssertionError("no non-zero colour assignment found")


@pytest.mark.parametrize("proc", ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg", "gg_gg"])
def test_decomposition_at_explicit_colours(proc):
    rng = np.random.default_rng(5)
    ng = 4 if proc == "gg_gg" else W.n_par(proc) - 2
    n_q = 0 if proc == "gg_gg" else 2
    p = oracle.rambo(13, W.sqrt_s(proc), W.final_masses(proc), 3)
    for ev in p:
        # typical size of one colour/helicity amplitude
        scale = math.sqrt(oracle.me(proc, ev) * 256 / (1 << len(ev)) / (8 ** ng * 3 ** n_q))
        for _ in range(4):
            d, c = nonzero_colours(proc, ev, rng, ng, n_q, scale)
            assert abs(d - c) <= 1e-13 * abs(d)


@pytest.mark.parametrize("proc", ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg", "gg_gg"])
def test_gauge_invariance(proc):
    """eps(k) -> k/k0 for any one gluon makes every colour-ordered amplitude vanish"""
    ng = 4 if proc == "gg_gg" else W.n_par(proc) - 2
    p = oracle.rambo(17, W.sqrt_s(proc), W.final_masses(proc), 2)
    gidx = [0, 1, 2, 3] if proc == "gg_gg" else [0, 1] + list(range(4, W.n_par(proc)))
    for ev in p:
        _, hel = oracle.me(proc, ev, per_helicity=True)
        for h in np.argsort(hel)[-3:]:
            A = oracle.partials(proc, ev, int(h))
            scale = np.max(np.abs(A))
            for g in range(ng):
                k0 = ev[gidx[g], 0]
                G = oracle.partials(proc, ev, int(h), gauge_gluon=g) / k0
                assert np.max(np.abs(G)) <= 1e-12 * scale


def boost(p, beta):
    b = np.asarray(beta, dtype=float)
    b2 = b @ b
    g = 1 / math.sqrt(1 - b2)
    out = p.copy()
    bp = p[..., 1:] @ b
    out[..., 0] = g * (p[..., 0] + bp)
    out[..., 1:] = p[..., 1:] + ((g - 1) * bp / b2 + g * p[..., 0])[..., None] * b
    return out


def rotate(p, axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    out = p.copy()
    out[..., 1:] = p[..., 1:] @ R.T
    return out


@pytest.mark.parametrize("proc", W.ALL + ["gg_gg", "ee_mumu_z"])
def test_lorentz_invariance(proc):
    p = oracle.rambo(19, W.sqrt_s(proc), W.final_masses(proc), 3 if proc != "gg_ttggg" else 1)
    for ev in p:
        ref = oracle.me(proc, ev)
        for beta, axis, ang in [((0.3, -0.5, 0.6), (1, 2, 3), 0.7), ((0.0, 0.0, -0.9), (0, 1, 0), 2.0)]:
            q = rotate(boost(ev, beta), axis, ang)
            assert oracle.me(proc, q) == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("proc", ["gg_ttg", "gg_ttgg", "gg_ttggg"])
def test_bose_symmetry(proc):
    """|M|^2 is symmetric under exchanging the incoming gluons and under permuting the
    final-state gluons"""
    n = W.n_par(proc)
    p = oracle.rambo(23, W.sqrt_s(proc), W.final_masses(proc), 2 if proc != "gg_ttggg" else 1)
    for ev in p:
        ref = oracle.me(proc, ev)
        swap_in = ev[[1, 0] + list(range(2, n))]
        assert oracle.me(proc, swap_in) == pytest.approx(ref, rel=1e-12)
        if n >= 6:
            perm = [0, 1, 2, 3] + list(range(n - 1, 3, -1))
            assert oracle.me(proc, ev[perm]) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("proc", W.QCD + ["gg_gg"])
def test_polarisation_basis_independence(proc):
    """helicity basis vs linear gluon polarisations and top spin along z"""
    p = oracle.rambo(29, W.sqrt_s(proc), W.final_masses(proc), 2 if proc != "gg_ttggg" else 1)
    for ev in p:
        assert oracle.me(proc, ev, basis=1) == pytest.approx(oracle.me(proc, ev), rel=1e-12)


@pytest.mark.parametrize("proc", W.ALL + ["gg_gg", "ee_mumu_z"])
def test_long_double_build_agrees(proc):
    p = oracle.rambo(31, W.sqrt_s(proc), W.final_masses(proc), 2 if proc != "gg_ttggg" else 1)
    for ev in p:
        a = oracle.me(proc, ev)
        b = oracle.me(proc, ev, precision="long double")
        assert a == pytest.approx(b, rel=1e-12)


def test_batch_matches_single():
    p = oracle.rambo(37, 1500.0, W.final_masses("gg_ttg"), 24)
    b = oracle.me_batch("gg_ttg", p, threads=3)
    for i in range(24):
        assert b[i] == oracle.me("gg_ttg", p[i])


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg"])
def test_oracle_alpha_s_power(name):
    """every tree amplitude of these processes has n_par - 2 strong couplings: the oracle,
    which recomputes every vertex at the given alpha_s, scales as alpha_s^(n_par - 2)"""
    p = oracle.rambo(5, 1500.0, W.final_masses(name), 2)
    n = oracle.n_par(name) - 2
    for ev in p:
        a = oracle.me(name, ev, params=(W.M_TOP, W.ALPHA_EM, 0.118))
        b = oracle.me(name, ev, params=(W.M_TOP, W.ALPHA_EM, 0.2))
        assert b / a == pytest.approx((0.2 / 0.118) ** n, rel=1e-12)


@pytest.mark.parametrize("rs", [500.0, 91.188, 200.0, 60.0])
def test_ee_mumu_z_closed_form(rs):
    """e+e- -> mu+mu- through photon and Z, massless: the textbook helicity amplitudes
    |M_ij|^2 = |A_ij|^2 (1 +- cos)^2 (+ when e- and mu- have the same helicity), with
    A_ij = e^2 Q_e Q_mu + (e^2 / (s_W^2 c_W^2)) g_i g_j s / (s - M_Z^2 + i M_Z Gamma_Z),
    g_L = T3 - Q s_W^2, g_R = -Q s_W^2; averaged |M|^2 = (1/4) sum_ij |M_ij|^2"""
    MZ, WZ, MW = 91.188, 2.441404, 80.419
    sw2 = 1 - MW ** 2 / MZ ** 2
    e2 = 4 * np.pi * W.ALPHA_EM
    gl, gr = -0.5 + sw2, sw2
    p = oracle.rambo(6, rs, [0.0, 0.0], 6)
    for ev in p:
        s = rs * rs
        chi = s / (s - MZ ** 2 + 1j * MZ * WZ)
        pe, pm = ev[1, 1:], ev[3, 1:]
        c = pe @ pm / (np.linalg.norm(pe) * np.linalg.norm(pm))
        tot = 0.0
        for gi in (gl, gr):
            for gj in (gl, gr):
                A = e2 + e2 / (sw2 * (1 - sw2)) * gi * gj * chi
                tot += abs(A) ** 2 * (1 + (c if gi == gj else -c)) ** 2
        assert oracle.me("ee_mumu_z", ev, params=W.PARAMS) == pytest.approx(tot / 4, rel=1e-12)
        # photon only: the ee_mumu process
        assert abs(oracle.ee_z_amplitude(ev, 0b0101, 1, W.PARAMS)) ** 2 == pytest.approx(
            abs(oracle.ee_z_amplitude(ev, 0b1010, 1, W.PARAMS)) ** 2, rel=1e-12)

"""Pins of the oracle's building blocks (CPU only): the Clifford algebra, completeness of
the external states in both bases, the SU(3) structure constants, and the colour
matrices' exact values and properties."""
import itertools
import math

import numpy as np
import pytest

import oracle

G = np.diag([1.0, -1.0, -1.0, -1.0])


def test_clifford_algebra():
    gam = oracle.gamma_matrices()
    for mu in range(4):
        for nu in range(4):
            ac = gam[mu] @ gam[nu] + gam[nu] @ gam[mu]
            assert np.allclose(ac, 2 * G[mu, nu] * np.eye(4), atol=1e-15)
    g5 = 1j * gam[0] @ gam[1] @ gam[2] @ gam[3]
    # chiral representation: gamma^5 = diag(-1, -1, 1, 1)
    assert np.allclose(g5, np.diag([-1, -1, 1, 1]), atol=1e-15)


def slash(p):
    gam = oracle.gamma_matrices()
    return gam[0] * p[0] - gam[1] * p[1] - gam[2] * p[2] - gam[3] * p[3]


MOMENTA = [
    (173.0, np.array([0.0, 120.0, -80.0, 310.0])),
    (173.0, np.array([0.0, 0.0, 0.0, -400.0])),       # along -z: branch of chi
    (173.0, np.array([0.0, 1e-3, 2e-3, -400.0])),     # nearly along -z
    (0.0, np.array([0.0, -33.0, 47.0, 12.0])),
    (0.0, np.array([0.0, 0.0, 0.0, -250.0])),
    (0.0, np.array([0.0, 0.0, 0.0, 250.0])),
]


@pytest.mark.parametrize("m,p3", MOMENTA)
@pytest.mark.parametrize("basis", [0, 1])
def test_spin_sums(m, p3, basis):
    """sum u ubar = pslash + m, sum v vbar = pslash - m, and for the gluon
    sum eps^i eps^j* = delta^ij - k^i k^j / |k|^2 (eps^0 = 0)."""
    E = math.sqrt(m * m + p3[1:] @ p3[1:])
    p = p3.copy()
    p[0] = E
    uu, vv, ee = oracle.spin_sums(p, m, basis)
    scale = max(E, 1.0)
    assert np.allclose(uu, slash(p) + m * np.eye(4), atol=1e-13 * scale)
    assert np.allclose(vv, slash(p) - m * np.eye(4), atol=1e-13 * scale)
    k = p[1:] / np.linalg.norm(p[1:])
    expect = np.zeros((4, 4))
    expect[1:, 1:] = np.eye(3) - np.outer(k, k)
    assert np.allclose(ee, expect, atol=1e-14)


def test_structure_constants():
    f = oracle.fabc()
    # total antisymmetry and the standard non-zero values (1-based labels)
    for a, b, c in itertools.product(range(8), repeat=3):
        assert abs(f[a, b, c] + f[b, a, c]) < 1e-15 and abs(f[a, b, c] + f[a, c, b]) < 1e-15
    vals = {(1, 2, 3): 1.0, (1, 4, 7): 0.5, (1, 5, 6): -0.5, (2, 4, 6): 0.5, (2, 5, 7): 0.5,
            (3, 4, 5): 0.5, (3, 6, 7): -0.5, (4, 5, 8): math.sqrt(3) / 2, (6, 7, 8): math.sqrt(3) / 2}
    for (a, b, c), v in vals.items():
        assert abs(f[a - 1, b - 1, c - 1] - v) < 1e-15
    # Casimir: f^{acd} f^{bcd} = N delta^{ab}
    assert np.allclose(np.einsum("acd,bcd->ab", f, f), 3 * np.eye(8), atol=1e-14)


@pytest.mark.parametrize("proc,n", [("gg_tt", 2), ("gg_ttg", 3), ("gg_ttgg", 4), ("gg_ttggg", 5)])
def test_quark_line_colour_matrix(proc, n):
    C = oracle.colour_matrix(proc)
    assert C.shape == (math.factorial(n),) * 2
    assert np.allclose(C, C.T, atol=1e-13)
    assert np.min(np.linalg.eigvalsh(C)) > -1e-12
    # diagonal N C_F^n: sum over colours of |(T^s)_ij|^2 = Tr(T^s T^s dagger) = N C_F^n
    assert np.allclose(np.diag(C), 3 * (4.0 / 3.0) ** n, rtol=1e-13)
    # every entry is a rational whose denominator divides 2^max(0,n-3) 3^(n-1): each
    # Fierz step contributes a factor 1/2 or 1/(2N)
    x = C * 3 ** (n - 1) * 2 ** max(0, n - 3)
    assert np.allclose(x, np.round(x), atol=1e-9)


def test_colour_matrix_two_gluons_exact():
    C = oracle.colour_matrix("gg_tt")
    assert np.allclose(C, [[16 / 3, -2 / 3], [-2 / 3, 16 / 3]], atol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_colour_matrix_relabelling(n):
    a, b = oracle.colour_matrix_methods(n)
    assert np.allclose(a, b, atol=1e-13)


def test_single_trace_colour_matrix():
    """Four gluons, single traces Tr(t^a4 t^s1 t^s2 t^s3): symmetric, positive, and the
    colour-summed |M|^2 of a constant amplitude vector equals the sum over explicit
    colours of |sum_s Tr(..)|^2, which for all-equal amplitudes is the total
    sum_{all} |Tr(t^{a4} (sum over orderings))|^2 -- checked directly here."""
    C = oracle.colour_matrix("gg_gg")
    assert C.shape == (6, 6)
    assert np.allclose(C, C.T, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(C)) > -1e-12
    # diagonal: sum_a |Tr(t^a t^b t^c t^d)|^2 = (N^2-1)(N^4-3N^2+3)/(16 N^2) * ... is not
    # used; instead: with f^{abc} written as traces the (1 2 3)-(3 2 1) combination
    # is the colour factor of a three-gluon vertex, whose square is N (N^2-1) f f / 4.
    v = np.zeros(6)
    orders = oracle.orderings("gg_gg")
    # Tr(t^4 [t^1,[t^2,t^3]]) = Tr(t^4 (t1 t2 t3 - t1 t3 t2 - t2 t3 t1 + t3 t2 t1))
    for s, sign in [((0, 1, 2), 1), ((0, 2, 1), -1), ((1, 2, 0), -1), ((2, 1, 0), 1)]:
        v[orders.index(s)] = sign
    # [t^2,t^3] = i f^{23e} t^e, [t^1, i f^{23e} t^e] = - f^{23e} f^{1eg} t^g,
    # Tr(t^4 ..) = - f^{23e} f^{1e4} / 2; sum over colours of its square = N^2 (N^2-1)/4 = 18
    assert abs(v @ C @ v - 18.0) < 1e-12

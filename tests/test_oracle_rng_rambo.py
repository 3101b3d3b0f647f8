"""Pins of the oracle's random numbers and RAMBO phase space (CPU only).

Philox4x64-10 is pinned to numpy's independent implementation of the same published
generator (Salmon et al., SC'11); numpy's bit generator increments its 256-bit counter
before each block, so its state counter c-1 yields our block c.  RAMBO (Kleiss, Stirling,
Ellis 1986) is pinned by what the algorithm guarantees: momentum conservation, mass
shells, and the isotropy of two-body decays.
"""
import math

import numpy as np
import pytest

import oracle
from tests import workloads as W


def numpy_block(counter, key):
    c = int(counter[0]) | int(counter[1]) << 64 | int(counter[2]) << 128 | int(counter[3]) << 192
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=words, key=np.array(key, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (5, 0)),
    ((123456789, 0, 0, 0), (0x5EED, 0)),
    ((2**64 - 1, 7, 0, 0), (2**64 - 1, 2**63)),
    ((3, 2**64 - 1, 2**64 - 1, 9), (0xDEADBEEF, 0x12345678)),
])
def test_philox_matches_numpy(counter, key):
    assert oracle.philox(counter, key) == numpy_block(counter, key)


def test_uniform_mapping_open_interval():
    assert oracle.lib().or_u01 is not None
    f = oracle.lib().or_u01
    f.restype = __import__("ctypes").c_double
    f.argtypes = [__import__("ctypes").c_uint64]
    assert f(0) == 0.5 * 2.0 ** -53
    assert f(2**64 - 1) == 1.0 - 0.5 * 2.0 ** -53
    assert f(1 << 63) == 0.5 + 0.5 * 2.0 ** -53


def test_uniforms_use_event_particle_counter():
    seed, evt, nf = 7, 11, 3
    for i in range(nf):
        raw = oracle.philox((evt * nf + i, 0, 0, 0), (seed, 0))
        r = oracle.uniforms(seed, evt, nf, i)
        assert np.array_equal(r, [((u >> 11) + 0.5) * 2.0 ** -53 for u in raw])


def minkowski_sq(p):
    return p[..., 0] ** 2 - p[..., 1] ** 2 - p[..., 2] ** 2 - p[..., 3] ** 2


@pytest.mark.parametrize("name", W.ALL)
def test_rambo_conservation_and_shells(name):
    m = W.final_masses(name)
    rs = W.sqrt_s(name)
    p = oracle.rambo(W.SEED, rs, m, 2000)
    tot_in = p[:, 0] + p[:, 1]
    tot_out = p[:, 2:].sum(axis=1)
    assert np.allclose(tot_in, [rs, 0, 0, 0], atol=0, rtol=0)
    assert np.max(np.abs(tot_out - tot_in)) <= 1e-12 * rs
    for i, mi in enumerate(m):
        assert np.max(np.abs(minkowski_sq(p[:, 2 + i]) - mi * mi)) <= 1e-12 * rs * rs
        assert np.all(p[:, 2 + i, 0] > 0)
    assert np.all(np.abs(minkowski_sq(p[:, 0])) == 0) and np.all(np.abs(minkowski_sq(p[:, 1])) == 0)


def test_rambo_two_body_isotropic():
    """For 2 -> 2 massless, RAMBO is uniform in cos(theta) and phi: Kolmogorov-Smirnov
    test of cos(theta) on 8192 events, and of phi/(2 pi)."""
    from scipy import stats
    p = oracle.rambo(0, 500.0, (0.0, 0.0), 8192)
    c = p[:, 2, 3] / np.linalg.norm(p[:, 2, 1:], axis=1)
    assert stats.kstest(c, stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    phi = (np.arctan2(p[:, 2, 2], p[:, 2, 1]) / (2 * math.pi)) % 1.0
    assert stats.kstest(phi, stats.uniform().cdf).pvalue > 1e-3
    # back to back with |p| = sqrt(s)/2
    assert np.allclose(np.linalg.norm(p[:, 2, 1:], axis=1), 250.0, rtol=1e-13)


def test_rambo_massive_two_body_momentum():
    rs, m = 1500.0, 173.0
    p = oracle.rambo(1, rs, (m, m), 512)
    pabs = math.sqrt(rs * rs / 4 - m * m)
    assert np.allclose(np.linalg.norm(p[:, 2, 1:], axis=1), pabs, rtol=1e-12)
    assert np.allclose(p[:, 2, 0], rs / 2, rtol=1e-13)


def test_rambo_deterministic_and_offset():
    a = oracle.rambo(3, 1500.0, W.final_masses("gg_ttg"), 40)
    b = oracle.rambo(3, 1500.0, W.final_masses("gg_ttg"), 10, evt0=30)
    assert np.array_equal(a[30:], b)
    c = oracle.rambo(4, 1500.0, W.final_masses("gg_ttg"), 40)
    assert not np.allclose(a[:, 2:], c[:, 2:])


def test_rambo_rejects_below_threshold():
    with pytest.raises(ValueError):
        oracle.rambo(0, 300.0, (173.0, 173.0), 4)


@pytest.mark.parametrize("n_final", [3, 4, 5])
def test_rambo_massless_n_body_energy_density(n_final):
    """Flat massless n-body phase space fixes each particle's energy spectrum.  With
    x = 2E/sqrt(s), the measure d^3p/E = 4 pi E dE of one particle times the volume of the
    other n-1 massless particles at invariant mass^2 s(1 - x), which grows as (s(1 - x))^(n-3),
    gives a density proportional to x (1 - x)^(n-3): Beta(2, n-2).  Kolmogorov-Smirnov test of
    every final particle on 6000 events.  This pins RAMBO's step 1 (energy density
    q0 exp(-q0), i.e. q0 = -ln(r3 r4)) and its conformal boost; the conservation, mass-shell and
    two-body tests above hold for wrong energy densities too."""
    from scipy import stats
    rs = 1000.0
    p = oracle.rambo(21, rs, (0.0,) * n_final, 6000)
    ref = stats.beta(2, n_final - 2).cdf
    for i in range(n_final):
        x = 2.0 * p[:, 2 + i, 0] / rs
        assert stats.kstest(x, ref).pvalue > 1e-3, (n_final, i)


def test_rambo_massless_three_body_dalitz_plane_uniform():
    """Massless three-body phase space is uniform on the Dalitz triangle x1 + x2 >= 1,
    x1, x2 <= 1 (x_i = 2 E_i / sqrt(s)): x1 has density 2 x1, and at fixed x1 the variable
    u = (x2 - 1 + x1) / x1 is uniform on [0, 1], independently of x1 (tested in both halves of
    the x1 range)."""
    from scipy import stats
    rs = 1000.0
    p = oracle.rambo(22, rs, (0.0, 0.0, 0.0), 8000)
    x1 = 2.0 * p[:, 2, 0] / rs
    x2 = 2.0 * p[:, 3, 0] / rs
    assert np.all(x1 + x2 >= 1.0 - 1e-12) and np.all(x1 <= 1.0 + 1e-12) and np.all(x2 <= 1.0 + 1e-12)
    assert stats.kstest(x1, lambda t: np.clip(t, 0, 1) ** 2).pvalue > 1e-3
    u = (x2 - 1.0 + x1) / x1
    for sel in (x1 < np.median(x1), x1 >= np.median(x1)):
        assert stats.kstest(u[sel], stats.uniform().cdf).pvalue > 1e-3

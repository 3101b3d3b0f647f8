"""CPU oracle for the leading-order matrix elements -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The product library never loads it; it shares no code with the
HIP path.  See ``me.c`` and ``rambo.c`` for what is computed and which published
definitions each step follows.

Process ids and particle orders:
  ee_mumu  (e+, e-, mu+, mu-)                 one photon diagram
  gg_tt    (g, g, t, t~)                      QCD
  gg_ttg   (g, g, t, t~, g)
  gg_ttgg  (g, g, t, t~, g, g)
  gg_ttggg (g, g, t, t~, g, g, g)
  gg_gg    (g, g, g, g)                       test process (pure gluon vertices)
  ee_mumu_z (e+, e-, mu+, mu-)                photon and Z exchange
Parameters: params = (m_t, alpha_em, alpha_s).

Pins (checks against what the physics fixes, never against this code's own formulas):
  test_oracle_me.py         textbook |M|^2 of ee_mumu (photon, and photon + Z), gg_gg and gg_tt
                            (Combridge) at several angles, the gg_tt threshold value and massless
                            limit, brute-force explicit-colour sums,
                            gauge, Lorentz and Bose invariance, basis independence;
  test_oracle_parke_taylor.py  m_t = 0: vanishing helicities, Parke-Taylor moduli of every MHV
                            amplitude of gg_tt .. gg_ttggg, the helicity-filter count;
  test_oracle_soft_limit.py m_t = 173: eikonal factorisation gg_tt -> gg_ttg -> gg_ttgg -> gg_ttggg;
  test_oracle_dirac_colour.py, test_oracle_rng_rambo.py, test_oracle_diagrams.py,
  test_oracle_select.py     spinors, colour algebra, Philox and RAMBO, the diagram-by-diagram
                            second algorithm, the selection draws.
No function here is left "parity unpinned".
"""
import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PROCESSES = {"ee_mumu": 0, "gg_tt": 1, "gg_ttg": 2, "gg_ttgg": 3, "gg_ttggg": 4, "gg_gg": 5, "ee_mumu_z": 6}
DEFAULT_PARAMS = (173.0, 1.0 / 132.507, 0.118)

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _ptr(a, t=_D):
    return a.ctypes.data_as(t)


def _load(name):
    path = os.path.join(HERE, name)
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(path)
    lib.or_me.restype = ctypes.c_double
    lib.or_me.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, _D]
    lib.or_me_batch.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int64, ctypes.c_int, _D]
    lib.or_partials.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
    lib.or_orderings.argtypes = [ctypes.c_int, _I]
    lib.or_colour_matrix.argtypes = [ctypes.c_int, _D]
    lib.or_colour_matrix_methods.argtypes = [ctypes.c_int, _D, _D]
    lib.or_amp_explicit_colour.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, _I, _D, _D]
    lib.or_tree_amp.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, _I, ctypes.c_int, _D]
    lib.or_ee_z_amp.argtypes = [_D, _D, ctypes.c_int, ctypes.c_int, _D]
    lib.or_me_brute_colour.restype = ctypes.c_double
    lib.or_me_brute_colour.argtypes = [ctypes.c_int, _D, _D]
    lib.or_spin_sums.argtypes = [_D, ctypes.c_double, ctypes.c_int, _D, _D, _D]
    lib.or_gamma.argtypes = [_D]
    lib.or_fabc.argtypes = [_D]
    if hasattr(lib, "or_rambo"):
        lib.or_rambo.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_int, _D,
                                 ctypes.c_int64, ctypes.c_int64, _D]
        lib.or_philox4x64_10.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 3
        lib.or_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _D]
    return lib


_LIBS = {}


def lib(precision="double"):
    name = {"double": "liboracle.so", "long double": "liboracle_ld.so"}[precision]
    if name not in _LIBS:
        _LIBS[name] = _load(name)
    return _LIBS[name]


def n_par(process):
    return lib().or_n_par(PROCESSES[process])


def _params(params):
    return np.ascontiguousarray(params if params is not None else DEFAULT_PARAMS, dtype=np.float64)


def me(process, p, params=None, basis=0, precision="double", per_helicity=False):
    """Averaged |M|^2 of one event p[n_par][4]; with per_helicity also the colour-summed
    |M_h|^2 of every helicity (index h: particle i's helicity bit at 2^(n_par-1-i))."""
    L = lib(precision)
    p = np.ascontiguousarray(p, dtype=np.float64)
    prm = _params(params)
    nh = 1 << n_par(process)
    hel = np.zeros(nh)
    v = L.or_me(PROCESSES[process], _ptr(prm), _ptr(p), basis, _ptr(hel))
    return (v, hel) if per_helicity else v


def me_batch(process, p, params=None, basis=0, precision="double", threads=None):
    """Averaged |M|^2 for p[n_evt][n_par][4], split over host threads (ctypes releases
    the GIL, so the C loops run in parallel)."""
    L = lib(precision)
    p = np.ascontiguousarray(p, dtype=np.float64)
    n = p.shape[0]
    out = np.zeros(n)
    prm = _params(params)
    pid = PROCESSES[process]
    threads = threads or os.cpu_count() or 1
    chunks = [(i, min(n, i + max(1, -(-n // (4 * threads))))) for i in range(0, n, max(1, -(-n // (4 * threads))))]

    def run(c):
        a, b = c
        sub_p = p[a:b]
        sub_o = np.zeros(b - a)
        L.or_me_batch(pid, _ptr(prm), _ptr(sub_p), b - a, basis, _ptr(sub_o))
        out[a:b] = sub_o

    if threads == 1 or n <= 1:
        run((0, n))
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, chunks))
    return out


def partials(process, p, helicity, params=None, basis=0, gauge_gluon=-1):
    """Colour-ordered amplitudes A(sigma) of one helicity, in the lexicographic order of
    ``orderings(process)``; gauge_gluon >= 0 replaces that gluon's polarisation by its
    momentum."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(2 * 120)
    k = lib().or_partials(PROCESSES[process], _ptr(_params(params)), _ptr(p), helicity, basis,
                          gauge_gluon, _ptr(out))
    return out[:2 * k:2] + 1j * out[1:2 * k:2]


def orderings(process):
    pid = PROCESSES[process]
    out = np.zeros(120 * 5, dtype=np.int32)
    k = lib().or_orderings(pid, _ptr(out, _I))
    n = 3 if process == "gg_gg" else n_par(process) - 2
    return [tuple(out[s * n:(s + 1) * n]) for s in range(k)]


def colour_matrix(process):
    out = np.zeros(120 * 120)
    k = lib().or_colour_matrix(PROCESSES[process], _ptr(out))
    return out[:k * k].reshape(k, k)


def colour_matrix_methods(n):
    """(by definition, by relabelling) for the quark line with n <= 4 gluons."""
    a = np.zeros(24 * 24)
    b = np.zeros(24 * 24)
    k = lib().or_colour_matrix_methods(n, _ptr(a), _ptr(b))
    return a[:k * k].reshape(k, k), b[:k * k].reshape(k, k)


def amp_explicit_colour(process, p, helicity, colours, params=None):
    """(colour-dressed amplitude, colour-decomposed amplitude) for explicit colours."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    c = np.ascontiguousarray(colours, dtype=np.int32)
    d = np.zeros(2)
    e = np.zeros(2)
    lib().or_amp_explicit_colour(PROCESSES[process], _ptr(_params(params)), _ptr(p), helicity,
                                 _ptr(c, _I), _ptr(d), _ptr(e))
    return complex(d[0], d[1]), complex(e[0], e[1])


def me_brute_colour(process, p, params=None):
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().or_me_brute_colour(PROCESSES[process], _ptr(_params(params)), _ptr(p))


def spin_sums(p, m, basis=0):
    p = np.ascontiguousarray(p, dtype=np.float64)
    uu = np.zeros(32)
    vv = np.zeros(32)
    ee = np.zeros(32)
    lib().or_spin_sums(_ptr(p), m, basis, _ptr(uu), _ptr(vv), _ptr(ee))
    f = lambda a: (a[0::2] + 1j * a[1::2]).reshape(4, 4)
    return f(uu), f(vv), f(ee)


def gamma_matrices():
    out = np.zeros(2 * 64)
    lib().or_gamma(_ptr(out))
    return (out[0::2] + 1j * out[1::2]).reshape(4, 4, 4)


def fabc():
    out = np.zeros(512)
    lib().or_fabc(_ptr(out))
    return out.reshape(8, 8, 8)


def philox(counter, key):
    c = (ctypes.c_uint64 * 4)(*counter)
    k = (ctypes.c_uint64 * 2)(*key)
    o = (ctypes.c_uint64 * 4)()
    lib().or_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def uniforms(seed, evt, n_final, i):
    r = np.zeros(4)
    lib().or_uniforms(seed, evt, n_final, i, _ptr(r))
    return r


def rambo(seed, sqrt_s, final_masses, n_evt, evt0=0):
    """Events evt0.. of the RAMBO stream `seed`: array [n_evt][2+n_final][4]."""
    m = np.ascontiguousarray(final_masses, dtype=np.float64)
    nf = len(m)
    out = np.zeros((n_evt, nf + 2, 4))
    rc = lib().or_rambo(seed, sqrt_s, nf, _ptr(m), evt0, n_evt, _ptr(out))
    if rc != 0:
        raise ValueError("bad RAMBO arguments")
    return out


# ----------------------------------------------------------------------------------------
# Per-event helicity and colour-flow choice (the two per-event records of an unweighted
# event that the paper, Sec. 4, lists as still missing): plain definitions.

def helicity_weights(process, p, params=None):
    """colour-summed |M_h|^2 of every helicity combination h (numbering as in ``me``)"""
    return me(process, p, params=params, per_helicity=True)[1]


def colour_weights(process, p, params=None):
    """leading-colour weight of every colour flow sigma (order of ``orderings``):
    w_sigma = sum over all helicities of |A_sigma|^2, the diagonal terms of the colour sum"""
    nh = 1 << n_par(process)
    w = None
    for h in range(nh):
        a = partials(process, p, h, params=params)
        w = np.abs(a) ** 2 if w is None else w + np.abs(a) ** 2
    return w


def draw(weights, r):
    """index j drawn from the weights with the uniform r in [0, 1): the smallest j with
    r * W < w_0 + ... + w_j (W the total, all sums left to right in FP64); if rounding
    leaves no such j, the last j of positive weight"""
    total = 0.0
    for x in weights:
        total += float(x)
    target = r * total
    cum, last = 0.0, 0
    for j, x in enumerate(weights):
        cum += float(x)
        if x > 0.0:
            last = j
        if target < cum:
            return j
    return last


def ee_z_amplitude(p, h, diagrams=3, params=None):
    """ee -> mumu with Z: amplitude of helicity h from the photon (1), the Z (2) or both (3)"""
    out = np.zeros(2)
    lib().or_ee_z_amp(_ptr(_params(params)), _ptr(np.ascontiguousarray(p, dtype=np.float64)), h, diagrams,
                      _ptr(out))
    return out[0] + 1j * out[1]


_GOOD = {}


def good_helicities(process, sqrt_s, final_masses, params=None, n_events=1024, seed=0x5EED, threshold=1e-20):
    """helicity combinations kept by the helicity filter, computed by the oracle itself: h is
    kept iff max over n_events RAMBO events (stream `seed`) of |M_h|^2 / sum_h |M_h|^2 exceeds
    the threshold"""
    key = (process, sqrt_s, tuple(final_masses), None if params is None else tuple(params), n_events, seed,
           threshold)
    if key not in _GOOD:
        p = rambo(seed, sqrt_s, final_masses, n_events)
        r = np.zeros(1 << n_par(process))
        for ev in p:
            _, hel = me(process, ev, params=params, per_helicity=True)
            tot = hel.sum()
            if tot > 0:
                r = np.maximum(r, hel / tot)
        _GOOD[key] = [h for h in range(len(r)) if r[h] > threshold]
    return _GOOD[key]

"""Feynman diagrams one at a time, for the single-diagram channel weights -- TEST
INFRASTRUCTURE ONLY (part of the CPU oracle; shares nothing with the HIP path).

The paper (Sec. 2) names MadEvent's single-diagram-enhancement (multichannel) algorithm among
the features of its ME engine: the integrand of channel c is |M|^2 times the channel weight
W_c / sum_d W_d, with W_d a single diagram's squared amplitude.  This module computes W_d
for the quark-line processes gg -> t t~ + gluons from the definition:

  W_d = sum over the helicities the filter keeps (see ``good_helicities``), over the
        diagram's four-gluon colour structures s (taken
        incoherently), of sum over explicit colours |CF_ds(colours) L_ds(helicity)|^2
      = sum_h sum_s |L_ds(h)|^2 K_ds,  K_ds = sum_colours |CF_ds|^2,

with L_ds the colour-stripped Lorentz amplitude (C oracle, ``or_tree_amp``: the Peskin &
Schroeder rules of ``me.c``) and CF_ds the product of t^a (quark line), f^{abc} and f f
(four-gluon structures) with every internal colour index summed, evaluated numerically
from the Gell-Mann matrices.

Diagrams are enumerated here by their own construction: an ordered sequence of gluon trees
attached along the quark line (from the antiquark end), the trees' leaf sets partitioning
the gluons, each tree built from unordered splits of its leaf set into two (three-gluon
vertex) or three (four-gluon vertex) parts.  A diagram is identified across programs by
its internal lines: the set of external particles on one side of each propagator
(bit i = particle i; the side without particle 0).
"""
import itertools

import numpy as np

from . import PROCESSES, _I, _params, _ptr, lib, n_par

# ----------------------------------------------------------------------------------------
# enumeration


def _splits(S, parts):
    """unordered partitions of the sorted tuple S into `parts` non-empty blocks, each block
    sorted, blocks ordered by their smallest element"""
    S = tuple(S)
    if parts == 1:
        yield (S,)
        return
    first, rest = S[0], S[1:]
    # the block holding the smallest element, then the rest split into parts - 1 blocks
    for r in range(0, len(rest) + 1):
        for comb in itertools.combinations(rest, r):
            block = (first,) + comb
            remaining = tuple(x for x in rest if x not in comb)
            if len(remaining) < parts - 1:
                continue
            for tail in _splits(remaining, parts - 1):
                yield (block,) + tail


def gluon_trees(S):
    """all gluon trees with leaf set S (sorted tuple): ('g', i), ('V3', A, B), ('V4', A, B, C)"""
    S = tuple(sorted(S))
    if len(S) == 1:
        return [("g", S[0])]
    out = []
    for A, B in _splits(S, 2):
        for ta in gluon_trees(A):
            for tb in gluon_trees(B):
                out.append(("V3", ta, tb))
    if len(S) >= 3:
        for A, B, C in _splits(S, 3):
            for ta in gluon_trees(A):
                for tb in gluon_trees(B):
                    for tc in gluon_trees(C):
                        out.append(("V4", ta, tb, tc))
    return out


def _ordered_partitions(S):
    """ordered sequences of non-empty blocks partitioning S"""
    S = tuple(S)
    if not S:
        yield ()
        return
    for r in range(1, len(S) + 1):
        for block in itertools.combinations(S, r):
            rest = tuple(x for x in S if x not in block)
            for tail in _ordered_partitions(rest):
                yield (block,) + tail


def diagrams(ng):
    """every tree diagram of g g -> t t~ + (ng - 2) g: tuples (G_1, .., G_k) of gluon trees
    along the quark line, G_1 next to the antiquark"""
    out = []
    for blocks in _ordered_partitions(range(ng)):
        for trees in itertools.product(*[gluon_trees(b) for b in blocks]):
            out.append(tuple(trees))
    return out


def leaves(t):
    return (t[1],) if t[0] == "g" else tuple(sorted(x for c in t[1:] for x in leaves(c)))


def n_four_vertices(t):
    return 0 if t[0] == "g" else (t[0] == "V4") + sum(n_four_vertices(c) for c in t[1:])


def structures(diagram):
    """assignments of a colour structure (0, 1, 2) to every four-gluon vertex"""
    n4 = sum(n_four_vertices(t) for t in diagram)
    return list(itertools.product(range(3), repeat=n4))


# ----------------------------------------------------------------------------------------
# identification by internal lines


def gluon_particle(process):
    """particle index of each gluon (gluons in particle order)"""
    return [0, 1] + list(range(4, n_par(process)))


def descriptor(process, diagram):
    """sorted masks of the internal lines (bit i = particle i, side without particle 0)"""
    gp = gluon_particle(process)
    full = (1 << n_par(process)) - 1

    def canon(m):
        return m if not (m & 1) else full ^ m

    def mask(ls):
        return sum(1 << gp[i] for i in ls)

    lines = []

    def walk(t):
        if t[0] == "g":
            return
        lines.append(canon(mask(leaves(t))))
        for c in t[1:]:
            walk(c)

    for t in diagram:
        walk(t)
    # quark propagators: the antiquark (particle 3) plus the gluons of G_1..G_j, j < k
    acc = 1 << 3
    for t in diagram[:-1]:
        acc |= mask(leaves(t))
        lines.append(canon(acc))
    return tuple(sorted(lines))


# ----------------------------------------------------------------------------------------
# Lorentz part (C oracle) and colour part (numeric)


def program(diagram, assign):
    """postfix program of ``or_tree_amp`` for the structure assignment `assign`"""
    prog = []
    it = iter(assign)

    def emit(t):
        if t[0] == "g":
            prog.append(t[1])
            return
        for c in t[1:]:
            emit(c)
        prog.append(-1 if t[0] == "V3" else -2 - next(it))

    for t in diagram:
        emit(t)
    prog.append(-10 - len(diagram))
    return prog


def lorentz(process, p, h, diagram, assign, params=None, precision="double"):
    prog = np.ascontiguousarray(program(diagram, assign), dtype=np.int32)
    out = np.zeros(2)
    rc = lib(precision).or_tree_amp(PROCESSES[process], _ptr(_params(params)), _ptr(np.ascontiguousarray(p, dtype=np.float64)),
                           h, _ptr(prog, _I), len(prog), _ptr(out))
    if rc != 0:
        raise ValueError("malformed diagram program")
    return out[0] + 1j * out[1]


_COLOUR = {}


def _colour_tables():
    if not _COLOUR:
        lam = np.zeros((8, 3, 3), dtype=complex)
        lam[0][0, 1] = lam[0][1, 0] = 1
        lam[1][0, 1], lam[1][1, 0] = -1j, 1j
        lam[2][0, 0], lam[2][1, 1] = 1, -1
        lam[3][0, 2] = lam[3][2, 0] = 1
        lam[4][0, 2], lam[4][2, 0] = -1j, 1j
        lam[5][1, 2] = lam[5][2, 1] = 1
        lam[6][1, 2], lam[6][2, 1] = -1j, 1j
        lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
        t = lam / 2
        comm = np.einsum("aij,bjk->abik", t, t) - np.einsum("bij,ajk->abik", t, t)
        f = np.real(-2j * np.einsum("abij,cji->abc", comm, t))
        ff = [np.einsum("abe,cde->abcd", f, f), np.einsum("ace,bde->abcd", f, f),
              np.einsum("ade,bce->abcd", f, f)]
        _COLOUR.update(t=t, f=f, ff=ff)
    return _COLOUR


def colour_tensor(diagram, assign, ng):
    """CF[i, j, a_0, .., a_{ng-1}] with every internal colour summed (leaf axes in gluon order)"""
    tab = _colour_tables()
    it = iter(assign)

    def node(t):
        # returns (tensor [root, leaf colours...], leaf order)
        if t[0] == "g":
            return np.eye(8), (t[1],)
        kids = [node(c) for c in t[1:]]
        order = tuple(x for _, o in kids for x in o)
        if t[0] == "V3":
            T = np.tensordot(tab["f"], kids[0][0], axes=([1], [0]))          # [a, c, A...]
            T = np.moveaxis(np.tensordot(T, kids[1][0], axes=([1], [0])), 0, 0)  # [a, A..., B...]
        else:
            T = np.tensordot(tab["ff"][next(it)], kids[0][0], axes=([1], [0]))   # [a, c, d, A...]
            T = np.tensordot(T, kids[1][0], axes=([1], [0]))                    # [a, d, A..., B...]
            T = np.tensordot(T, kids[2][0], axes=([1], [0]))                    # [a, A..., B..., C...]
        return T, order

    # quark line: (t^{a_k} .. t^{a_1})_{ij}, contracted with each attachment's tensor
    M = None
    order = ()
    for t in diagram:                       # G_1 first: M <- t^{a} M
        T, o = node(t)
        step = np.tensordot(tab["t"], T, axes=([0], [0]))                    # [i, l, leaves of t]
        if M is None:
            M = step                                                         # [i, j, leaves]
        else:
            M = np.tensordot(step, M, axes=([1], [0]))                       # [i, leaves t, j, leaves M]
            nt = len(o)
            M = np.moveaxis(M, 1 + nt, 1)                                    # [i, j, leaves t, leaves M]
        order = o + order
    perm = [2 + order.index(k) for k in range(ng)]
    return np.transpose(M, [0, 1] + perm)


# ----------------------------------------------------------------------------------------
# channel weights


def entries(process):
    """(diagram, structure assignment) of every amplitude entry"""
    ng = n_par(process) - 2
    return [(d, s) for d in diagrams(ng) for s in structures(d)]


def colour_weights_K(process):
    """K_ds = sum over colours |CF_ds|^2 of every entry"""
    ng = n_par(process) - 2
    return np.array([np.sum(np.abs(colour_tensor(d, s, ng)) ** 2) for d, s in entries(process)])


def diagram_weights(process, p, params=None, K=None, helicities=None):
    """{descriptor: W_d} for one event, summed over `helicities` (default: all).  A
    helicity whose full amplitude vanishes can still have non-zero single diagrams, so the
    set matters: MadEvent sums over the helicities its filter keeps."""
    ents = entries(process)
    K = colour_weights_K(process) if K is None else K
    hs = range(1 << n_par(process)) if helicities is None else helicities
    W = {}
    for (d, s), k in zip(ents, K):
        w = 0.0
        for h in hs:
            w += abs(lorentz(process, p, h, d, s, params)) ** 2
        key = descriptor(process, d)
        W[key] = W.get(key, 0.0) + w * k
    return W


def channel_factor(process, p, channel_descriptor, params=None, K=None, helicities=None):
    """W_c / sum_d W_d for the diagram with the given internal lines"""
    W = diagram_weights(process, p, params, K, helicities)
    return W[channel_descriptor] / sum(W.values())


# ----------------------------------------------------------------------------------------
# the matrix element as a sum of Feynman diagrams (the GPU's algorithm, evaluated by the
# oracle's own machinery): conditioning of that algorithm in FP64

_FLOWS = {}


def flow_coefficients(process):
    """c[e, sigma] with CF_e = sum_sigma c[e, sigma] (t^{a_sigma1} .. t^{a_sigman})_{ij}: each
    entry's colour tensor projected on the colour strings of ``orderings`` (least squares,
    exact for tree diagrams)"""
    if process not in _FLOWS:
        from . import orderings
        ng = n_par(process) - 2
        t = _colour_tables()["t"]
        strings = []
        for sigma in orderings(process):
            # T[i, j, a_0 .. a_{ng-1}] = (t^{a_sigma1} .. t^{a_sigman})_{ij}
            T = None
            for k in sigma:
                k = int(k)
                # factor t^{a_k}[x, y] with its own colour axis, placed at gluon k's position
                if T is None:
                    T = np.moveaxis(t, 0, 2)                                # [i, y, a_k]
                    axes = [k]
                else:
                    T = np.tensordot(T, t, axes=([1], [1]))                 # [i, a..., b, y]
                    T = np.moveaxis(T, -1, 1)                               # [i, y, a..., b]
                    axes.append(k)
            perm = [0, 1] + [2 + axes.index(g) for g in range(ng)]
            strings.append(np.transpose(T, perm).ravel())
        S = np.array(strings).T                                             # [colours, flows]
        CF = np.array([colour_tensor(d, s, ng).ravel() for d, s in entries(process)]).T
        c, *_ = np.linalg.lstsq(S, CF, rcond=None)
        assert np.allclose(S @ c, CF, atol=1e-12)
        _FLOWS[process] = c.T                                               # [entries, flows]
    return _FLOWS[process]


def diagram_me(process, p, params=None, precision="double"):
    """averaged |M|^2 from the Feynman diagrams: jamps J_sigma = sum_e c[e, sigma] L_e (all
    helicities), colour sum with the oracle's numeric colour matrix; the Lorentz parts in the
    given precision of the C oracle, the jamp and colour sums in FP64"""
    from . import colour_matrix
    c = flow_coefficients(process)
    C = colour_matrix(process)
    ents = entries(process)
    tot = 0.0
    for h in range(1 << n_par(process)):
        L = np.array([lorentz(process, p, h, d, s, params, precision) for d, s in ents])
        J = L @ c
        tot += float(np.real(np.conj(J) @ C @ J))
    return tot / 256

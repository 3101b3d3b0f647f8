"""Exact SU(3) colour algebra for the process generator.

Two jobs, both in exact arithmetic (no floating point):

1. Colour decomposition of a Feynman diagram.  For one quark line with gluons attached,
   every diagram's colour factor is a product of t^a along the line and f^{abc} at the
   gluon vertices.  Contracting each internal gluon with f^{xab} t^x = -i [t^a, t^b]
   turns it into a sum of ordered strings (t^{a_s1} ... t^{a_sn})_{ij} over
   permutations s of the gluons, with coefficients in {+-1, +-i}.  These strings are the
   colour flows; the diagram's amplitude is added to the flow amplitudes ("jamps") with
   those coefficients (the colour-flow decomposition of Mangano & Parke, Phys. Rep. 200
   (1991) 301).  For pure-gluon processes, the gluon on the root leg closes the string
   into 2 Tr(t^{a_root} ...).

2. The colour matrix C[s][t] = sum over colour indices of (T^s)_{ij} (T^t)^*_{ij}
   = Tr(t^{s1}..t^{sn} t^{tn}..t^{t1}), evaluated with the SU(N) Fierz identities
       t^a X t^a        = Tr(X)/2 - X/(2N)
       Tr(X t^a) Tr(Y t^a) = Tr(XY)/2 - Tr(X) Tr(Y)/(2N)
   with Tr(1) = N, as exact fractions.
"""
from fractions import Fraction
from functools import lru_cache
from itertools import permutations

NC = 3


class GaussInt:
    """a + b i with integer a, b (coefficients of the colour decomposition)."""
    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re, self.im = int(re), int(im)

    def __mul__(self, o):
        return GaussInt(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def __add__(self, o):
        return GaussInt(self.re + o.re, self.im + o.im)

    def __neg__(self):
        return GaussInt(-self.re, -self.im)

    def __eq__(self, o):
        return self.re == o.re and self.im == o.im

    def __hash__(self):
        return hash((self.re, self.im))

    def is_zero(self):
        return self.re == 0 and self.im == 0

    def __repr__(self):
        return f"({self.re}{self.im:+d}i)"


ONE = GaussInt(1, 0)
MINUS_I = GaussInt(0, -1)
MINUS_ONE = GaussInt(-1, 0)


def _lin(*terms):
    """sum of coefficient * expansion; expansions are dicts {sequence: GaussInt}"""
    out = {}
    for c, e in terms:
        for s, v in e.items():
            w = out.get(s, GaussInt()) + c * v
            if w.is_zero():
                out.pop(s, None)
            else:
                out[s] = w
    return out


def _concat(a, b):
    out = {}
    for s1, c1 in a.items():
        for s2, c2 in b.items():
            out[s1 + s2] = out.get(s1 + s2, GaussInt()) + c1 * c2
    return {s: c for s, c in out.items() if not c.is_zero()}


def commutator(a, b):
    return _lin((ONE, _concat(a, b)), (MINUS_ONE, _concat(b, a)))


def leaf(i):
    return {(i,): ONE}


def three_vertex(a, b):
    """colour of f^{x a b} t^x with the subtrees' colours a, b: -i [a, b]"""
    return _lin((MINUS_I, commutator(a, b)))


def four_vertex(k, a, b, c):
    """colour of one of the three f f structures of the four-gluon vertex with legs
    (x, a, b, c), x the leg towards the quark line, contracted into t^x:
      k = 0: f^{x a e} f^{b c e}  ->  -[a, [b, c]]
      k = 1: f^{x b e} f^{a c e}  ->  -[b, [a, c]]
      k = 2: f^{x c e} f^{a b e}  ->  -[c, [a, b]]"""
    if k == 0:
        e = commutator(a, commutator(b, c))
    elif k == 1:
        e = commutator(b, commutator(a, c))
    else:
        e = commutator(c, commutator(a, b))
    return _lin((MINUS_ONE, e))


def string_product(blocks):
    """colour of a quark line with blocks attached in order (quark side first)"""
    out = {(): ONE}
    for b in blocks:
        out = _concat(out, b)
    return out


# ---------------------------------------------------------------------------------------
# Fierz evaluation of fully contracted traces


def _canon(traces):
    """relabel adjoint indices by first appearance and rotate each trace to its smallest
    rotation; sort traces.  The value of a product of traces is invariant under both."""
    order = {}
    for t in traces:
        for a in t:
            if a not in order:
                order[a] = len(order)
    tt = []
    for t in traces:
        r = tuple(order[a] for a in t)
        if r:
            r = min(r[i:] + r[:i] for i in range(len(r)))
        tt.append(r)
    return tuple(sorted(tt))


@lru_cache(maxsize=None)
def _contract(traces):
    """value of prod_k Tr(t^{..}) with every adjoint label appearing exactly twice"""
    n_empty = sum(1 for t in traces if len(t) == 0)
    traces = tuple(t for t in traces if len(t) > 0)
    factor = Fraction(NC) ** n_empty
    if not traces:
        return factor
    # first label: find its two positions
    a = traces[0][0]
    pos = [(ti, pi) for ti, t in enumerate(traces) for pi, x in enumerate(t) if x == a]
    (t1, p1), (t2, p2) = pos
    half = Fraction(1, 2)
    inv2n = Fraction(1, 2 * NC)
    if t1 == t2:
        # Tr(A a B a C) = Tr(B) Tr(C A)/2 - Tr(B C A)/(2N)
        t = traces[t1]
        A, B, C = t[:p1], t[p1 + 1:p2], t[p2 + 1:]
        rest = traces[:t1] + traces[t1 + 1:]
        v = half * _contract(_canon(rest + (B, C + A))) - inv2n * _contract(_canon(rest + (B + C + A,)))
    else:
        # Tr(A a B) Tr(C a D) = Tr(B A D C)/2 - Tr(B A) Tr(D C)/(2N)
        x, y = traces[t1], traces[t2]
        A, B = x[:p1], x[p1 + 1:]
        C, D = y[:p2], y[p2 + 1:]
        rest = tuple(t for i, t in enumerate(traces) if i not in (t1, t2))
        v = half * _contract(_canon(rest + (B + A + D + C,))) - \
            inv2n * _contract(_canon(rest + (B + A, D + C)))
    return factor * v


def trace_value(traces):
    return _contract(_canon(tuple(tuple(t) for t in traces)))


def colour_matrix_quark_line(n):
    """C[s][t] = Tr(t^{s1}..t^{sn} t^{tn}..t^{t1}) over the permutations of n gluons,
    in lexicographic order; exact Fractions."""
    perms = list(permutations(range(n)))
    return perms, [[trace_value([list(s) + list(reversed(t))]) for t in perms] for s in perms]


def colour_matrix_single_trace(n):
    """C[s][t] = Tr(t^{r} T^s) Tr(T^t^dagger t^{r}) for n gluons, r = n-1 the root gluon,
    s, t orderings of the other n-1 (lexicographic)."""
    r = n - 1
    perms = list(permutations(range(n - 1)))
    return perms, [[trace_value([[r] + list(s), list(reversed(t)) + [r]]) for t in perms]
                   for s in perms]


def common_denominator(C):
    from math import lcm
    d = 1
    for row in C:
        for x in row:
            d = lcm(d, x.denominator)
    return d

"""Feynman-diagram enumeration and the shared-current evaluation plan.

Processes with one heavy-quark line and n gluons (g g -> t t~ + (n-2) g), all tree-level
diagrams in Feynman gauge built from the quark-gluon, three-gluon and four-gluon
vertices; and pure-gluon g g -> g g.

A diagram is an ordered tuple of gluon trees ("blocks") attached along the quark line,
from the outgoing top (row spinor ubar) to the outgoing antitop (column spinor v).  A tree
is a leaf ("L", i), a three-gluon node ("V3", a, b) or one colour structure of a
four-gluon node ("V4", k, a, b, c); the tree's root leg is the gluon line that meets the
quark line (for gg -> gg: the external gluon n-1).  Children are kept in a canonical order
(by smallest gluon) and the colour factor and the Lorentz evaluation use that same order.

Each diagram is evaluated as ONE vertex contraction (its "amplitude") of currents that are
computed once and shared by every diagram containing the same sub-diagram:
  G(tree)          gluon current of a subtree (off-shell root leg, with propagator)
  U(blocks)        the top-side quark string ubar (i g gamma.G) S(q) ... (row spinor)
  V(blocks)        the antitop-side string S(q) (i g gamma.G) ... v (column spinor)
  JF(pre, suf)     the quark line with a gap: the gluon current it emits
The amplitude vertex of a diagram is either a quark-gluon vertex on the line (FFV) or the
root vertex of one of its trees (VVV / VVVV with the JF current as one leg); it is chosen
per diagram, greedily, to minimise the total cost of the distinct currents.
"""
from fractions import Fraction
from functools import lru_cache
from itertools import combinations

from . import colour

# ---------------------------------------------------------------------------------------
# trees and diagrams


def leaves(t):
    if t[0] == "L":
        return (t[1],)
    kids = t[1:] if t[0] == "V3" else t[2:]
    out = ()
    for k in kids:
        out += leaves(k)
    return tuple(sorted(out))


def children(t):
    if t[0] == "L":
        return ()
    return t[1:] if t[0] == "V3" else t[2:]


def _splits2(S):
    """unordered partitions of the tuple S into two non-empty parts; the first part holds
    S[0]"""
    first, rest = S[0], S[1:]
    for r in range(0, len(rest)):
        for c in combinations(rest, r):
            A = (first,) + c
            B = tuple(x for x in rest if x not in c)
            if B:
                yield A, B


def _splits3(S):
    for A, R in _splits2(S):
        if len(R) < 2:
            continue
        for B, C in _splits2(R):
            yield A, B, C


@lru_cache(maxsize=None)
def trees(S):
    """all gluon trees whose leaves are the sorted tuple S (four-gluon nodes once per
    colour structure)"""
    if len(S) == 1:
        return (("L", S[0]),)
    out = []
    for A, B in _splits2(S):
        for ta in trees(A):
            for tb in trees(B):
                out.append(("V3", ta, tb))
    for A, B, C in _splits3(S):
        for ta in trees(A):
            for tb in trees(B):
                for tc in trees(C):
                    for k in range(3):
                        out.append(("V4", k, ta, tb, tc))
    return tuple(out)


def feynman_count(t):
    """number of Feynman diagrams a structure counts for: a four-gluon node's three colour
    structures are one diagram"""
    if t[0] == "L":
        return 1
    return 1


def quark_line_diagrams(n):
    """all diagrams for one quark line and n gluons: ordered tuples of trees whose leaves
    partition {0..n-1}; four-gluon colour structures are separate entries"""
    out = []

    def rec(remaining, prefix):
        if not remaining:
            out.append(tuple(prefix))
            return
        rem = tuple(sorted(remaining))
        for r in range(1, len(rem) + 1):
            for blk in combinations(rem, r):
                for t in trees(blk):
                    rec(remaining - set(blk), prefix + [t])

    rec(set(range(n)), [])
    return out


def n_four_vertices(t):
    if t[0] == "L":
        return 0
    own = 1 if t[0] == "V4" else 0
    return own + sum(n_four_vertices(c) for c in children(t))


def is_canonical_structure(d):
    """True for one representative per Feynman diagram: all four-gluon nodes at k = 0"""
    def ok(t):
        if t[0] == "L":
            return True
        if t[0] == "V4" and t[1] != 0:
            return False
        return all(ok(c) for c in children(t))
    return all(ok(t) for t in d)


def tree_colour(t):
    if t[0] == "L":
        return colour.leaf(t[1])
    if t[0] == "V3":
        return colour.three_vertex(tree_colour(t[1]), tree_colour(t[2]))
    return colour.four_vertex(t[1], tree_colour(t[2]), tree_colour(t[3]), tree_colour(t[4]))


def diagram_colour(d, kind):
    """{ordering: coefficient} of the diagram's colour factor in the flow basis.
    kind 'qline': (T^s)_{ij}; kind 'gluon': Tr(t^{root} T^s), coefficient doubled (the
    root gluon closes the string as 2 Tr(t^root ...))."""
    if kind == "qline":
        return colour.string_product([tree_colour(t) for t in d])
    e = tree_colour(d[0])
    two = colour.GaussInt(2, 0)
    return {s: two * c for s, c in e.items()}


# ---------------------------------------------------------------------------------------
# evaluation plan with shared currents

# estimated FP64 flop cost of computing each node type (the exact count is taken from the
# emitted code later; this only steers the choice of amplitude vertices)
COST = {"G3": 130, "G4": 120, "U": 150, "V": 150, "JF": 75,
        "A_FFV": 95, "A_V3": 140, "A_V4": 135}


def wf_key(t):
    return ("EXT_G", t[1]) if t[0] == "L" else ("G", t)


def node_deps(key):
    kind = key[0]
    if kind in ("EXT_G", "EXT_U", "EXT_V", "EXT_ROOT"):
        return ()
    if kind == "G":
        return tuple(wf_key(c) for c in children(key[1]))
    if kind == "U":
        blocks = key[1]
        prev = ("U", blocks[:-1]) if len(blocks) > 1 else ("EXT_U",)
        return (prev, wf_key(blocks[-1]))
    if kind == "V":
        blocks = key[1]
        nxt = ("V", blocks[1:]) if len(blocks) > 1 else ("EXT_V",)
        return (nxt, wf_key(blocks[0]))
    if kind == "JF":
        pre, suf = key[1], key[2]
        return (("U", pre) if pre else ("EXT_U",), ("V", suf) if suf else ("EXT_V",))
    raise ValueError(key)


def node_cost(key):
    kind = key[0]
    if kind.startswith("EXT"):
        return 0
    if kind == "G":
        return COST["G3"] if key[1][0] == "V3" else COST["G4"]
    return COST[kind]


def amplitude_options(d, kind):
    """list of (option, deps, cost) for diagram d"""
    opts = []
    if kind == "gluon":
        t = d[0]
        deps = (("EXT_ROOT",),) + tuple(wf_key(c) for c in children(t))
        opts.append((("ROOT", 0), deps, COST["A_V3"] if t[0] == "V3" else COST["A_V4"]))
        return opts
    m = len(d)
    for j in range(m):
        pre, suf = d[:j], d[j + 1:]
        deps = (("U", pre) if pre else ("EXT_U",), ("V", suf) if suf else ("EXT_V",), wf_key(d[j]))
        opts.append((("FFV", j), deps, COST["A_FFV"]))
        t = d[j]
        if t[0] != "L":
            deps = (("JF", pre, suf),) + tuple(wf_key(c) for c in children(t))
            opts.append((("ROOT", j), deps, COST["A_V3"] if t[0] == "V3" else COST["A_V4"]))
    return opts


class Plan:
    """the chosen amplitude vertex of every diagram and the closure of needed nodes"""

    def __init__(self, diagrams, kind, passes=6):
        self.diagrams = diagrams
        self.kind = kind
        self.options = [amplitude_options(d, kind) for d in diagrams]
        self.ref = {}
        self.choice = [None] * len(diagrams)
        self._closure_cache = {}
        for _ in range(passes):
            changed = False
            for i in range(len(diagrams)):
                if self.choice[i] is not None:
                    self._release(self.options[i][self.choice[i]][1])
                best, best_cost = None, None
                for oi, (_, deps, c) in enumerate(self.options[i]):
                    extra = c + sum(node_cost(k) for k in self._closure(deps) if self.ref.get(k, 0) == 0)
                    if best_cost is None or extra < best_cost:
                        best, best_cost = oi, extra
                if best != self.choice[i]:
                    changed = True
                self.choice[i] = best
                self._acquire(self.options[i][best][1])
            if not changed:
                break

    def _closure(self, deps):
        out = set()
        stack = list(deps)
        while stack:
            k = stack.pop()
            if k in out:
                continue
            out.add(k)
            stack.extend(node_deps(k))
        return out

    def _acquire(self, deps):
        for k in self._closure(deps):
            self.ref[k] = self.ref.get(k, 0) + 1

    def _release(self, deps):
        for k in self._closure(deps):
            self.ref[k] -= 1

    def nodes(self):
        return {k for k, v in self.ref.items() if v > 0}

    def amplitudes(self):
        """[(diagram index, option, deps)]"""
        return [(i, self.options[i][c][0], self.options[i][c][1]) for i, c in enumerate(self.choice)]

    def estimated_cost(self):
        return sum(node_cost(k) for k in self.nodes()) + \
            sum(self.options[i][c][2] for i, c in enumerate(self.choice))


# ---------------------------------------------------------------------------------------
# evaluation order with a small live set


def node_size(key, remat_ext=False):
    """registers (FP64 VGPRs) a computed node occupies while live; external wavefunctions
    that are recomputed at each use occupy none"""
    if key[0].startswith("EXT") and (remat_ext is True or
                                     (remat_ext == "gluons" and key[0] in ("EXT_G", "EXT_ROOT")) or
                                     (remat_ext == "gluons_lds" and key[0] == "EXT_G") or
                                     (remat_ext == "spinors" and key[0] in ("EXT_U", "EXT_V"))):
        return 0
    if key[0] == "EXT_G" or key[0] == "EXT_ROOT":
        return 14   # eps^0 = 0 and Im eps^3 = 0
    return 16


def schedule(plan, remat_ext=False, amps=None):
    """Order the amplitudes (and the nodes they need, computed just before their first
    use) greedily so that few computed currents are live at once: at each step take the
    amplitude that needs the fewest new registers net of the registers it frees.
    amps: the units to order (default: the plan's amplitudes), each (diagram index, option,
    deps); a unit may stand for several amplitudes evaluated in a row (deps: all of theirs).
    Returns the units in evaluation order."""
    amps = plan.amplitudes() if amps is None else amps
    nodes = plan.nodes()
    consumers = {k: 0 for k in nodes}
    for k in nodes:
        for d in node_deps(k):
            consumers[d] += 1
    for _, _, deps in amps:
        for d in deps:
            consumers[d] += 1
    pending = dict(consumers)
    computed = set()

    def missing(deps):
        out = []
        seen = set()

        def rec(k):
            if k in computed or k in seen:
                return
            for d in node_deps(k):
                rec(d)
            seen.add(k)
            out.append(k)
        for d in deps:
            rec(d)
        return out

    def score(deps):
        new = missing(deps)
        add = sum(node_size(k, remat_ext) for k in new)
        dec = {}
        for k in new:
            for d in node_deps(k):
                dec[d] = dec.get(d, 0) + 1
        for d in deps:
            dec[d] = dec.get(d, 0) + 1
        freed = 0
        newset = set(new)
        for d, c in dec.items():
            total = pending[d] + (consumers[d] if d in newset else 0)
            if c >= total:
                freed += node_size(d, remat_ext)
        return add - freed, add

    remaining = list(range(len(amps)))
    order = []
    while remaining:
        best, best_s = None, None
        for idx in remaining:
            s = score(amps[idx][2])
            if best_s is None or s < best_s:
                best, best_s = idx, s
        remaining.remove(best)
        deps = amps[best][2]
        for k in missing(deps):
            computed.add(k)
            for d in node_deps(k):
                pending[d] -= 1
        for d in deps:
            pending[d] -= 1
        order.append(amps[best])
    return order


def schedule_window(amps, nodes, jamp_sets, beta, window, remat_ext=False):
    """Greedy order like `schedule`, with an extra cost of `beta` per jamp of the candidate
    amplitude that is not in an LRU window of `window` jamps (jamp locality: fewer window
    evictions).  amps: [(diagram index, option, deps)]; jamp_sets[diagram] = jamp indices."""
    import collections
    consumers = {k: 0 for k in nodes}
    for k in nodes:
        for d in node_deps(k):
            consumers[d] += 1
    for _, _, deps in amps:
        for d in deps:
            consumers[d] += 1
    pending = dict(consumers)
    computed = set()
    win = collections.OrderedDict()

    def missing(deps):
        out, seen = [], set()

        def rec(k):
            if k in computed or k in seen:
                return
            for d in node_deps(k):
                rec(d)
            seen.add(k)
            out.append(k)
        for d in deps:
            rec(d)
        return out

    def score(i):
        deps = amps[i][2]
        new = missing(deps)
        add = sum(node_size(k, remat_ext) for k in new)
        dec = {}
        for k in new:
            for d in node_deps(k):
                dec[d] = dec.get(d, 0) + 1
        for d in deps:
            dec[d] = dec.get(d, 0) + 1
        freed = 0
        newset = set(new)
        for d, c in dec.items():
            total = pending[d] + (consumers[d] if d in newset else 0)
            if c >= total:
                freed += node_size(d, remat_ext)
        miss = sum(1 for j in jamp_sets[amps[i][0]] if j not in win)
        return (add - freed + beta * miss, add)

    remaining = list(range(len(amps)))
    order = []
    while remaining:
        best = min(remaining, key=score)
        remaining.remove(best)
        deps = amps[best][2]
        for k in missing(deps):
            computed.add(k)
            for d in node_deps(k):
                pending[d] -= 1
        for d in deps:
            pending[d] -= 1
        for j in sorted(jamp_sets[amps[best][0]]):
            if j in win:
                win.move_to_end(j)
            else:
                if len(win) >= window:
                    win.popitem(last=False)
                win[j] = 1
        order.append(amps[best])
    return order


def proportional_classes(jcoef, perm_index):
    """Amplitude entries whose colour coefficients are proportional: [[(entry, (ur, ui)), ..]],
    where entry m's coefficients are (ur + i ui) times the first member's on every colour flow
    (a unit of the Gaussian integers).  Such entries add to the same jamps in the same ratio, so
    their amplitudes can be summed first (J_k += c_k (a_1 + u_2 a_2 + ..)): one set of jamp
    updates per class instead of one per entry.  Classes are listed by their first entry."""
    groups = {}
    for di, coef in enumerate(jcoef):
        co = {perm_index[q]: c for q, c in coef.items()}
        k0 = min(co)
        c0 = co[k0]
        n0 = c0.re * c0.re + c0.im * c0.im
        key, unit = [], None
        for k in sorted(co):
            # co[k] / c0 as an exact pair of fractions
            c = co[k]
            r = (Fraction(c.re * c0.re + c.im * c0.im, n0), Fraction(c.im * c0.re - c.re * c0.im, n0))
            key.append((k, r))
        key = tuple(key)
        groups.setdefault(key, []).append((di, co))
    out = []
    for members in sorted(groups.values(), key=lambda m: m[0][0]):
        d0, co0 = members[0]
        k0 = min(co0)
        row = []
        for di, co in members:
            a, b = co[k0], co0[k0]   # unit u with co = u * co0
            nb = b.re * b.re + b.im * b.im
            ur = (a.re * b.re + a.im * b.im) // nb
            ui = (a.im * b.re - a.re * b.im) // nb
            assert ur * b.re - ui * b.im == a.re and ur * b.im + ui * b.re == a.im
            assert (ur, ui) in ((1, 0), (-1, 0), (0, 1), (0, -1))
            row.append((di, (ur, ui)))
        out.append(row)
    return out


def closure(deps):
    need, st = set(), list(deps)
    while st:
        x = st.pop()
        if x in need:
            continue
        need.add(x)
        st.extend(node_deps(x))
    return need


def segment_plan(plan, jamp_sets, n_segments, beta, window, amps=None, cut="amps", remat_ext=False):
    """Cut the jamp-aware order into n_segments contiguous pieces (one kernel each, which
    recomputes the currents it needs) and reorder each piece the same way.  amps: the units
    to order (default: the plan's amplitudes; see `schedule`).  cut: "amps" cuts where the
    amplitudes evaluated so far (a unit counts its members) reach k / n_segments of all, so the
    kernels share the work evenly; "units" cuts into equal numbers of units; a function of the
    unit gives each unit that weight instead."""
    amps = plan.amplitudes() if amps is None else amps
    order = schedule_window(amps, plan.nodes(), jamp_sets, beta, window, remat_ext)
    if callable(cut):
        size = [cut(u) for u in order]
    else:
        size = [len(u[1][1]) if (cut == "amps" and u[1][0] == "CLASS") else 1 for u in order]
    total = sum(size)
    cuts, acc = [0], 0
    for i, w in enumerate(size):
        acc += w
        if len(cuts) < n_segments and acc * n_segments >= len(cuts) * total:
            cuts.append(i + 1)
    cuts += [len(order)] * (n_segments + 1 - len(cuts))
    segs = []
    for k in range(n_segments):
        piece = order[cuts[k]:cuts[k + 1]]
        need = closure([d for _, _, deps in piece for d in deps])
        segs.append(schedule_window(piece, need, jamp_sets, beta, window, remat_ext))
    return segs


def window_program(order, jamp_sets, window, policy="opt"):
    """Static allocation of jamps to `window` slots along `order`.  Returns, per amplitude,
    [(jamp, slot, flush)] where flush is None or (slot, partial index, jamp) to write out
    before the slot is reused, plus the final flushes and the jamp of every partial slot.
    policy: when a slot must be freed, "opt" evicts the jamp whose next use lies furthest ahead
    (or never comes), which the static order makes known (Belady's optimal replacement);
    "lru" the least recently used."""
    import collections
    seq = [sorted(jamp_sets[u[0]]) for u in order]
    uses = collections.defaultdict(list)
    for i, js in enumerate(seq):
        for j in js:
            uses[j].append(i)

    def next_use(j, i):
        """first step after step i that uses jamp j"""
        lst = uses[j]
        lo, hi = 0, len(lst)
        while lo < hi:
            mid = (lo + hi) // 2
            if lst[mid] <= i:
                lo = mid + 1
            else:
                hi = mid
        return lst[lo] if lo < len(lst) else len(seq)

    win = collections.OrderedDict()   # jamp -> slot, least recently used first
    free = list(range(window))[::-1]
    partial_jamp = []
    steps = []
    for i, js in enumerate(seq):
        ops = []
        for j in js:
            flush = None
            if j in win:
                win.move_to_end(j)
            else:
                if not free:
                    if policy == "lru":
                        jj = next(iter(win))
                    else:
                        cand = [x for x in win if x not in js]
                        jj = max(cand, key=lambda x: (next_use(x, i), -list(win).index(x)))
                    s = win.pop(jj)
                    flush = (s, len(partial_jamp), jj)
                    partial_jamp.append(jj)
                    free.append(s)
                win[j] = free.pop()
            ops.append((j, win[j], flush))
        steps.append(ops)
    final = []
    for jj, s in win.items():
        final.append((s, len(partial_jamp), jj))
        partial_jamp.append(jj)
    return steps, final, partial_jamp

"""CPU tests of the process generator (diagram enumeration, colour algebra, evaluation
plan, jamp window) against independent definitions."""
import collections
import itertools
import math
import re

import numpy as np
import pytest

import oracle
from paper_2210_11122_amd.gen import colour, diagrams as D, emit

# Gell-Mann matrices, written out here (not taken from the generator)
_L = np.zeros((8, 3, 3), complex)
_L[0][0, 1] = _L[0][1, 0] = 1
_L[1][0, 1], _L[1][1, 0] = -1j, 1j
_L[2][0, 0], _L[2][1, 1] = 1, -1
_L[3][0, 2] = _L[3][2, 0] = 1
_L[4][0, 2], _L[4][2, 0] = -1j, 1j
_L[5][1, 2] = _L[5][2, 1] = 1
_L[6][1, 2], _L[6][2, 1] = -1j, 1j
_L[7] = np.diag([1, 1, -2]) / math.sqrt(3)
T = _L / 2


@pytest.mark.parametrize("n,count,amps", [(2, 3, 3), (3, 16, 18), (4, 123, 159), (5, 1240, 1890)])
def test_diagram_counts(n, count, amps):
    ds = D.quark_line_diagrams(n)
    assert len(ds) == amps
    assert sum(1 for d in ds if D.is_canonical_structure(d)) == count
    for d in ds:
        assert sorted(g for t in d for g in D.leaves(t)) == list(range(n))


def test_gluon_trees():
    # trees with 1..4 leaves under a root leg: 1, 1, 4 (3 + one quartic), 25
    for k, want in [(1, 1), (2, 1), (3, 4), (4, 25)]:
        ts = D.trees(tuple(range(k)))
        assert sum(1 for t in ts if D.is_canonical_structure((t,))) == want
    # gg -> gg: s, t, u and the contact diagram
    assert sum(1 for t in D.trees((0, 1, 2)) if D.is_canonical_structure((t,))) == 4


@pytest.mark.parametrize("proc,n", [("gg_tt", 2), ("gg_ttg", 3), ("gg_ttgg", 4), ("gg_ttggg", 5)])
def test_colour_matrix_exact_vs_oracle(proc, n):
    perms, C = colour.colour_matrix_quark_line(n)
    assert [tuple(p) for p in perms] == oracle.orderings(proc)
    Co = oracle.colour_matrix(proc)
    assert np.allclose(np.array(C, dtype=float), Co, atol=1e-12)


def test_single_trace_matrix_exact_vs_oracle():
    perms, C = colour.colour_matrix_single_trace(4)
    assert [tuple(p) for p in perms] == oracle.orderings("gg_gg")
    assert np.allclose(np.array(C, dtype=float), oracle.colour_matrix("gg_gg"), atol=1e-13)


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg", "gg_gg"])
def test_colour_numerators_exact_in_fp16(name):
    P = emit.Process(name)
    h = np.array(P.cnum, dtype=np.float64)
    assert np.array_equal(h.astype(np.float16).astype(np.float64), h)


def explicit_tree(t, col, f):
    """adjoint colour vector of a subtree for explicit external colours"""
    if t[0] == "L":
        v = np.zeros(8)
        v[col[t[1]]] = 1
        return v
    if t[0] == "V3":
        A, B = explicit_tree(t[1], col, f), explicit_tree(t[2], col, f)
        return np.einsum("xab,a,b->x", f, A, B)
    k = t[1]
    A, B, C = (explicit_tree(c, col, f) for c in t[2:])
    if k == 0:
        return np.einsum("xae,bce,a,b,c->x", f, f, A, B, C)
    if k == 1:
        return np.einsum("xbe,ace,a,b,c->x", f, f, A, B, C)
    return np.einsum("xce,abe,a,b,c->x", f, f, A, B, C)


@pytest.mark.parametrize("n,n_diag", [(2, 3), (3, 18), (4, 40), (5, 60)])
def test_diagram_colour_decomposition_explicit(n, n_diag):
    """every checked diagram: explicit f/t contraction == sum_s c_s (T^s)_ij"""
    f = oracle.fabc()
    rng = np.random.default_rng(n)
    ds = D.quark_line_diagrams(n)
    idx = rng.choice(len(ds), size=min(n_diag, len(ds)), replace=False)
    for i in idx:
        d = ds[int(i)]
        dec = D.diagram_colour(d, "qline")
        for _ in range(3):
            col = rng.integers(0, 8, n)
            M = np.eye(3, dtype=complex)
            for t in d:
                M = M @ np.einsum("x,xij->ij", explicit_tree(t, col, f), T)
            S = np.zeros((3, 3), complex)
            for seq, c in dec.items():
                P = np.eye(3, dtype=complex)
                for g in seq:
                    P = P @ T[col[g]]
                S += complex(c.re, c.im) * P
            assert np.allclose(M, S, atol=1e-12)


def test_pure_gluon_decomposition_explicit():
    f = oracle.fabc()
    rng = np.random.default_rng(3)
    for t in D.trees((0, 1, 2)):
        dec = D.diagram_colour((t,), "gluon")
        for _ in range(4):
            col = rng.integers(0, 8, 4)
            X = explicit_tree(t, col, f)[col[3]]
            S = 0
            for seq, c in dec.items():
                P = T[col[3]].copy()
                for g in seq:
                    P = P @ T[col[g]]
                S += complex(c.re, c.im) * np.trace(P)
            assert abs(X - S) < 1e-12


def expand_sums(text):
    """the text with every operand-sum node (const W4<R> sN = ...;) written out at its uses"""
    defs = dict(re.findall(r"const W4<R> (s\d+) = (w4_acc[^;]*);", text))
    return re.sub(r"\b(s\d+)\b(?! =)", lambda m: defs.get(m.group(1), m.group(1)), text)


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg"])
def test_every_diagram_evaluated_once(name):
    P = emit.Process(name)
    # the helicity-wave kernel (the one-lane-per-event kernel after it repeats the program)
    src = P.source().split("void amp_lanes(")[0]
    # one vertex line per group of entries that differ in one operand (the vertex on the sum of
    # those operands), each entry in exactly one group
    lines = re.findall(r"^\s+a = amp_(.*)$", expand_sums(src), re.M)
    assert len(lines) == len(P.emit_groups)
    assert sum(len(g) for g in P.emit_groups) == P.n_amplitudes
    assert [ln.count("w4_acc<R") for ln in lines] == [len(g) - 1 for g in P.emit_groups]
    # every node of the plan computed exactly once; external gluons of programs that take them
    # from the LDS bases are rebuilt at each use instead; external wavefunctions kept in LDS
    # per lane are computed once at the start (one store each) and read at their uses
    names = re.findall(r"const W4<R> (w\d+) =", src)
    kept = re.findall(r"if constexpr \(XWP\[(\d+)\] >= 0\) st_w4<R>\(xw, XWP\[\d+\], lane, t\)", src)
    assert len(kept) == len(set(kept)) == len(P.xw_init) >= len(set().union(*emit.EXT_IN_LDS.get(name, ((), ()))))
    assert all(f"XW({k})" in src for k in kept)
    nodes = P.plan.nodes()
    if name in emit.GLUONS_FROM_LDS:
        nodes = {k for k in nodes if k[0] != "EXT_G"}
        assert "ext_vec<" not in src and len(re.findall(r"ext_vec_b<R>\(g\d+_\d+, lam\[\d\], ", src)) > 0
    assert len(names) == len(set(names)) and len(names) + len(kept) == len(nodes)


def test_plan_covers_every_diagram_with_its_own_subdiagrams():
    """each amplitude's dependencies reproduce exactly the diagram's blocks"""
    ds = D.quark_line_diagrams(4)
    plan = D.Plan(ds, "qline")
    for di, opt, deps in plan.amplitudes():
        d = ds[di]
        kind, j = opt
        leaves = set()
        for k in D.closure(deps):
            if k[0] == "EXT_G":
                leaves.add(k[1])
        assert leaves == set(range(4))
        if kind == "FFV":
            assert deps[2] == D.wf_key(d[j])


def test_window_program_reproduces_direct_accumulation():
    """replay the gg_ttggg jamp window (LRU slots, flushes, partial slots, reduction) with
    random amplitudes and compare with direct accumulation of every diagram"""
    P = emit.Process("gg_ttggg")
    P.source()  # builds the segments and the partial-slot map
    perm_index = {tuple(p): i for i, p in enumerate(P.perms)}
    jsets = [set(perm_index[q] for q in P.jcoef[i]) for i in range(len(P.diagrams))]
    n_seg, window, beta = P.segments
    segs = P.segment_orders
    rng = np.random.default_rng(0)
    amp = rng.normal(size=len(P.diagrams)) + 1j * rng.normal(size=len(P.diagrams))
    direct = np.zeros(P.nc, complex)
    for di in range(len(P.diagrams)):
        for q, c in P.jcoef[di].items():
            direct[perm_index[q]] += complex(c.re, c.im) * amp[di]
    partial = np.zeros(P.nslot, complex)
    base = 0
    seen = []
    for order in segs:
        steps, final, pj = D.window_program(order, jsets, window)
        win = np.zeros(window, complex)
        for unit, ops in zip(order, steps):
            # a unit: entries with proportional colour coefficients, summed with their factors
            members = P.unit_members(unit)
            seen += [m[0] for m in members]
            a = sum(complex(*m[3]) * amp[m[0]] for m in members)
            di = members[0][0]
            coef = {perm_index[q]: c for q, c in P.jcoef[di].items()}
            for m in members:
                cm = {perm_index[q]: complex(c.re, c.im) for q, c in P.jcoef[m[0]].items()}
                assert all(abs(cm[k] - complex(*m[3]) * complex(coef[k].re, coef[k].im)) == 0 for k in coef)
            for j, slot, flush in ops:
                if flush is not None:
                    partial[base + flush[1]] = win[flush[0]]
                    win[flush[0]] = 0
                c = coef[j]
                win[slot] += complex(c.re, c.im) * a
        for slot, pidx, _ in final:
            partial[base + pidx] = win[slot]
        base += len(pj)
    assert sorted(seen) == list(range(len(P.diagrams)))
    assert base == P.nslot
    red = np.zeros(P.nc, complex)
    for s, j in enumerate(P.partial_jamp):
        red[j] += partial[s]
    assert np.allclose(red, direct, atol=1e-12 * np.abs(direct).max())


def test_emitted_window_kernels_and_reduction_accumulate_every_jamp():
    """interpret the emitted gg_ttggg segment kernels macro by macro, in program order (LDS
    window slots: JADD, JTAKE, JLAST; registers; partial slots in HBM: JPUT), then the emitted
    reduction tables (slot_offset, slot_list); with random amplitudes the reduced jamps must
    equal direct accumulation, every partial slot written exactly once"""
    import re
    P = emit.Process("gg_ttggg")
    src = P.source()
    perm_index = {tuple(p): i for i, p in enumerate(P.perms)}
    jsets = [set(perm_index[q] for q in P.jcoef[i]) for i in range(len(P.diagrams))]
    n_seg, window, beta = P.segments
    segs = P.segment_orders
    rng = np.random.default_rng(1)
    amp = rng.normal(size=len(P.diagrams)) + 1j * rng.normal(size=len(P.diagrams))
    direct = np.zeros(P.nc, complex)
    for di in range(len(P.diagrams)):
        for q, c in P.jcoef[di].items():
            direct[perm_index[q]] += complex(c.re, c.im) * amp[di]
    partial = np.full(P.nslot, np.nan + 1j * np.nan)
    written = np.zeros(P.nslot, int)
    jadd = re.compile(r"JADD\((\d+), ([01]), ([^;]*)\);")
    macro = re.compile(r"(JTAKE|JLAST|JPUT)\((\d+), (\d+)\);")
    for k, order in enumerate(segs):
        text = P.extra_files[f"proc_gg_ttggg_amp_seg{k}.hip"]
        body = expand_sums(text[text.index("#define SDEACC"):text.index("\n    if constexpr (SDE) {\n")])
        win = np.zeros(window, complex)
        fr = {}
        assert sorted(e for g in P.segment_emit_groups[k] for e, _ in g) == sorted(
            m[0] for unit in order for m in P.unit_members(unit))
        it = iter(P.segment_emit_groups[k])
        a = sa = None
        acc = {"sa.r += a.r; sa.i += a.i;": 1, "sa.r -= a.r; sa.i -= a.i;": -1,
               "sa.r -= a.i; sa.i += a.r;": 1j, "sa.r += a.i; sa.i -= a.r;": -1j}
        for line in body.splitlines()[1:]:
            if re.match(r"\s*a = amp", line):
                # the line's vertex on operand sums is the sum of its entries' amplitudes with these
                # units (test_emitted_vertices_on_sums_equal_the_diagram_amplitudes checks the text)
                grp = next(it)
                a = sum(complex(*u) * amp[e] for e, u in grp)
                continue
            if line.strip() == "sa = a;":
                sa = a
                continue
            if line.strip() in acc:
                sa = sa + acc[line.strip()] * a
                continue
            for s_, ri, v in jadd.findall(line):
                env = {"ar": a.real, "ai": a.imag, "sar": sa.real if sa is not None else 0,
                       "sai": sa.imag if sa is not None else 0}
                val = eval(v.replace("(R)", "").replace("sa.r", "sar").replace("sa.i", "sai")
                           .replace("a.r", "ar").replace("a.i", "ai"), env)
                win[int(s_)] += val if ri == "0" else 1j * val
            for m, x, y in macro.findall(line):
                x, y = int(x), int(y)
                if m == "JTAKE":
                    fr[y], win[x] = win[x], 0
                elif m == "JLAST":
                    fr[y] = win[x]
                else:
                    partial[x] = fr.pop(y)
                    written[x] += 1
        assert next(it, None) is None and not fr
    assert np.all(written == 1)
    offs = [int(v) for v in re.search(r"slot_offset\[NC \+ 1\] = \{([^}]*)\}", src).group(1).split(",")]
    lst = [int(v) for v in re.search(r"slot_list\[NSLOT\] = \{([^}]*)\}", src).group(1).split(",")]
    red = np.array([sum(partial[lst[i]] for i in range(offs[c], offs[c + 1])) for c in range(P.nc)])
    assert np.allclose(red, direct, rtol=0, atol=1e-12 * np.abs(direct).max())


@pytest.mark.parametrize("name", ["gg_ttg", "gg_ttgg", "gg_gg"])
def test_emitted_kernel_accumulates_every_jamp(name):
    """interpret the emitted single-kernel program (amplitudes, class sums sa, JADD updates) with
    random amplitudes: every jamp equals direct accumulation of every entry's colour coefficients"""
    P = emit.Process(name)
    src = P.source()
    perm_index = {tuple(p): i for i, p in enumerate(P.perms)}
    rng = np.random.default_rng(2)
    amp = rng.normal(size=len(P.diagrams)) + 1j * rng.normal(size=len(P.diagrams))
    direct = np.zeros(P.nc, complex)
    for di in range(len(P.diagrams)):
        for q, c in P.jcoef[di].items():
            direct[perm_index[q]] += complex(c.re, c.im) * amp[di]
    body = expand_sums(src[src.index("#define SDEACC"):src.index("\n    if constexpr (SDE) {\n")])
    jadd = re.compile(r"JADD\((\d+), ([01]), ([^;]*)\);")
    acc = {"sa.r += a.r; sa.i += a.i;": 1, "sa.r -= a.r; sa.i -= a.i;": -1,
           "sa.r -= a.i; sa.i += a.r;": 1j, "sa.r += a.i; sa.i -= a.r;": -1j}
    assert sorted(P.emit_order) == list(range(len(P.diagrams)))
    assert sorted(e for g in P.emit_groups for e, _ in g) == list(range(len(P.diagrams)))
    it = iter(P.emit_groups)
    J = np.zeros(P.nc, complex)
    a = sa = None
    for line in body.splitlines()[1:]:
        t = line.strip()
        if re.match(r"a = amp", t):
            # a vertex on a sum of operands stands for the sum of its entries' amplitudes
            grp = next(it)
            units = [(int(x), int(y)) for x, y in re.findall(r"w4_acc<R, (-?\d), (-?\d)>", t)]
            assert units[::-1] == [u for _, u in grp[1:]]   # nested: the last added outermost
            a = sum(complex(*u) * amp[e] for e, u in grp)
        elif t == "sa = a;":
            sa = a
        elif t in acc:
            sa = sa + acc[t] * a
        for s_, ri, v in jadd.findall(line):
            env = {"ar": a.real, "ai": a.imag, "sar": sa.real if sa is not None else 0,
                   "sai": sa.imag if sa is not None else 0}
            val = eval(v.replace("(R)", "").replace("sa.r", "sar").replace("sa.i", "sai")
                       .replace("a.r", "ar").replace("a.i", "ai"), env)
            J[int(s_)] += val if ri == "0" else 1j * val
    assert next(it, None) is None
    assert np.allclose(J, direct, rtol=0, atol=1e-12 * np.abs(direct).max())
    if name == "gg_ttgg":
        # entries with proportional coefficients share one set of updates: 336 instead of 672
        assert len(jadd.findall(body)) == 2 * 336


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg"])
def test_single_diagram_data_matches_oracle(name):
    """per Feynman diagram (matched by internal lines) the generator's colour weights
    K = c^dagger C c of its entries equal the oracle's numeric colour sums"""
    import collections
    from oracle import diagrams as Dg
    P = emit.Process(name)
    P.source()
    g = collections.defaultdict(list)
    for fd, k in zip(P.fd_index, P.kweight):
        g[P.lines[fd]].append(round(k, 9))
    o = collections.defaultdict(list)
    for (d, s), k in zip(Dg.entries(name), Dg.colour_weights_K(name)):
        o[Dg.descriptor(name, d)].append(round(k, 9))
    assert set(g) == set(o) and len(g) == P.n_diagrams
    for key in g:
        assert sorted(g[key]) == sorted(o[key])


@pytest.mark.parametrize("name", ["gg_ttgg", "gg_ttggg"])
def test_spare_waves_write_nothing(name):
    """with several waves (helicities) per workgroup, a spare wave of an odd last group repeats
    a helicity; every global store of the emitted kernels must sit inside a `live` guard (the
    good helicity counts of these processes are even, so the GPU tests never run a spare wave)"""
    import re
    assert emit.WAVES_PER_GROUP[name] != (1, 1)
    P = emit.Process(name)
    src = P.source()
    store = re.compile(r"(\b(o|so|po)\s*\[[^]]*\]\s*\+?=[^=])|(reinterpret_cast<double\*>\(jamp\)\[[^]]*\]\s*=[^=])")
    n_stores = 0
    for text in [src] + list(getattr(P, "extra_files", {}).values()):
        for m in re.finditer(r"__global__[^{]*void (amp_kernel|amp_seg\d+)\([^{]*\{\n", text):
            body = text[m.end():text.index("\n}\n", m.end())]
            guarded = []   # per open brace: does its block sit under a `live` test
            for line in body.splitlines():
                code = line.strip()
                if code.startswith("#define"):
                    if code.startswith("#define JPUT"):
                        assert "if (live)" in code, code
                    continue
                if store.search(code):
                    n_stores += 1
                    assert "live" in code or any(guarded), code
                for ch in code:
                    if ch == "{":
                        guarded.append("if (live" in code)
                    elif ch == "}":
                        guarded.pop()
            assert not guarded
    assert n_stores > 0


@pytest.mark.parametrize("name,merged", [("gg_tt", 0), ("gg_ttg", 0), ("gg_ttgg", 36), ("gg_ttggg", 810)])
def test_shared_vertices_differ_in_one_operand_of_equal_momentum(name, merged):
    """the groups that share one vertex: within one colour class, the same vertex (and four-gluon
    colour structure), the same nodes in every slot but one, and in that slot nodes of the same
    external legs (so the same momentum enters the vertex); the groups cover every member once,
    the first starts with the class's first member"""
    from paper_2210_11122_amd.gen import diagrams as D
    P = emit.Process(name)
    P.source()
    saved = 0
    for unit in P.units():
        members = P.unit_members(unit)
        groups = P._linear_groups(members)
        assert sorted(i for g in groups for i in g) == list(range(len(members)))
        assert groups[0][0] == 0
        for g in groups:
            saved += len(g) - 1
            heads = set()
            for i in g:
                di, (kind, j), deps, _ = members[i]
                t = None if kind == "FFV" else P.diagrams[di][j]
                heads.add("FFV" if t is None else (t[0], t[1] if t[0] == "V4" else None))
            assert len(heads) == 1
            d0 = members[g[0]][2]
            slots = {k for i in g[1:] for k in range(len(d0)) if members[i][2][k] != d0[k]}
            assert len(slots) <= 1
            if slots:
                k = slots.pop()
                def legs(node):
                    if node[0] == "G":
                        return tuple(sorted(D.leaves(node[1])))
                    if node[0] == "EXT_G":
                        return (node[1],)
                    if node[0] in ("U", "V"):
                        return node[0], tuple(sorted(x for b in node[1] for x in D.leaves(b)))
                    return node
                assert len({legs(members[i][2][k]) for i in g}) == 1, (unit[0], g)
    assert saved == merged


# arguments of each emitted routine that are wavefunctions (the others are momenta or couplings)
_WF_ARGS = {"vvv_cur": (0, 2), "vvvv_cur": (0, 1, 2), "fstr_u": (0, 1), "fstr_v": (0, 1), "jf": (0, 1),
            "amp_ffv": (0, 1, 2), "amp_vvv": (0, 2, 4), "amp_vvvv": (0, 1, 2, 3), "w4_acc": (0, 1)}


def _split_call(e):
    """'f<T..>(a, b, ..)' -> ('f<T..>', [a, b, ..]) split at the top-level commas; else None"""
    m = re.match(r"^(\w+(?:<[^>]*>)?)\((.*)\)$", e.strip())
    if not m:
        return None
    args, depth, cur = [], 0, ""
    for ch in m.group(2):
        if ch == "," and depth == 0:
            args.append(cur.strip())
            cur = ""
            continue
        depth += ch in "(<"
        depth -= ch in ")>"
        cur += ch
    args.append(cur.strip())
    return m.group(1), args


def _symbolic_terms(expr, defs, memo):
    """the emitted expression as sum_j c_j T_j: every operand sum (w4_acc) distributed through the
    vertices, which are linear in each wavefunction; T_j is a tree of routine names down to the
    external states, ('ext', particle)"""
    expr = expr.strip()
    if expr in memo:
        return memo[expr]
    if re.fullmatch(r"[wsz]\d+|y\d+_\d+|XW\(\d+\)", expr):
        out = _symbolic_terms(defs[expr], defs, memo)
    else:
        fn, args = _split_call(expr)
        base = fn.split("<")[0]
        if base.startswith("ext_"):
            p = re.search(r"PM\((\d+)\)|m\d+_(\d+)", args[0])
            out = [(1, ("ext", int(p.group(1) or p.group(2))))]
        elif base == "w4_acc":
            u = complex(*(int(x) for x in re.findall(r"-?\d+", fn[fn.index("<"):])))
            out = _symbolic_terms(args[0], defs, memo) + [(c * u, t) for c, t in _symbolic_terms(args[1], defs, memo)]
        else:
            tag = base + ("" if base not in ("vvvv_cur", "amp_vvvv") else fn[fn.index(","):])
            out = [(1, ())]
            for i in _WF_ARGS[base]:
                out = [(c * c2, t + (t2,)) for c, t in out for c2, t2 in _symbolic_terms(args[i], defs, memo)]
            out = [(c, (tag,) + t) for c, t in out]
    memo[expr] = out
    return out


def _node_tree(P, key):
    """the same tree from the generator's plan node, independently of the emitted text"""
    kind = key[0]
    if kind == "EXT_G":
        return ("ext", P.gpar[key[1]])
    if kind in ("EXT_U", "EXT_V"):
        return ("ext", 2 if kind == "EXT_U" else 3)
    deps = tuple(_node_tree(P, k) for k in D.node_deps(key))
    if kind == "G":
        t = key[1]
        return (("vvv_cur",) if t[0] == "V3" else (f"vvvv_cur, {t[1]}>",)) + deps
    return ({"U": "fstr_u", "V": "fstr_v", "JF": "jf"}[kind],) + deps


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"])
def test_emitted_vertices_on_sums_equal_the_diagram_amplitudes(name):
    """expand every `a = amp_...` line of the emitted kernels symbolically (operand sums distributed
    through the vertices): it equals the sum of its diagram amplitudes, each with its unit factor,
    built from the plan's nodes"""
    P = emit.Process(name)
    src = P.source()
    if P.segments:
        texts = [P.extra_files[f"proc_{name}_amp_seg{k}.hip"] for k in range(P.segments[0])]
        groups = P.segment_emit_groups
        orders = P.segment_orders
    else:
        texts, groups, orders = [src], [P.emit_groups], [None]
    members = {}
    for unit in P.units():
        for m in P.unit_members(unit):
            members[m[0]] = m
    n_lines = 0
    for text, grps in zip(texts, groups):
        body = text[text.index("#define SDEACC"):text.index("\n    if constexpr (SDE) {\n")]
        body = re.sub(r"^\s*if constexpr \(SDE\).*$", "", body, flags=re.M)
        defs = dict(re.findall(r"const W4<R> ([wsz]\d+) = ([^;]*);", body))
        # external states kept in LDS: the prefetched copies y<step>_<slot> of XW(slot)
        xw = {f"XW({k})": code for k, (code, _, _) in enumerate(P.xw_init)}
        defs.update(xw)
        defs.update({y: f"XW({k})" for y, k in re.findall(r"W4<R> (y\d+_\d+) = XW\((\d+)\);", body)})
        lines = re.findall(r"^\s*a = (amp_[^;]*);", body, re.M)
        assert len(lines) == len(grps)
        memo = {}
        for line, grp in zip(lines, grps):
            got = collections.Counter()
            for c, t in _symbolic_terms(line, defs, memo):
                got[t] += c
            want = collections.Counter()
            for e, (ur, ui) in grp:
                di, (kind, j), deps, _ = members[e]
                if kind == "FFV":
                    tag = "amp_ffv"
                else:
                    tr = P.diagrams[di][j]
                    tag = "amp_vvv" if tr[0] == "V3" else f"amp_vvvv, {tr[1]}>"
                want[(tag,) + tuple(_node_tree(P, k) for k in deps)] += complex(ur, ui)
            assert {t: c for t, c in got.items() if c != 0} == dict(want), (name, line[:120])
            n_lines += 1
    assert n_lines == sum(len(g) for g in groups)

"""Emit the HIP diagram program and the constant tables of each process.

For every process this writes ``csrc/generated/proc_<name>.hip`` with
  * the amplitude kernel, a template over the working precision (double, float), in which
    one lane evaluates one (event, helicity): external wavefunctions, the shared currents,
    one vertex contraction per Feynman diagram, and the accumulation of the diagram
    amplitudes into the colour-flow amplitudes ("jamps") with the exact coefficients of
    the colour decomposition;
  * the process descriptor (particle content, colour matrix numerators over a common
    denominator, jamp-slot map, exact algorithmic flop counts) used by the C ABI.

Flop counts are the real additions and multiplications written in ``helas.hpp`` for each
call (complex multiply = 6, complex add = 2, real x complex = 2), plus momentum sums (4 per
four-vector addition) and jamp updates (2 per update).
"""
import collections
import os
import re
from fractions import Fraction
from itertools import permutations

from . import colour, diagrams as D

# flops per helas.hpp routine (see module docstring)
FLOPS = {
    "ext_vec": 22, "ext_spinor": 26, "fstr": 141, "jf": 89, "vvv_cur": 151, "vvvv_cur": 134,
    "jf_chiral": 137, "amp_ffv_chiral": 100,
    "amp_ffv": 96, "amp_vvv": 156, "amp_vvvv": 137, "p4add": 4, "jamp": 2,
}

QCD_PROCESSES = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5}
# name -> (segment kernels, LDS jamp-window slots, weight of window misses in the schedule)
SEGMENTS = {"gg_ttggg": (14, 35, 2.0)}
# how the segments are cut from the schedule (diagrams.segment_plan): "amps" (a unit weighs its
# members), "units", or "vertices" (a unit weighs the vertices it evaluates once members share
# vertices; measured slower for gg_ttggg: per 2^17 events FP64 with 12 / 13 / 14 segments 222 / 225
# / 232 ms, mixed 127 / 130 / 135, against 219 and 125 with "amps" and 14)
SEGMENT_CUT = "amps"
# sum the amplitudes of entries with proportional colour coefficients before their jamp updates
PRESUM = True
# within such a class, evaluate the entries that differ in one wavefunction only (same vertex,
# the other operands and every momentum the same) as one vertex on the sum of those
# wavefunctions, each times its unit factor: the vertices are linear in each wavefunction
LINEAR_MERGE = True
# and form a sum of operands that several of those vertices use once, as a node of its own
SUM_NODES = False
# processes whose operand sums also pass through the vertices that made their terms, where those
# differ in one operand at the same momenta (recursively): one current on a sum instead of a sum
# of currents.  Each such sum is then a node of its own, formed once per kernel
DEEP_MERGE = {"gg_ttggg"}
# sa += u a for the units u of the Gaussian integers
ACC_TEXT = {(1, 0): "sa.r += a.r; sa.i += a.i;", (-1, 0): "sa.r -= a.r; sa.i -= a.i;",
            (0, 1): "sa.r -= a.i; sa.i += a.r;", (0, -1): "sa.r += a.i; sa.i -= a.r;"}
# read each amplitude step's momenta from LDS ahead of the previous step's jamp updates
PREFETCH_MOMENTA = True
# and keep the compiler from summing them before the step that uses them
PIN_MOMENTA = True
# name -> minimum waves per SIMD asked of the compiler for the (FP64, FP32) amplitude kernels
# (the second __launch_bounds__ argument: it caps the registers per lane at 512 / waves)
MIN_WAVES = {"gg_tt": (4, 6), "gg_ttg": (2, 3), "gg_ttgg": (1, 2), "gg_ttggg": (1, 2)}
# name -> waves per workgroup (FP64, FP32 kernels): consecutive helicities of one 64-event block
# that share the staged momenta (less LDS per wave where LDS, not registers, limits the waves).
# With several waves per group, FP32 kernels with register jamps stage them for the colour sum in
# an LDS area of their own (a single wave reuses the momentum area).  gg_tt FP64 per 2^19 events
# 0.197 -> 0.182 ms, mixed (six waves per SIMD) 0.272 -> 0.252 ms; gg_ttg FP64 per 2^20 3.14 ->
# 2.77 ms (its three LDS externals and shared momenta then fit two waves per SIMD), mixed 2.86 ->
# 2.62 ms (2.59 ms with its top spinors in LDS as well)
# The test process gg_gg has six good helicities, so its second group of four carries two spare
# waves: its parity tests cover that path.
WAVES_PER_GROUP = {"gg_tt": (4, 4), "gg_ttg": (4, 4), "gg_ttgg": (4, 4), "gg_ttggg": (4, 8), "gg_gg": (4, 4)}
# processes whose programs keep no external gluon wavefunction in registers: the workgroup
# stages each event's gluon bases in LDS once (helas.hpp, stage_gluon_basis) and every use
# rebuilds the polarisation vector from there.  It removes the FP64 kernels' spills but costs
# a multiply by the helicity sign per component at each of the many uses, plus LDS reads, and
# measured slower (gg_ttgg FP64 25.2 -> 27.4 ms per 2^19 events, with 2 / 4 waves per group to
# keep the occupancy); off
GLUONS_FROM_LDS = set()
# name -> (FP64 kernel, FP32 kernel): the external wavefunctions ("EXT_U", "EXT_V", "EXT_G", or
# "EXT_G:<j>" for gluon j) that the kernel keeps in LDS, private to each lane, instead of in
# registers across the program: computed once, read ahead of each step that uses them (as the
# momenta).  Only for processes without segment kernels.
# * gg_ttgg FP64: the top spinors, 4 KB per wave each, room made by four waves per workgroup
#   sharing the staged momenta (143 KB per workgroup, one per CU); per 2^19 events 24.89 -> 24.17
#   ms (four waves alone: 24.59 ms; a third slot, a gluon, removes every scratch spill but
#   measured 24.8 ms).
# * gg_ttgg FP32: the same two, 2 KB per wave each, with four waves per workgroup (78 KB, two per
#   CU); per 2^19 events 14.54 -> 14.20 ms (four waves alone: 14.33 ms; one spinor: 14.45 ms).
# * gg_ttg FP64: the top spinors and a gluon (no spill left); per 2^20 events 4.01 -> 3.48 ms
#   with one wave per workgroup (the spinors alone 3.64 ms; a fourth slot, 4.11 ms, left LDS
#   for fewer than two waves per SIMD; with four waves per group a fourth slot gives 2.94 ms
#   against 2.77 ms for three).
EXT_IN_LDS = {"gg_ttgg": (("EXT_U", "EXT_V"), ("EXT_U", "EXT_V")),
              "gg_ttg": (("EXT_U", "EXT_V", "EXT_G:1"), ("EXT_U", "EXT_V"))}
# read those ahead of the step that uses them (else at each use), and pin the copies
PREFETCH_EXT = True
PIN_EXT = True
# processes with at most 16 helicity combinations whose kernel also sums the helicities: one
# workgroup holds every good helicity of an event block (64 lanes each), and its first wave adds
# their D |M_h|^2 from LDS after the colour sum, so one launch gives |M|^2.  Only the tiny
# e+e- processes, where a call is bound by launches: ee_mumu at 8192 events 29.7 -> 17.8 us per
# call; gg_tt at 2^19 was slower (2.36e9 -> 2.20e9 MEs/s FP64, 1.98e9 -> 1.68e9 mixed), its
# 16-wave workgroups waiting for each other at the barriers
HEL_SUM_IN_KERNEL = {"ee_mumu", "ee_mumu_z"}
# ... and whose |M|^2 comes from a kernel with one lane per event that evaluates the event's
# good helicities in turn (amp_lanes): no helicity waves to combine, no barrier after the
# momentum staging.  In the mixed forms the one-flow 16-bit tile has a scalar equivalent
# (colorsum.hpp, cs1_h16), so they use it too
LANE_PER_EVENT = {"ee_mumu", "ee_mumu_z", "gg_tt"}
# the batch size from which calls take that kernel (smaller batches fill the GPU only with a
# wave per helicity)
LANE_MIN_EVENTS = 1 << 16
# in that kernel, compute each external state for both helicities once per event, before the
# helicity loop, which then selects them (instead of computing them for every helicity): ee_mumu
# at 2^20 events FP64 82 -> 77 us per call, mixed FP16 89 -> 79 us
LANE_HOIST_EXT = True
# minimum waves per SIMD asked of that kernel (FP64, FP32): the eight hoisted FP64 states take 128
# registers.  Measured with the hoisted states: FP64 77 us at two waves, 79 at three; FP32 90 us at
# two, 79 at three
LANE_MIN_WAVES = (2, 3)
ALL_PROCESSES = ["ee_mumu", "gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg", "gg_gg", "ee_mumu_z"]
# electroweak constants of ee -> mumu with Z exchange: M_Z, Gamma_Z, M_W [GeV]
EW_MZ, EW_WZ, EW_MW = 91.188, 2.441404, 80.419


class Process:
    def __init__(self, name):
        self.name = name
        self.zboson = name == "ee_mumu_z"
        if name in ("ee_mumu", "ee_mumu_z"):
            self.kind, self.npar, self.ng = "ee", 4, 0
            self.gpar = []
            self.final_masses = ["0", "0"]
            self.avg, self.sym = 4, 1
            self.coupling = "alpha_em"
        elif name == "gg_gg":
            self.kind, self.npar, self.ng = "gluon", 4, 4
            self.gpar = [0, 1, 2, 3]
            self.final_masses = ["0", "0"]
            self.avg, self.sym = 256, 2
            self.coupling = "alpha_s"
        else:
            n = QCD_PROCESSES[name]
            self.kind, self.npar, self.ng = "qline", n + 2, n
            self.gpar = [0, 1] + list(range(4, n + 2))
            self.final_masses = ["m", "m"] + ["0"] * (n - 2)
            self.avg = 256
            self.sym = {2: 1, 3: 1, 4: 2, 5: 6}[n]
            self.coupling = "alpha_s"
        # processes too large for one kernel: the diagram program is cut into segments
        # (one kernel each) and the jamps go through a window of LDS slots, written out as
        # partial sums that a reduce kernel adds up
        self.segments = SEGMENTS.get(name)
        self._build()

    # -----------------------------------------------------------------------------------
    def _build(self):
        if self.kind == "ee":
            self.perms = [()]
            self.cnum, self.cden = [[1]], 1
            # the photon (and Z) diagram: internal line {e+, e-} | {mu+, mu-}
            nd = 2 if self.zboson else 1
            self.n_diagrams = self.n_amplitudes = nd
            self.fd_index, self.kweight, self.lines = list(range(nd)), [1.0] * nd, [(0b1100,)] * nd
            return
        if self.kind == "qline":
            self.diagrams = D.quark_line_diagrams(self.ng)
            self.perms, C = colour.colour_matrix_quark_line(self.ng)
            dkind = "qline"
        else:
            root_leaves = tuple(range(self.ng - 1))
            self.diagrams = [(t,) for t in D.trees(root_leaves)]
            self.perms, C = colour.colour_matrix_single_trace(self.ng)
            dkind = "gluon"
        self.dkind = dkind
        den = colour.common_denominator(C)
        self.cden = den
        self.cnum = [[int(x * den) for x in row] for row in C]
        self.n_diagrams = sum(1 for d in self.diagrams if D.is_canonical_structure(d))
        self.n_amplitudes = len(self.diagrams)
        self.jcoef = [D.diagram_colour(d, dkind) for d in self.diagrams]
        self.perm_index = {tuple(p): i for i, p in enumerate(self.perms)}
        if PRESUM:
            self.classes = D.proportional_classes(self.jcoef, self.perm_index)
        else:
            self.classes = [[(di, (1, 0))] for di in range(len(self.diagrams))]
        self.plan = D.Plan(self.diagrams, dkind)
        self._single_diagram_data(C)

    def _single_diagram_data(self, C):
        """per amplitude entry: its Feynman diagram (four-gluon colour structures of one
        diagram share it) and its colour weight K = c^dagger C c, the entry's colour-summed
        square per |amplitude|^2 (c: its coefficients on the colour flows); per Feynman
        diagram: its internal lines (bit i = particle i, the side without particle 0).
        Only the quark-line processes carry single-diagram weights."""
        self.fd_index, self.kweight, self.lines = None, None, None
        if self.dkind != "qline":
            return
        pidx = {tuple(p): i for i, p in enumerate(self.perms)}

        def strip(t):
            if t[0] == "L":
                return t
            if t[0] == "V3":
                return ("V3",) + tuple(strip(c) for c in t[1:])
            return ("V4",) + tuple(strip(c) for c in t[2:])

        keys, self.fd_index, self.kweight = {}, [], []
        full = (1 << self.npar) - 1

        def canon(m):
            return full ^ m if m & 1 else m

        def gmask(t):
            return sum(1 << self.gpar[i] for i in D.leaves(t))

        self.lines = []
        for d, coef in zip(self.diagrams, self.jcoef):
            k = tuple(strip(t) for t in d)
            if k not in keys:
                keys[k] = len(keys)
                lines = []

                def walk(t):
                    if t[0] == "L":
                        return
                    lines.append(canon(gmask(t)))
                    for c in D.children(t):
                        walk(c)

                for t in d:
                    walk(t)
                acc = 1 << 2           # quark propagators: the top plus the blocks before them
                for t in d[:-1]:
                    acc |= gmask(t)
                    lines.append(canon(acc))
                self.lines.append(tuple(sorted(lines)))
            self.fd_index.append(keys[k])
            v = [(pidx[tuple(q)], c) for q, c in coef.items()]
            K = 0
            for a, ca in v:
                for b, cb in v:
                    # Re(conj(ca) C_ab cb); C is real symmetric, so the sum is real
                    K += C[a][b] * (ca.re * cb.re + ca.im * cb.im)
            self.kweight.append(float(K))
        assert len(keys) == self.n_diagrams

    @property
    def nc(self):
        return len(self.perms)

    # -----------------------------------------------------------------------------------
    # code emission for the QCD processes

    def _q_expr(self, i):
        """incoming momentum of gluon i"""
        p = self.gpar[i]
        return f"p[{p}]" if p < 2 else f"(-p[{p}])"

    def _emit_qcd_body(self, out, remat_ext, order=None, steps=None, final=None, prefetch=None):
        """Emit the diagram program.  Momentum sums are written inline from fresh LDS reads
        (so no four-momentum stays live in registers across the program); with remat_ext the
        external wavefunctions are recomputed at every use instead of being kept live.
        With prefetch (default: on) the LDS reads of each amplitude step are issued as one
        group before the previous step's amplitude and jamp updates (software pipelining):
        a read issued after the jamps' LDS atomic adds could only complete after them, since
        LDS operations complete in order, so every step would start with a stall.
        Returns the algorithmic flop count (each distinct node once)."""
        if prefetch is None:
            prefetch = PREFETCH_MOMENTA
        body_start = len(out)
        marks = []   # per step: (first node line, amplitude line, first jamp-update line)
        puts = []    # per step: the JPUT lines of the slots it evicted
        names = {}
        flops = [0]
        ksums = set()

        def q(i):
            p = self.gpar[i]
            return f"PM({p})" if p < 2 else f"(-PM({p}))"

        def K(lv):
            lv = tuple(sorted(lv))
            if lv not in ksums:
                ksums.add(lv)
                flops[0] += FLOPS["p4add"] * (len(lv) - 1)
            return "(" + " + ".join(q(i) for i in lv) + ")"

        ext_count = [0]

        def ext_code(key):
            kind = key[0]
            if kind == "EXT_G":
                p = self.gpar[key[1]]
                outg = "true" if p >= 2 else "false"
                if remat_ext == "gluons_lds":
                    return f"ext_vec_b<R>(GB({key[1]}), lam[{p}], {outg})", FLOPS["ext_vec"]
                return f"ext_vec<R>(PM({p}), lam[{p}], {outg})", FLOPS["ext_vec"]
            if kind == "EXT_ROOT":
                p = self.gpar[self.ng - 1]
                return f"ext_vec<R>(PM({p}), lam[{p}], true)", FLOPS["ext_vec"]
            if kind == "EXT_U":
                return "ext_ubar<R>(PM(2), mt, lam[2])", FLOPS["ext_spinor"]
            return "ext_v<R>(PM(3), mt, lam[3])", FLOPS["ext_spinor"]

        counted = set()
        # external wavefunctions kept in LDS: slot of each, and the code that computes it
        lds64, lds32 = ((), ()) if self.segments else EXT_IN_LDS.get(self.name, ((), ()))
        ext_lds = set(lds64) | set(lds32)
        xslot = {}
        self.xw_init = []    # (code, in LDS in the FP64 kernel, in LDS in the FP32 kernel)

        def in_set(key, kinds):
            return key[0] in kinds or (len(key) > 1 and f"{key[0]}:{key[1]}" in kinds)

        def remat(kind):
            if remat_ext is True:
                return True
            if remat_ext == "gluons":
                return kind in ("EXT_G", "EXT_ROOT")
            if remat_ext == "gluons_lds":
                return kind == "EXT_G"
            if remat_ext == "spinors":
                return kind in ("EXT_U", "EXT_V")
            return False

        def emit(key):
            kind = key[0]
            if in_set(key, ext_lds):
                if key not in xslot:
                    code, fl = ext_code(key)
                    xslot[key] = len(self.xw_init)
                    self.xw_init.append((code, in_set(key, lds64), in_set(key, lds32)))
                    flops[0] += fl
                return f"XW({xslot[key]})"
            if kind.startswith("EXT") and remat(kind):
                code, fl = ext_code(key)
                if key not in counted:
                    counted.add(key)
                    flops[0] += fl
                ext_count[0] += 1
                nm = f"x{ext_count[0]}"
                out.append(f"    const W4<R> {nm} = {code};")
                return nm
            if key in names:
                return names[key]
            if kind.startswith("EXT"):
                code, fl = ext_code(key)
                nm = f"w{len(names)}"
                out.append(f"    const W4<R> {nm} = {code};")
                flops[0] += fl
                names[key] = nm
                return nm
            deps = [emit(dk) for dk in D.node_deps(key)]
            nm = f"w{len(names)}"
            code, fl = node_code(key, deps)
            out.append(f"    const W4<R> {nm} = {code};")
            flops[0] += fl
            names[key] = nm
            return nm

        def node_code(key, deps, count=True):
            """the call that computes node `key` from its operands `deps` (names or expressions),
            and its flops; count: the momentum sums it introduces enter the algorithmic count"""
            kind = key[0]
            Kc = K if count else (lambda lv: "(" + " + ".join(q(i) for i in sorted(lv)) + ")")
            if kind == "G":
                t = key[1]
                kids = D.children(t)
                if t[0] == "V3":
                    ka, kb = Kc(D.leaves(kids[0])), Kc(D.leaves(kids[1]))
                    return f"vvv_cur<R>({deps[0]}, {ka}, {deps[1]}, {kb}, gs)", FLOPS["vvv_cur"]
                return (f"vvvv_cur<R, {t[1]}>({deps[0]}, {deps[1]}, {deps[2]}, {Kc(D.leaves(t))}, gs)",
                        FLOPS["vvvv_cur"])
            if kind in ("U", "V"):
                Km = Kc([g for b in key[1] for g in D.leaves(b)])
                if kind == "U":
                    return f"fstr_u<R>({deps[0]}, {deps[1]}, PM(2) - {Km}, mt, gs)", FLOPS["fstr"] + FLOPS["p4add"]
                return f"fstr_v<R>({deps[0]}, {deps[1]}, {Km} - PM(3), mt, gs)", FLOPS["fstr"] + FLOPS["p4add"]
            if kind == "JF":
                used = set(g for b in key[1] + key[2] for g in D.leaves(b))
                gap = sorted(set(range(self.ng)) - used)
                return f"jf<R>({deps[0]}, {deps[1]}, {Kc(gap)}, gs)", FLOPS["jf"]
            raise ValueError(key)

        def emit_local(key, local, lines):
            """a node for the channel-weight instance only: taken from the program if it is there,
            else computed into `lines` (a block of that instance) under a name of the block"""
            if key[0].startswith("EXT") or key in names:
                return emit(key)
            if key in local:
                return local[key]
            deps = [emit_local(dk, local, lines) for dk in D.node_deps(key)]
            nm = f"z{len(local)}"
            lines.append(f"const W4<R> {nm} = {node_code(key, deps, count=False)[0]};")
            local[key] = nm
            return nm

        def vertex_of(key):
            """(vertex, operand nodes, momenta) of a computed node through which a sum of such
            nodes can pass (the vertex is linear in each operand), or None"""
            kind = key[0]
            if kind == "G":
                t = key[1]
                kids = D.children(t)
                ops = [D.wf_key(c) for c in kids]
                if t[0] == "V3":
                    return ("V3",), ops, (tuple(sorted(D.leaves(kids[0]))), tuple(sorted(D.leaves(kids[1]))))
                return ("V4", t[1]), ops, (tuple(sorted(D.leaves(t))),)
            if kind in ("U", "V"):
                return (kind,), list(D.node_deps(key)), (tuple(sorted(g for b in key[1] for g in D.leaves(b))),)
            return None

        def opsum(terms):
            """the node sum_i u_i X_i (terms: (node, unit), the first unit 1), formed once per body:
            nodes made by the same vertex from the same operands but one, at the same momenta,
            are summed in that operand first (recursively), so that the vertex runs once"""
            tkey = tuple(terms)
            if tkey in sums:
                return sums[tkey]
            parts = []   # [term indices, slot]
            for i, (k, _) in enumerate(terms):
                v = vertex_of(k)
                for g in parts:
                    v0 = vertex_of(terms[g[0][0]][0])
                    if v is None or v0 is None or v0[0] != v[0] or v0[2] != v[2] or len(v0[1]) != len(v[1]):
                        continue
                    diff = [j for j in range(len(v[1])) if v[1][j] != v0[1][j]]
                    if len(diff) == 1 and g[1] in (None, diff[0]):
                        g[0].append(i)
                        g[1] = diff[0]
                        break
                else:
                    parts.append([[i], None])
            exprs = []
            for idx, slot in parts:
                k0, u0 = terms[idx[0]]
                if len(idx) == 1:
                    exprs.append((emit(k0), u0))
                    continue
                ops0 = vertex_of(k0)[1]
                inner = opsum([(vertex_of(terms[i][0])[1][slot], unit_div(terms[i][1], u0)) for i in idx])
                deps = [inner if j == slot else emit(o) for j, o in enumerate(ops0)]
                code, fl = node_code(k0, deps)
                flops[0] += fl
                exprs.append((code, u0))
            assert exprs[0][1] == (1, 0)
            comb = exprs[0][0]
            for e, u in exprs[1:]:
                comb = f"w4_acc<R, {u[0]}, {u[1]}>({comb}, {e})"
                flops[0] += 8
            nm = f"s{len(sums)}"
            out.append(f"    const W4<R> {nm} = {comb};")
            sums[tkey] = nm
            return nm

        def unit_div(u, v):
            """u / v for units of the Gaussian integers"""
            return (u[0] * v[0] + u[1] * v[1], u[1] * v[0] - u[0] * v[1])

        if order is None:
            order = D.schedule(self.plan, remat_ext=remat_ext, amps=self.units())
        # the amplitude entries in the order their `a = amp_...` lines are emitted
        self.emit_order = [m[0] for unit in order for m in self.unit_members(unit)]
        # per `a = amp_...` line: [(entry, unit factor relative to the line's first entry)]
        self.emit_groups = []

        def call_text(member, ops):
            """the vertex call of one amplitude entry on operands `ops` (names or expressions, in
            the order of its dependencies) as (function, arguments)"""
            di, (kind, j), _, _ = member
            if kind == "FFV":
                return "amp_ffv<R>", list(ops) + ["gs"]
            t = self.diagrams[di][j]
            kids = D.children(t)
            if t[0] == "V3":
                kx = K((self.ng - 1,)) if self.kind == "gluon" else "(-" + K(D.leaves(t)) + ")"
                ka, kb = K(D.leaves(kids[0])), K(D.leaves(kids[1]))
                return "amp_vvv<R>", [ops[0], kx, ops[1], ka, ops[2], kb, "gs"]
            return f"amp_vvvv<R, {t[1]}>", [ops[0], ops[1], ops[2], ops[3], "gs"]

        def call_of(member):
            """emit the nodes of one amplitude entry; its vertex call as (function, arguments)"""
            return call_text(member, [emit(k) for k in member[2]])

        def amp_flops(fn):
            return FLOPS["amp_ffv" if fn.startswith("amp_ffv") else "amp_vvv" if fn.startswith("amp_vvv<")
                         else "amp_vvvv"]

        sums = {}
        deep = LINEAR_MERGE and self.name in DEEP_MERGE
        comb_refs = collections.Counter()
        if LINEAR_MERGE:
            for unit in order:
                members = self.unit_members(unit)
                for grp in self._linear_groups(members):
                    if len(grp) > 1:
                        comb_refs[self._group_terms(members, grp)] += 1
        for ai, unit in enumerate(order):
            members = self.unit_members(unit)
            groups = self._linear_groups(members) if LINEAR_MERGE else [[i] for i in range(len(members))]
            for gi, grp in enumerate(groups):
                last = gi == len(groups) - 1
                m_node = len(out)
                uf = members[grp[0]][3]
                line = [(members[grp[0]][0], (1, 0))]
                sde_block = None
                if len(grp) > 1 and deep:
                    # the operand sum through the vertices that made its terms (opsum); each
                    # diagram's own amplitude, for the channel weights only, in a block of that instance
                    terms = self._group_terms(members, grp)
                    d0 = members[grp[0]][2]
                    slot = next(j for i in grp[1:] for j in range(len(d0)) if members[i][2][j] != d0[j])
                    sub = opsum(list(terms))
                    fn, args = call_text(members[grp[0]], [sub if j == slot else emit(dk) for j, dk in enumerate(d0)])
                    line += [(members[i][0], rel) for i, (_, rel) in zip(grp[1:], terms[1:])]
                    if self.fd_index is not None:
                        local, blk = {}, []
                        for i in grp:
                            f, a_ = call_text(members[i], [emit_local(dk, local, blk) for dk in members[i][2]])
                            blk.append(f"{{ const cx<R> a = {f}({', '.join(a_)}); SDEACC({self.fd_index[members[i][0]]}, "
                                       f"{self.kweight[members[i][0]]!r}); }}")
                        sde_block = blk
                    calls = None
                else:
                    calls = [call_of(members[i]) for i in grp]
                    fn, args = calls[0]
                if len(grp) > 1 and not deep:
                    # one vertex on the sum of the operands that differ, each times its unit
                    # relative to the first member's: sum_m u_m V(.., w_m, ..) = u_f V(.., sum_m (u_m/u_f) w_m, ..)
                    diff = {k for f, a in calls[1:] for k in range(len(args)) if a[k] != args[k]}
                    assert len(diff) == 1 and all(f == fn for f, _ in calls), (unit[0], grp)
                    k = diff.pop()
                    comb = args[k]
                    terms = [(args[k], (1, 0))]
                    for i, (_, a) in zip(grp[1:], calls[1:]):
                        ur, ui = members[i][3]
                        rel = (ur * uf[0] + ui * uf[1], ui * uf[0] - ur * uf[1])
                        comb = f"w4_acc<R, {rel[0]}, {rel[1]}>({comb}, {a[k]})"
                        terms.append((a[k], rel))
                        line.append((members[i][0], rel))
                    # a sum that several groups use is formed once, as a node of its own
                    tkey = self._group_terms(members, grp)
                    if SUM_NODES and comb_refs[tkey] > 1:
                        if tkey not in sums:
                            sums[tkey] = f"s{len(sums)}"
                            out.append(f"    const W4<R> {sums[tkey]} = {comb};")
                            flops[0] += 8 * (len(grp) - 1)
                        comb = sums[tkey]
                    else:
                        flops[0] += 8 * (len(grp) - 1)
                    args = args[:k] + [comb] + args[k + 1:]
                m_amp = len(out)
                self.emit_groups.append(line)
                out.append(f"    a = {fn}({', '.join(args)});")
                flops[0] += amp_flops(fn)
                out.append("    pin_cx<R>(a);")
                if self.fd_index is not None:
                    if len(grp) == 1:
                        di = members[grp[0]][0]
                        out.append(f"    SDEACC({self.fd_index[di]}, {self.kweight[di]!r});")
                    elif sde_block is not None:
                        out.append(f"    if constexpr (SDE) {{ {' '.join(sde_block)} }}")
                    else:
                        # the channel weights need each diagram's own amplitude
                        sde = " ".join(f"{{ const cx<R> a = {f}({', '.join(a)}); SDEACC({self.fd_index[members[i][0]]}, "
                                       f"{self.kweight[members[i][0]]!r}); }}" for i, (f, a) in zip(grp, calls))
                        out.append(f"    if constexpr (SDE) {{ {sde} }}")
                # the groups of a class with proportional colour coefficients are summed first:
                # sa = a_1, then sa += u a; its jamp updates use sa
                if len(groups) > 1:
                    if gi == 0:
                        assert uf == (1, 0)
                        out.append("    sa = a;")
                    else:
                        out.append("    " + ACC_TEXT[uf])
                        flops[0] += FLOPS["jamp"]
                marks.append((m_node, m_amp, len(out)))
                if not last:
                    if prefetch and steps is not None:
                        puts.append([])
                    continue
                var = "sa" if len(groups) > 1 else "a"
                di0 = members[0][0]
                if steps is None:
                    for seq, c in sorted(self.jcoef[di0].items()):
                        out.append(self._jamp_update(self.perm_index[seq], c, var))
                        flops[0] += FLOPS["jamp"]
                else:
                    coef = {self.perm_index[seq]: c for seq, c in self.jcoef[di0].items()}
                    mine = []
                    for j, slot, flush in steps[ai]:
                        if flush is not None:
                            k = flush[1]
                            out.append(f"    JTAKE({flush[0]}, {k});")
                            mine.append(f"    JPUT({k}, {k});")
                        out.append(self._jamp_update(slot, coef[j], var))
                        flops[0] += FLOPS["jamp"]
                    if prefetch:
                        puts.append(mine)
                    else:
                        out += mine
        tail = []
        if puts:
            tail += puts[-1]
        if final:
            tail += [f"    JLAST({slot}, {pidx});" for slot, pidx, _ in final]
            tail += [f"    JPUT({pidx}, {pidx});" for slot, pidx, _ in final]
        if prefetch and marks:
            out[body_start:] = _pipeline_momenta(out[body_start:], [tuple(m - body_start for m in t)
                                                                    for t in marks], puts)
        out += tail
        return flops[0]

    @staticmethod
    def _jamp_update(s, c, v="a"):
        """J[s] += c * v (v: the amplitude a, or a class sum s) through the JADD(slot, re/im,
        value) macro"""
        cr, ci = c.re, c.im
        if (cr, ci) == (1, 0):
            return f"    JADD({s}, 0, {v}.r); JADD({s}, 1, {v}.i);"
        if (cr, ci) == (-1, 0):
            return f"    JADD({s}, 0, -{v}.r); JADD({s}, 1, -{v}.i);"
        if (cr, ci) == (0, 1):
            return f"    JADD({s}, 0, -{v}.i); JADD({s}, 1, {v}.r);"
        if (cr, ci) == (0, -1):
            return f"    JADD({s}, 0, {v}.i); JADD({s}, 1, -{v}.r);"
        return (f"    JADD({s}, 0, (R)({cr}) * {v}.r - (R)({ci}) * {v}.i); "
                f"JADD({s}, 1, (R)({cr}) * {v}.i + (R)({ci}) * {v}.r);")

    # -----------------------------------------------------------------------------------
    # units of the diagram program: classes of amplitude entries with proportional colour
    # coefficients (singletons when PRESUM is off)

    def units(self):
        """[(first entry, ("CLASS", members), deps of all members)], members = ((entry, option,
        deps, unit factor), ..); the order of self.classes"""
        if getattr(self, "_units", None) is None:
            amps = {a[0]: a for a in self.plan.amplitudes()}
            out = []
            for cls in self.classes:
                mem = tuple((di, amps[di][1], amps[di][2], u) for di, u in cls)
                deps = tuple(dict.fromkeys(k for m in mem for k in m[2]))
                out.append((cls[0][0], ("CLASS", mem), deps))
            self._units = out
        return self._units

    def _linear_groups(self, members):
        """Partition a unit's members into groups evaluated as one vertex each: members with the
        same vertex (FFV, three-gluon, or four-gluon of the same colour structure) whose operands
        are the same nodes in all slots but one, and whose nodes in that slot carry the same
        momentum (the same external legs).  Greedy in member order; the first group starts with
        the first member.  Returns lists of member indices."""
        def sig(m):
            di, (kind, j), deps, _ = m
            if kind == "FFV":
                return ("FFV",), tuple(deps), None
            t = self.diagrams[di][j]
            legs = (None,) + tuple(tuple(sorted(D.leaves(k))) for k in D.children(t))
            return ((t[0],) if t[0] == "V3" else (t[0], t[1])), tuple(deps), legs

        sigs = [sig(m) for m in members]
        groups = []   # [member indices, slot or None]
        for i, (head, deps, legs) in enumerate(sigs):
            for g in groups:
                h0, d0, l0 = sigs[g[0][0]]
                if h0 != head or len(d0) != len(deps) or l0 != legs:
                    continue
                diff = [k for k in range(len(deps)) if deps[k] != d0[k]]
                if len(diff) == 1 and g[1] in (None, diff[0]):
                    g[0].append(i)
                    g[1] = diff[0]
                    break
            else:
                groups.append([[i], None])
        return [g[0] for g in groups]

    @staticmethod
    def _group_terms(members, grp):
        """the operand sum of a group (of at least two members): ((node in the slot where the
        members differ, unit relative to the first member's), ..)"""
        d0, uf = members[grp[0]][2], members[grp[0]][3]
        slot = next(j for i in grp[1:] for j in range(len(d0)) if members[i][2][j] != d0[j])
        return tuple((members[i][2][slot], (members[i][3][0] * uf[0] + members[i][3][1] * uf[1],
                                            members[i][3][1] * uf[0] - members[i][3][0] * uf[1])) for i in grp)

    @staticmethod
    def unit_members(unit):
        """the (entry, option, deps, unit factor) of each amplitude a unit stands for"""
        di, opt, deps = unit
        if opt[0] == "CLASS":
            return opt[1]
        return ((di, opt, deps, (1, 0)),)

    def _emit_ee_body(self, out):
        # (e+, e-, mu+, mu-): vbar(p0) (i e gamma) u(p1) -> photon -> ubar(p3) (i e gamma) v(p2)
        out.append("    const W4<R> w0 = ext_vbar<R>(PM(0), 0.0, lam[0]);")
        out.append("    const W4<R> w1 = ext_u<R>(PM(1), 0.0, lam[1]);")
        out.append("    const W4<R> w2 = ext_v<R>(PM(2), 0.0, lam[2]);")
        out.append("    const W4<R> w3 = ext_ubar<R>(PM(3), 0.0, lam[3]);")
        out.append("    const W4<R> w4 = jf<R>(w0, w1, PM(0) + PM(1), gs);")
        out.append("    a = amp_ffv<R>(w3, w2, w4, gs);")
        out.append("    SDEACC(0, 1.0);")
        out.append("    JADD(0, 0, a.r); JADD(0, 1, a.i);")
        fl = 4 * FLOPS["ext_spinor"] + FLOPS["p4add"] + FLOPS["jf"] + FLOPS["amp_ffv"] + FLOPS["jamp"]
        if self.zboson:
            # Z exchange: i (g / cos theta_W) gamma^mu (T3 P_L - Q sin^2 theta_W), Q = -1, T3 = -1/2,
            # g = e / sin theta_W; sin^2 theta_W = 1 - M_W^2 / M_Z^2
            sw2 = 1.0 - EW_MW ** 2 / EW_MZ ** 2
            gz = 1.0 / (sw2 * (1.0 - sw2)) ** 0.5
            cl, cr = -0.5 + sw2, sw2
            out.append(f"    const W4<R> w5 = jf_chiral<R>(w0, w1, PM(0) + PM(1), gs * {gz!r}, {cl!r}, {cr!r}, "
                       f"{EW_MZ!r}, {EW_WZ!r});")
            out.append(f"    a = amp_ffv_chiral<R>(w3, w2, w5, gs * {gz!r}, {cl!r}, {cr!r});")
            out.append("    SDEACC(1, 1.0);")
            out.append("    JADD(0, 0, a.r); JADD(0, 1, a.i);")
            fl += FLOPS["jf_chiral"] + FLOPS["amp_ffv_chiral"] + FLOPS["jamp"]
        return fl

    # -----------------------------------------------------------------------------------
    def source(self, jamps_in_lds=None, remat_ext=None, jamp_mode="auto"):
        """jamps_in_lds: accumulate the jamps in LDS (else registers); jamp_mode for LDS:
        'atomic' (LDS atomic add in the working precision), 'rmw' (plain LDS read-add-write),
        'atomic64' (LDS atomic add into an FP64 accumulator), 'auto' (atomic add for the FP64
        kernel, read-add-write for the FP32 kernel: measured fastest on gfx950, where the
        FP32 LDS atomic add is far slower than the FP64 one).  remat_ext: recompute external
        wavefunctions at each use: True, False, 'gluons' or 'spinors'."""
        self.perm_index = {tuple(p): i for i, p in enumerate(self.perms)}
        if jamps_in_lds is None:
            jamps_in_lds = self.nc > 6
        if remat_ext is None:
            remat_ext = "gluons_lds" if self.name in GLUONS_FROM_LDS else False
        self.remat_ext = remat_ext
        nc = self.nc
        nm = self.name
        kernels = []      # (kernel name, body lines, jamp slots in LDS, output mode)
        self.nslot = 0
        if self.kind == "ee":
            body = []
            fl = self._emit_ee_body(body)
            kernels.append(("amp_kernel", body, nc, "jamps"))
            self.flops_exec = fl
        elif not self.segments:
            body = []
            fl = self._emit_qcd_body(body, remat_ext)
            kernels.append(("amp_kernel", body, nc, "jamps"))
            self.flops_exec = fl
        else:
            n_seg, window, beta = self.segments
            jsets = [set(self.perm_index[q] for q in self.jcoef[i]) for i in range(len(self.diagrams))]
            # algorithmic count: every node once, in any order
            fl = self._emit_qcd_body([], remat_ext, order=self.units())
            cut = SEGMENT_CUT
            if cut == "vertices":
                cut = lambda u: len(self._linear_groups(self.unit_members(u))) if LINEAR_MERGE else len(self.unit_members(u))
            segs = D.segment_plan(self.plan, jsets, n_seg, beta, window, amps=self.units(), cut=cut,
                                  remat_ext=remat_ext)
            self.segment_orders = segs
            self.segment_emit_groups = []
            self.flops_exec = 0
            partial_jamp = []
            for k, order in enumerate(segs):
                steps, final, pj = D.window_program(order, jsets, window)
                base = len(partial_jamp)
                steps = [[(j, sl, None if f is None else (f[0], f[1] + base, f[2])) for j, sl, f in st]
                         for st in steps]
                final = [(sl, pi + base, j) for sl, pi, j in final]
                partial_jamp += pj
                body = []
                self.flops_exec += self._emit_qcd_body(body, remat_ext, order=order, steps=steps, final=final)
                self.segment_emit_groups.append(self.emit_groups)
                kernels.append((f"amp_seg{k}", body, window, "slots"))
            self.nslot = len(partial_jamp)
            self.partial_jamp = partial_jamp
        self.flops_lane = fl
        cn = ", ".join(str(x) for row in self.cnum for x in row)
        masses = ", ".join("1" if m == "m" else "0" for m in self.final_masses)
        perm_flat = ", ".join(str(x) for p in self.perms for x in p) or "0"
        n_order = len(self.perms[0]) if self.perms else 0
        L = []
        L.append(f"// Generated by paper_2210_11122_amd.gen for the process {nm}; do not edit.")
        L.append(f"// {self.n_diagrams} Feynman diagrams ({self.n_amplitudes} vertex contractions), "
                 f"{nc} colour flows, {1 << self.npar} helicity combinations.")
        if self.segments:
            L.append(f"// {len(kernels)} segment kernels, {self.segments[1]}-slot LDS jamp window, "
                     f"{self.nslot} partial jamp slots; executed flops per lane {self.flops_exec} "
                     f"(algorithmic {fl}).")
        # a kernel that ends with all jamps of its lane (no window, no partial slots) can finish
        # with the colour sum itself
        fused = not self.segments
        self.fused_colour = fused
        L.append('#include "../helas.hpp"')
        L.append('#include "../process.hpp"')
        if fused:
            L.append('#include "../colorsum.hpp"')
            L.append('#include "me.h"')
        L.append("namespace me {")
        L.append(f"namespace proc_{nm} {{")
        L.append(f"constexpr int NPAR = {self.npar};")
        L.append(f"constexpr int NC = {nc};")
        L.append(f"constexpr int NSLOT = {self.nslot};")
        self.extra_files = {}
        if self.segments:
            # one source file per segment kernel (compiled in parallel); the main file calls
            # their host-side launchers
            for kname, body, nwin, mode in kernels:
                F = [f"// Generated by paper_2210_11122_amd.gen: {nm}, {kname}; do not edit.",
                     '#include "../helas.hpp"', "namespace me {", f"namespace proc_{nm} {{",
                     f"constexpr int NPAR = {self.npar};", f"constexpr int NC = {nc};",
                     f"constexpr int NSLOT = {self.nslot};"]
                F += self._kernel_text(kname, body, nwin, mode, jamps_in_lds, jamp_mode, first=(kname == "amp_seg0"))
                g64, g32 = WAVES_PER_GROUP.get(self.name, (1, 1))
                for R, tag, wg in (("double", "f64", g64), ("float", "f32", g32)):
                    F.append(f"hipError_t {kname}_launch_{tag}(const double* mom, int64_t n_evt, int64_t ld, "
                             f"const signed char* hel, int n_good, double mt, double gs, {R}* jamp, const int* chan, "
                             "double* sde, hipStream_t st, int64_t blocks)")
                    F.append("{")
                    F.append("    if (chan)")
                    F.append(f"        hipLaunchKernelGGL(({kname}<{R}, true>), dim3((unsigned)blocks), dim3({64 * wg}), 0, st, mom, "
                             "n_evt, ld, hel, n_good, mt, gs, jamp, chan, sde);")
                    F.append("    else")
                    F.append(f"        hipLaunchKernelGGL(({kname}<{R}, false>), dim3((unsigned)blocks), dim3({64 * wg}), 0, st, mom, "
                             "n_evt, ld, hel, n_good, mt, gs, jamp, nullptr, nullptr);")
                    F.append("    return hipGetLastError();")
                    F.append("}")
                F += ["}  // namespace", "}  // namespace me"]
                self.extra_files[f"proc_{nm}_{kname}.hip"] = "\n".join(F) + "\n"
                for R, tag in (("double", "f64"), ("float", "f32")):
                    L.append(f"hipError_t {kname}_launch_{tag}(const double*, int64_t, int64_t, const signed char*, "
                             f"int, double, double, {R}*, const int*, double*, hipStream_t, int64_t);")
        else:
            for kname, body, nwin, mode in kernels:
                L += self._kernel_text(kname, body, nwin, mode, jamps_in_lds, jamp_mode, fused=fused)
            if fused and nm in LANE_PER_EVENT:
                L += self._lane_kernel_text(kernels[0][1])
        L.append("")
        L.append(f"static const int colour_num[NC * NC] = {{{cn}}};")
        L.append(f"static const int final_massive[NPAR - 2] = {{{masses}}};")
        L.append(f"static const int orderings[] = {{{perm_flat}}};")
        nlines = max(1, self.npar - 3)
        if self.lines is not None:
            flat = ", ".join(str(x) for ln in self.lines for x in (list(ln) + [0] * (nlines - len(ln))))
        else:
            flat = "0"
        L.append(f"static const int diagram_lines[] = {{{flat}}};")
        if self.segments:
            L += self._reduce_text()
        L.append("template <class R>")
        L.append("static hipError_t launch(const double* mom, int64_t n_evt, int64_t ld, const signed char* hel, "
                 "int n_good, double mt, double gs, R* jamp, const int* chan, double* sde, const FusedColour* fc, "
                 "hipStream_t st)")
        L.append("{")
        if not fused:
            L.append("    if (fc) return hipErrorInvalidValue;  // no fused colour sum for this process")
        else:
            L.append("    if (fc && (chan || !fc->aop || (sizeof(R) == 8) != (fc->form == ME_FP64))) "
                     "return hipErrorInvalidValue;")
            L.append("    const FusedColour none{nullptr, nullptr, 0, 0, nullptr, 0.0, 1};")
        g64, g32 = WAVES_PER_GROUP.get(self.name, (1, 1))
        L.append(f"    constexpr int WG = sizeof(R) == 8 ? {g64} : {g32};  // waves (helicities) per workgroup")
        L.append("    int64_t blocks = ((n_evt + 63) / 64) * ((n_good + WG - 1) / WG);")
        L.append("    if (blocks == 0) return hipSuccess;")
        for kname, _, _, _ in kernels:
            if self.segments:
                L.append("    {")
                L.append(f"        hipError_t e = sizeof(R) == 8 ? {kname}_launch_f64(mom, n_evt, ld, hel, n_good, mt, gs, "
                         "(double*)jamp, chan, sde, st, blocks)")
                L.append(f"                                      : {kname}_launch_f32(mom, n_evt, ld, hel, n_good, mt, gs, "
                         "(float*)jamp, chan, sde, st, blocks);")
                L.append("        if (e != hipSuccess) return e;")
                L.append("    }")
            else:
                if fused and (self.name in HEL_SUM_IN_KERNEL or nm in LANE_PER_EVENT):
                    L.append("    if (fc && fc->hsum_out) {  // the kernel also sums the helicities")
                    if nm in LANE_PER_EVENT:
                        L.append("        // batches large enough to fill the GPU with one lane per event (the mixed forms when")
                        L.append("        // their one colour operand is exact in the 16-bit type, as the scalar form assumes)")
                        L.append(f"        if (n_evt >= {LANE_MIN_EVENTS} && (sizeof(R) == 8 || (NC == 1 && !(fc->lo_mask & 1)))) {{")
                        L.append("            hipLaunchKernelGGL((amp_lanes<R>), dim3((unsigned)((n_evt + 63) / 64)), dim3(64), 0, st, "
                                 "mom, n_evt, hel, n_good, mt, gs, *fc);")
                        L.append("            return hipGetLastError();")
                        L.append("        }")
                    if self.name in HEL_SUM_IN_KERNEL:
                        L.append("        if (n_good > 16) return hipErrorInvalidValue;")
                        L.append(f"        hipLaunchKernelGGL(({kname}<R, false, true>), dim3((unsigned)((n_evt + 63) / 64)), dim3(64 * n_good), 0, st, "
                                 "mom, n_evt, ld, hel, n_good, mt, gs, jamp, nullptr, nullptr, *fc);")
                        L.append("        return hipGetLastError();")
                    else:
                        L.append("        return hipErrorInvalidValue;  // below the lane kernel's batch size: no such kernel")
                    L.append("    }")
                L.append("    if (chan)")
                tail = ", none" if fused else ""
                L.append(f"        hipLaunchKernelGGL(({kname}<R, true>), dim3((unsigned)blocks), dim3(64 * WG), 0, st, mom, n_evt, "
                         f"ld, hel, n_good, mt, gs, jamp, chan, sde{tail});")
                L.append("    else")
                tail = ", fc ? *fc : none" if fused else ""
                L.append(f"        hipLaunchKernelGGL(({kname}<R, false>), dim3((unsigned)blocks), dim3(64 * WG), 0, st, mom, n_evt, "
                         f"ld, hel, n_good, mt, gs, jamp, nullptr, nullptr{tail});")
        if self.segments:
            L.append("    hipLaunchKernelGGL(reduce_kernel<R>, dim3((unsigned)((n_evt + 255) / 256), (unsigned)n_good), "
                     "dim3(256), 0, st, jamp, ld, n_good, n_evt);")
        L.append("    return hipGetLastError();")
        L.append("}")
        L.append("}  // namespace")
        L.append(f"const ProcessDesc* process_{nm}()")
        L.append("{")
        L.append("    static const ProcessDesc d = {")
        L.append(f'        "{nm}", proc_{nm}::NPAR, proc_{nm}::NC, {1 << self.npar}, '
                 f"{self.avg}, {self.sym}, {1 if self.coupling == 'alpha_s' else 0},")
        L.append(f"        proc_{nm}::colour_num, {self.cden}, proc_{nm}::final_massive, proc_{nm}::orderings, "
                 f"{n_order},")
        L.append(f"        {self.n_diagrams}, {self.n_amplitudes}, {fl}.0, {self.flops_exec}.0, proc_{nm}::NSLOT,")
        L.append(f"        proc_{nm}::diagram_lines, {nlines}, {0 if self.lines is None else 1}, {1 if fused else 0}, "
                 f"{1 if fused and nm in HEL_SUM_IN_KERNEL else 0}, {LANE_MIN_EVENTS if fused and nm in LANE_PER_EVENT else 0},")
        L.append(f"        proc_{nm}::launch<double>, proc_{nm}::launch<float>,")
        L.append("    };")
        L.append("    return &d;")
        L.append("}")
        L.append("}  // namespace me")
        return "\n".join(L) + "\n"

    def _kernel_text(self, kname, body, nwin, mode, jamps_in_lds, jamp_mode, first=True, fused=False):
        """one amplitude kernel: momenta staging, helicity signs, jamp storage, body, output.
        mode 'jamps': the NC jamps are written at the end, layout [h][2c + re/im][column];
        mode 'slots': the body evicts window slots to partial slots (JTAKE, later JPUT), layout
        [h][2s + re/im][column] after the jamp region.
        With SDE the kernel also sums, per lane, the colour-summed single-diagram squares
        K_e |a_e|^2 of its amplitude entries (all, and those of the event's channel chan[e])
        into sde[h][0/1][column]; `first` is false for segment kernels that add to the
        sums of the segments before them."""
        L = []
        hsum = fused and self.name in HEL_SUM_IN_KERNEL
        # HS: the instance that also sums the helicities (its workgroup holds an event block's
        # good helicities; the LDS it needs for that is only in this instance)
        L.append("template <class R, bool SDE, bool HS = false>" if hsum else "template <class R, bool SDE>")
        w64, w32 = MIN_WAVES.get(self.name, (1, 1))
        g64, g32 = WAVES_PER_GROUP.get(self.name, (1, 1))
        if hsum and (g64, g32) != (1, 1):
            raise ValueError("the helicity sum in the kernel sizes the workgroup by the good helicities")
        threads = "64" if (g64, g32) == (1, 1) else f"64 * (sizeof(R) == 8 ? {g64} : {g32})"
        if hsum:
            threads = "1024"   # up to 16 helicity waves of one event block
        bounds = threads if (w64, w32) == (1, 1) else f"{threads}, (sizeof(R) == 8 ? {w64} : {w32})"
        L.append(f"__global__ __launch_bounds__({bounds}) void {kname}(const double* __restrict__ mom, int64_t n_evt, "
                 "int64_t ld, const signed char* __restrict__ hel, int n_good, double mt, double gs, "
                 "R* __restrict__ jamp, const int* __restrict__ chan, double* __restrict__ sde"
                 + (", FusedColour fc)" if fused else ")"))
        L.append("{")
        L.append(f"    constexpr int WG = sizeof(R) == 8 ? {g64} : {g32};  // waves per workgroup")
        L.append("    __shared__ double lds[4 * NPAR * 64];")
        L.append("    const int lane = threadIdx.x & 63;")
        L.append("    const int64_t w = xcd_remap(blockIdx.x, gridDim.x);")
        if hsum:
            L.append("    // with the helicity sum here, one workgroup holds all good helicities of its block")
            L.append("    constexpr bool hsum = HS && !SDE;")
            L.append("    const int wg = hsum ? n_good : WG;")
            L.append("    const int hpb = (n_good + wg - 1) / wg;  // workgroups per event block")
        else:
            L.append("    const int hpb = (n_good + WG - 1) / WG;  // workgroups per event block")
        L.append("    const int64_t e0 = (w / hpb) * 64;")
        L.append(f"    const int hr = (int)(w % hpb) * {'wg' if hsum else 'WG'} + (int)(threadIdx.x >> 6);")
        L.append("    const bool live = hr < n_good;  // a spare wave of the last group repeats a helicity, writes nothing")
        L.append("    const int h = live ? hr : n_good - 1;")
        L.append("    const int64_t e = e0 + lane;  // < ld: ld is a multiple of 64 covering the grid")
        if hsum:
            L.append("    if constexpr (hsum)")
            L.append("        stage_momenta_n<NPAR>(mom, n_evt, e0, lds, threadIdx.x, 64 * wg);")
            L.append("    else")
            L.append("        stage_momenta<NPAR, WG>(mom, n_evt, e0, lds, threadIdx.x);")
        else:
            L.append("    stage_momenta<NPAR, WG>(mom, n_evt, e0, lds, threadIdx.x);")
        L.append("#define PM(i) lds_p4(lds, i, lane)")
        if getattr(self, "remat_ext", False) == "gluons_lds":
            gp = ", ".join(str(p) for p in self.gpar)
            L.append(f"    // the gluons' polarisation bases, for every helicity wave of the block")
            L.append(f"    constexpr int GPART[{len(self.gpar)}] = {{{gp}}};")
            L.append(f"    __shared__ R gbl[6 * {len(self.gpar)} * 64];")
            L.append(f"    stage_gluon_basis<R, {len(self.gpar)}, WG>(lds, gbl, GPART, threadIdx.x);")
            L.append("#define GB(j) lds_gb<R>(gbl, j, lane)")
        L.append("    int lam[NPAR];")
        L.append("#pragma unroll")
        L.append("    for (int i = 0; i < NPAR; ++i) lam[i] = hel[h * NPAR + i];")
        xw_init = getattr(self, "xw_init", [])
        if xw_init:
            nx = len(xw_init)
            # LDS position of each slot in this precision's kernel, -1: kept in registers
            pos = {}
            for j, prec in ((1, "64"), (2, "32")):
                n, pos[prec] = 0, []
                for item in xw_init:
                    pos[prec].append(n if item[j] else -1)
                    n += 1 if item[j] else 0
                pos[prec + "n"] = n
            xwp = ", ".join(f"sizeof(R) == 8 ? {a} : {b}" for a, b in zip(pos["64"], pos["32"]))
            L.append(f"    // {nx} external wavefunctions computed once: in LDS, private to the lane, or in registers")
            L.append(f"    constexpr int XWP[{nx}] = {{{xwp}}};")
            L.append(f"    constexpr int NXL = sizeof(R) == 8 ? {pos['64n']} : {pos['32n']};")
            L.append("    __shared__ R xw_wg[NXL > 0 ? WG * NXL * 8 * 64 : 1];")
            L.append("    R* const xw = xw_wg + (threadIdx.x >> 6) * (NXL * 8 * 64);")
            L.append(f"    [[maybe_unused]] W4<R> xwr[{nx}];")
            for k, (code, _, _) in enumerate(xw_init):
                L.append(f"    {{ const W4<R> t = {code}; if constexpr (XWP[{k}] >= 0) st_w4<R>(xw, XWP[{k}], lane, t); "
                         f"else xwr[{k}] = t; }}")
            L.append("#define XW(k) (XWP[k] >= 0 ? ld_w4<R>(xw, XWP[k], lane) : xwr[k])")
        L.append(f"    constexpr int NW = {nwin};")
        if jamps_in_lds or mode == "slots":
            acc = "double" if jamp_mode == "atomic64" else "R"
            L.append(f"    // jamps accumulate in LDS, one private slot per lane ({jamp_mode})")
            L.append(f"    __shared__ {acc} Jl_wg[WG * 2 * NW * 64];")
            L.append(f"    {acc}* const Jl = Jl_wg + (threadIdx.x >> 6) * (2 * NW * 64);")
            L.append("#pragma unroll")
            if jamp_mode == "auto":
                L.append("    for (int s = 0; s < 2 * NW; ++s) jamp_zero<R>(&Jl[s * 64 + lane]);")
            else:
                L.append(f"    for (int s = 0; s < 2 * NW; ++s) Jl[s * 64 + lane] = ({acc})0;")
            if jamp_mode == "rmw":
                L.append("#define JADD(s, ri, v) (Jl[(2 * (s) + (ri)) * 64 + lane] += (v))")
                L.append("#define JGET(s, ri) ((R)Jl[(2 * (s) + (ri)) * 64 + lane])")
                L.append(f"#define JZERO(s, ri) (Jl[(2 * (s) + (ri)) * 64 + lane] = ({acc})0)")
            elif jamp_mode == "auto":
                L.append("#define JADD(s, ri, v) jamp_add<R>(&Jl[(2 * (s) + (ri)) * 64 + lane], (v))")
                L.append("#define JGET(s, ri) jamp_get<R>(&Jl[(2 * (s) + (ri)) * 64 + lane])")
                L.append("#define JZERO(s, ri) jamp_zero<R>(&Jl[(2 * (s) + (ri)) * 64 + lane])")
            else:
                L.append(f"#define JADD(s, ri, v) lds_add<{acc}>(&Jl[(2 * (s) + (ri)) * 64 + lane], ({acc})(v))")
                L.append(f"#define JGET(s, ri) ((R)__hip_atomic_load(&Jl[(2 * (s) + (ri)) * 64 + lane], "
                         "__ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT))")
                L.append(f"#define JZERO(s, ri) __hip_atomic_store(&Jl[(2 * (s) + (ri)) * 64 + lane], ({acc})0, "
                         "__ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT)")
        else:
            L.append("    R Jr[2 * NW];")
            L.append("#pragma unroll")
            L.append("    for (int s = 0; s < 2 * NW; ++s) Jr[s] = (R)0;")
            L.append("#define JADD(s, ri, v) (Jr[2 * (s) + (ri)] += (v))")
            L.append("#define JGET(s, ri) Jr[2 * (s) + (ri)]")
        if mode == "slots":
            L.append("    R* const po = jamp + (int64_t)n_good * (2 * NC) * ld + (int64_t)h * (2 * NSLOT) * ld + e;")
            # evicting a window slot: JTAKE reads it into registers and clears it (LDS
            # accesses complete in order, so no wait is needed there); JPUT stores the pair
            # to its partial slot later, once the read has long completed
            L.append("#define JTAKE(s, k) const R fr##k = JGET(s, 0), fi##k = JGET(s, 1); JZERO(s, 0); JZERO(s, 1)")
            L.append("#define JLAST(s, k) const R fr##k = JGET(s, 0), fi##k = JGET(s, 1)")
            L.append("#define JPUT(p, k) do { if (live) { po[(int64_t)(2 * (p)) * ld] = fr##k; "
                     "po[(int64_t)(2 * (p) + 1) * ld] = fi##k; } } while (0)")
        L.append("    cx<R> a, sa;")
        L.append("    int ch = -1;")
        L.append("    double sde_ch = 0.0, sde_all = 0.0;")
        L.append("    if constexpr (SDE) ch = (e < n_evt) ? chan[e] : -1;")
        L.append("#define SDEACC(d, k) do { if constexpr (SDE) { "
                 "const double w_ = (k) * ((double)a.r * (double)a.r + (double)a.i * (double)a.i); "
                 "sde_all += w_; sde_ch += ((d) == ch) ? w_ : 0.0; } } while (0)")
        L.extend(body)
        L.append("    if constexpr (SDE) {")
        L.append("        if (live && e < n_evt) {")
        L.append("            double* so = sde + (int64_t)h * 2 * ld + e;")
        if first:
            L.append("            so[0] = sde_ch;")
            L.append("            so[ld] = sde_all;")
        else:
            L.append("            so[0] += sde_ch;")
            L.append("            so[ld] += sde_all;")
        L.append("        }")
        L.append("    }")
        if mode == "jamps":
            if fused:
                L.append("    if (fc.aop) {  // colour sum here: D |M_h|^2 of this lane's event, to [h][event]")
                L.append("        double me_h;")
                if not jamps_in_lds and self.nc <= 6:
                    # up to six flows in FP64: the scalar colour sum from the registers
                    L.append("        if constexpr (sizeof(R) == 8) {")
                    L.append("            me_h = colour_sum_regs<NC>(Jr, static_cast<const double*>(fc.aop));")
                    L.append("        } else {")
                if jamps_in_lds:
                    src = "Jl"
                    L.append("        __syncthreads();  // every jamp update of the wave has completed")
                else:
                    # register jamps go to the momentum area of LDS, which is no longer read (with
                    # the helicity sum here: an area per wave)
                    src = "Js"
                    L.append("        __syncthreads();")
                    if hsum:
                        L.append("        R* Js = reinterpret_cast<R*>(lds);")
                        L.append("        if constexpr (hsum) {")
                        L.append("            __shared__ R Jst[16 * 2 * NC * 64];")
                        L.append("            Js = Jst + (threadIdx.x >> 6) * (2 * NC * 64);")
                        L.append("        }")
                    else:
                        L.append("        R* Js = reinterpret_cast<R*>(lds);")
                        L.append("        if constexpr (WG > 1) {  // the momentum area is shared: a staging area per wave")
                        L.append("            __shared__ R Jst_wg[WG * 2 * NC * 64];")
                        L.append("            Js = Jst_wg + (threadIdx.x >> 6) * (2 * NC * 64);")
                        L.append("        }")
                    L.append("#pragma unroll")
                    L.append("        for (int s = 0; s < 2 * NC; ++s) Js[s * 64 + lane] = Jr[s];")
                    L.append("        __syncthreads();")
                L.append("        if constexpr (sizeof(R) == 8)")
                L.append(f"            me_h = colour_sum_lds<NC>({src}, static_cast<const double*>(fc.aop), lane);")
                L.append("        else if (fc.form == ME_MIXED_BF16)")
                L.append(f"            me_h = colour_sum_lds_h16<NC, Bf16Terms>({src}, static_cast<const __bf16*>(fc.aop), "
                         "static_cast<const __bf16*>(fc.aop_lo), fc.lo_mask, lane);")
                L.append("        else")
                L.append(f"            me_h = colour_sum_lds_h16<NC, Fp16Terms>({src}, static_cast<const _Float16*>(fc.aop), "
                         "static_cast<const _Float16*>(fc.aop), 0, lane);")
                if not jamps_in_lds and self.nc <= 6:
                    L.append("        }")
                if hsum:
                    L.append("        if constexpr (hsum) {  // the helicity sum: the separate kernel's groups and order")
                    L.append("            __shared__ double red[16 * 64];")
                    L.append("            red[hr * 64 + lane] = me_h;")
                    L.append("            __syncthreads();")
                    L.append("            if (threadIdx.x < 64 && e < n_evt) {")
                    L.append("                double s = 0.0;")
                    L.append("                for (int h0 = 0; h0 < n_good; h0 += fc.hel_per_group) {")
                    L.append("                    const int h1 = min(n_good, h0 + fc.hel_per_group);")
                    L.append("                    double m = 0.0;")
                    L.append("                    for (int k = h0; k < h1; ++k) m += red[k * 64 + lane];")
                    L.append("                    s += m;")
                    L.append("                }")
                    L.append("                fc.hsum_out[e] = s * fc.hsum_scale;")
                    L.append("            }")
                    L.append("            return;")
                    L.append("        }")
                L.append("        if (live && e < n_evt) reinterpret_cast<double*>(jamp)[(int64_t)h * n_evt + e] = me_h;")
                L.append("        return;")
                L.append("    }")
            # all reads first (one wait), then the stores
            L.append("    R jo[2 * NC];")
            L.append("#pragma unroll")
            L.append("    for (int s = 0; s < NC; ++s) {")
            L.append("        jo[2 * s] = JGET(s, 0);")
            L.append("        jo[2 * s + 1] = JGET(s, 1);")
            L.append("    }")
            L.append("    if (live && e < n_evt) {")
            L.append("        R* o = jamp + (int64_t)h * (2 * NC) * ld + e;")
            L.append("#pragma unroll")
            L.append("        for (int s = 0; s < 2 * NC; ++s) o[s * ld] = jo[s];")
            L.append("    }")
        for m in ("PM", "GB", "XW", "JADD", "JGET", "JZERO", "JTAKE", "JLAST", "JPUT", "SDEACC"):
            L.append(f"#undef {m}")
        L.append("}")
        return L

    def _lane_kernel_text(self, body):
        """Kernel of the e+e- processes with one lane per event: the momenta staged once, then
        for each good helicity the diagram program, the colour sum (one flow; in the mixed forms
        the scalar equivalent of the 16-bit tile) and the helicity sum in the groups and order of
        the separate helicity-sum kernel, so the result is bitwise that of the other paths."""
        if self.nc > 6:
            raise ValueError("the lane-per-event kernel sums at most six colour flows in registers")
        L = []
        L.append("template <class R>")
        L.append(f"__global__ __launch_bounds__(64, sizeof(R) == 8 ? {LANE_MIN_WAVES[0]} : {LANE_MIN_WAVES[1]}) void amp_lanes("
                 "const double* __restrict__ mom, int64_t n_evt, "
                 "const signed char* __restrict__ hel, int n_good, double mt, double gs, FusedColour fc)")
        L.append("{")
        L.append("    __shared__ double lds[4 * NPAR * 64];")
        L.append("    const int lane = threadIdx.x;")
        L.append("    const int64_t e0 = xcd_remap(blockIdx.x, gridDim.x) * 64;")
        L.append("    const int64_t e = e0 + lane;")
        L.append("    stage_momenta<NPAR, 1>(mom, n_evt, e0, lds, lane);")
        L.append("    // momenta re-read from LDS at each use, so that nothing computed from them is held")
        L.append("    // across the helicity loop")
        L.append("#define PM(i) lds_p4(lds, i, lane)")
        L.append("#define SDEACC(d, k) do { } while (0)")
        L.append("#define JADD(s, ri, v) (Jr[2 * (s) + (ri)] += (v))")
        if LANE_HOIST_EXT:
            # each external state for both helicities, once per event; the loop selects
            ext = re.compile(r"^\s*const W4<R> (w\d+) = (ext_\w+<R>\(.*lam\[(\d+)\].*\));$")
            kept = []
            for ln in body:
                m = ext.match(ln)
                if not m:
                    kept.append(ln)
                    continue
                w, call, i = m.groups()
                call = re.sub(r"\bm\d+_(\d+)\b", r"PM(\1)", call)   # momenta read before the loop
                plus, minus = (call.replace(f"lam[{i}]", v) for v in ("1", "-1"))
                L.append(f"    const W4<R> {w}_p = {plus}, {w}_m = {minus};")
                kept.append(f"    const W4<R> {w} = lam[{i}] > 0 ? {w}_p : {w}_m;")
            body = kept
        L.append("    double s = 0.0, m = 0.0;")
        L.append("    int in_group = 0;")
        L.append("#pragma unroll 1")
        L.append("    for (int h = 0; h < n_good; ++h) {")
        L.append("        int lam[NPAR];")
        L.append("#pragma unroll")
        L.append("        for (int i = 0; i < NPAR; ++i) lam[i] = hel[h * NPAR + i];")
        L.append("        R Jr[2 * NC] = {};")
        L.append("        cx<R> a, sa;")
        L += ["    " + ln for ln in body]
        L.append("#pragma unroll")
        L.append("        for (int k = 0; k < 2 * NC; ++k) asm volatile(\"\" : \"+v\"(Jr[k]));  // the jamps as the other paths hold them")
        L.append("        if constexpr (sizeof(R) == 8)")
        L.append("            m += colour_sum_regs<NC>(Jr, static_cast<const double*>(fc.aop));")
        L.append("        else if constexpr (NC == 1) {  // the 16-bit forms: one flow only")
        L.append("            if (fc.form == ME_MIXED_BF16)")
        L.append("                m += cs1_h16<Bf16Terms>(Jr[0], Jr[1], static_cast<const __bf16*>(fc.aop));")
        L.append("            else")
        L.append("                m += cs1_h16<Fp16Terms>(Jr[0], Jr[1], static_cast<const _Float16*>(fc.aop));")
        L.append("        }")
        L.append("        if (++in_group == fc.hel_per_group || h + 1 == n_good) {")
        L.append("            s += m;")
        L.append("            m = 0.0;")
        L.append("            in_group = 0;")
        L.append("        }")
        L.append("    }")
        L.append("    if (e < n_evt) fc.hsum_out[e] = s * fc.hsum_scale;")
        L.append("#undef PM")
        L.append("#undef SDEACC")
        L.append("#undef JADD")
        L.append("}")
        return L

    def _reduce_text(self):
        """the partial slots of each jamp, summed in flush order, into the jamp layout"""
        offs = [0]
        lst = []
        for c in range(self.nc):
            lst += [p for p, j in enumerate(self.partial_jamp) if j == c]
            offs.append(len(lst))
        L = []
        L.append(f"__constant__ int slot_offset[NC + 1] = {{{', '.join(map(str, offs))}}};")
        L.append(f"__constant__ int slot_list[NSLOT] = {{{', '.join(map(str, lst))}}};")
        L.append("template <class R>")
        L.append("__global__ __launch_bounds__(256) void reduce_kernel(R* __restrict__ jamp, int64_t ld, int n_good, "
                 "int64_t n_evt)")
        L.append("{")
        L.append("    const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;")
        L.append("    const int h = blockIdx.y;")
        L.append("    if (col >= n_evt) return;")
        L.append("    const R* P = jamp + (int64_t)n_good * (2 * NC) * ld + (int64_t)h * (2 * NSLOT) * ld + col;")
        L.append("    R* J = jamp + (int64_t)h * (2 * NC) * ld + col;")
        L.append("    for (int c = 0; c < NC; ++c) {")
        L.append("        R re = (R)0, im = (R)0;")
        L.append("        for (int k = slot_offset[c]; k < slot_offset[c + 1]; ++k) {")
        L.append("            const int s = slot_list[k];")
        L.append("            re += P[(int64_t)(2 * s) * ld];")
        L.append("            im += P[(int64_t)(2 * s + 1) * ld];")
        L.append("        }")
        L.append("        J[(int64_t)(2 * c) * ld] = re;")
        L.append("        J[(int64_t)(2 * c + 1) * ld] = im;")
        L.append("    }")
        L.append("}")
        return L


# processes whose diagram program is not emitted yet: the library reports them as unknown
NOT_EMITTED = set()


_PM = re.compile(r"PM\((\d+)\)")
_GB = re.compile(r"GB\((\d+)\)")
_XW = re.compile(r"XW\((\d+)\)")


def _pipeline_momenta(lines, marks, puts=None):
    """Rewrite a diagram program so that the LDS reads of amplitude step s (momenta PM(i),
    gluon bases GB(j)) land in registers (const P4 m<s>_<i>, GB g<s>_<j>) at one point: before
    the amplitude of step s-1 (step 0: at its start).  marks[s] = (first node line, amplitude
    line, first jamp-update line) of step s, indices into lines.  puts[s] (window programs): the
    partial-slot stores of the slots step s evicted, placed after the amplitude of step s+1 (the
    caller places those of the last step)."""
    out = []
    used = []
    for s, (a, b, c) in enumerate(marks):
        ks = sorted({int(k) for ln in lines[a:c] for k in _PM.findall(ln)})
        gs = sorted({int(k) for ln in lines[a:c] for k in _GB.findall(ln)})
        xs = sorted({int(k) for ln in lines[a:c] for k in _XW.findall(ln)}) if PREFETCH_EXT else []
        used.append((ks, gs, xs))

    def decl(s):
        ks, gs, xs = used[s]
        return ([f"    P4 m{s}_{k} = PM({k});" for k in ks] + [f"    GBT<R> g{s}_{k} = GB({k});" for k in gs]
                + [f"    W4<R> y{s}_{k} = XW({k});" for k in xs])

    def pin(s):
        if not PIN_MOMENTA:
            return []
        ks, gs, xs = used[s]
        return ([f"    pin_p4<R>(m{s}_{k});" for k in ks] + [f"    pin_gb<R>(g{s}_{k});" for k in gs]
                + ([f"    pin_w4<R>(y{s}_{k});" for k in xs] if PIN_EXT else []))

    def sub(s, ln):
        ln = _PM.sub(lambda m: f"m{s}_{m.group(1)}", ln)
        if PREFETCH_EXT:
            ln = _XW.sub(lambda m: f"y{s}_{m.group(1)}", ln)
        return _GB.sub(lambda m: f"g{s}_{m.group(1)}", ln)

    pos = 0
    for s, (a, b, c) in enumerate(marks):
        out += lines[pos:a]                      # jamp updates of step s-1 (or preamble)
        if s == 0:
            out += decl(0)
        out += pin(s)
        out += [sub(s, ln) for ln in lines[a:b]]   # nodes of step s
        if s + 1 < len(marks):
            out += decl(s + 1)                   # next step's reads, ahead of this step's atomics
        out += [sub(s, ln) for ln in lines[b:c]]   # amplitude (+ channel weight) of step s
        if puts and s > 0:
            out += puts[s - 1]
        pos = c
    out += lines[pos:]
    return out


def stub_source(nm):
    return (f"// {nm}: diagram program not generated in this build\n"
            '#include "../process.hpp"\n'
            f"namespace me {{ const ProcessDesc* process_{nm}() {{ return nullptr; }} }}\n")


def generate(outdir, names=None):
    os.makedirs(outdir, exist_ok=True)
    written = []
    for nm in names or ALL_PROCESSES:
        if nm in NOT_EMITTED:
            path = os.path.join(outdir, f"proc_{nm}.hip")
            src = stub_source(nm)
            if not os.path.exists(path) or open(path).read() != src:
                with open(path, "w") as f:
                    f.write(src)
            written.append((nm, path, None))
            continue
        P = Process(nm)
        src = P.source()
        extra = getattr(P, "extra_files", {})
        for stale in os.listdir(outdir):
            if stale.startswith(f"proc_{nm}_amp_seg") and stale not in extra:
                os.remove(os.path.join(outdir, stale))
        for fname, fsrc in extra.items():
            fpath = os.path.join(outdir, fname)
            if not os.path.exists(fpath) or open(fpath).read() != fsrc:
                with open(fpath, "w") as f:
                    f.write(fsrc)
        path = os.path.join(outdir, f"proc_{nm}.hip")
        old = open(path).read() if os.path.exists(path) else None
        if old != src:
            with open(path, "w") as f:
                f.write(src)
        written.append((nm, path, P))
    return written

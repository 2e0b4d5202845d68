"""Tree-level Feynman-diagram generator that emits the per-process HIP code of
the GPU path (build-time only; not used at run time).

The paper's Born and real-emission equations define a tree amplitude as the
sum of Feynman diagrams, |M|^2 as its absolute square summed over helicities
and colours.  For every process this module:

1. enumerates the tree diagrams of a QCD+QED model (Feynman gauge, quark-
   gluon / fermion-photon / three-gluon / four-gluon vertices, the four-gluon
   vertex split into its three colour structures), sharing every off-shell
   sub-current between the diagrams that contain it;
2. computes each diagram's colour factor numerically from explicit SU(3)
   generators and projects it on the colour-flow basis (strings of generators
   along the quark lines), giving exact rational complex coefficients;
3. builds the colour matrix of that basis and its Cholesky factor;
4. finds the helicity combinations that are not identically zero by the
   chirality of massless fermion lines;
5. emits straight-line HIP device code: a helicity-independent FP64 prologue
   (internal momenta, propagator denominators, external-state data) and a
   per-helicity body that evaluates every sub-current once and accumulates
   the flow vector J.

Conventions: all particles are treated as incoming; an outgoing particle is
an incoming antiparticle with momentum -p.  Vertex rules are those of
Peskin-Schroeder (quark-gluon i g gamma^mu T^a, fermion-photon -i e Q gamma^mu,
three-gluon g f^{abc} V_{mu nu rho}, four-gluon -i g^2 sum f f (g g - g g),
propagators i(pslash+m)/(p^2-m^2) and -i g_{mu nu}/p^2).  Coupling
magnitudes and the factors of i are tracked symbolically and folded into the
colour coefficients and one overall FP64 factor, so the device routines
carry neither.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np

# ---------------------------------------------------------------------------
# model
# ---------------------------------------------------------------------------
FERMIONS = {  # name: (mass symbol, charge, coloured)
    "t": ("MT", Fraction(2, 3), True),
    "u": ("0", Fraction(2, 3), True),
    "e-": ("0", Fraction(-1), False),
    "mu-": ("0", Fraction(-1), False),
}
ANTI = {"t": "t~", "u": "u~", "e-": "e+", "mu-": "mu+"}
ANTI.update({v: k for k, v in list(ANTI.items())})
ANTI["g"] = "g"
ANTI["a"] = "a"


def is_fermion(t):
    return t in FERMIONS


def is_antifermion(t):
    return t in ANTI and ANTI[t] in FERMIONS


def flavour(t):
    return t if is_fermion(t) else ANTI[t]


def coloured(t):
    if t == "g":
        return True
    if t == "a":
        return False
    return FERMIONS[flavour(t)][2]


def cdim(t):
    if t == "g":
        return 8
    if t == "a":
        return 1
    return 3 if coloured(t) else 1


# ---------------------------------------------------------------------------
# SU(3), built here from the Gell-Mann matrices
# ---------------------------------------------------------------------------
def _su3():
    T = np.zeros((8, 3, 3), complex)
    T[0][0, 1] = T[0][1, 0] = 0.5
    T[1][0, 1], T[1][1, 0] = -0.5j, 0.5j
    T[2][0, 0], T[2][1, 1] = 0.5, -0.5
    T[3][0, 2] = T[3][2, 0] = 0.5
    T[4][0, 2], T[4][2, 0] = -0.5j, 0.5j
    T[5][1, 2] = T[5][2, 1] = 0.5
    T[6][1, 2], T[6][2, 1] = -0.5j, 0.5j
    T[7] = np.diag([1.0, 1.0, -2.0]) / (2.0 * math.sqrt(3.0))
    # [T^a, T^b] = i f^{abc} T^c  and Tr(T^c T^d) = delta/2
    comm = np.einsum('aij,bjk->abik', T, T) - np.einsum('bij,ajk->abik', T, T)
    f = np.real(-2j * np.einsum('abik,cki->abc', comm, T))
    f[np.abs(f) < 1e-14] = 0.0
    return T, f


TGEN, FSTR = _su3()


# ---------------------------------------------------------------------------
# diagram enumeration
# ---------------------------------------------------------------------------
class Node:
    """An external wavefunction or an off-shell sub-current."""

    def __init__(self, kind, legs, ptype, children=(), phase=0, qfac=Fraction(1), ncoup=(0, 0)):
        self.kind = kind
        self.legs = frozenset(legs)
        self.ptype = ptype
        self.children = list(children)
        self.phase = phase      # power of i
        self.qfac = qfac        # product of electric charges
        self.ncoup = ncoup      # (powers of g_s, powers of e)
        self.ctens = None
        self.caxes = None
        self.id = None
        self.mass = "0"
        self.boson = None


class Amp:
    """One diagram amplitude (a four-gluon diagram gives three, one per colour structure)."""

    def __init__(self, kind, children, phase, qfac, ncoup, diagram):
        self.kind = kind
        self.children = children
        self.phase = phase
        self.qfac = qfac
        self.ncoup = ncoup
        self.diagram = diagram
        self.ctens = None
        self.coef = None
        self.boson = None


def _vertex_bosons(ptype, bosons):
    """Vector bosons that couple to fermion flavour ptype in the model."""
    out = []
    f = flavour(ptype)
    if "g" in bosons and FERMIONS[f][2]:
        out.append("g")
    if "a" in bosons:
        out.append("a")
    return out


class Process:
    def __init__(self, name, incoming, outgoing, bosons, avg, ident=1.0):
        self.name = name
        self.incoming = list(incoming)
        self.outgoing = list(outgoing)
        self.bosons = bosons
        self.avg = avg
        self.ident = ident
        self.phys = self.incoming + self.outgoing
        self.npart = len(self.phys)
        # all-incoming particle type of every leg
        self.itype = [p for p in self.incoming] + [ANTI[p] for p in self.outgoing]
        self.memo = {}
        self.nodes = []
        self.amps = []
        self.ndiagrams = 0

    # -- enumeration ---------------------------------------------------------
    def _ext(self, k):
        key = (frozenset([k]), self.itype[k])
        if key not in self.memo:
            n = Node("ext", [k], self.itype[k])
            t = self.itype[k]
            n.mass = FERMIONS[flavour(t)][0] if t not in ("g", "a") else "0"
            self.memo[key] = [n]
        return self.memo[key]

    def subtrees(self, S, X):
        """All distinct sub-currents over leg set S whose off-shell line enters
        its parent vertex as an incoming particle of type X."""
        S = frozenset(S)
        key = (S, X)
        if key in self.memo:
            return self.memo[key]
        if len(S) == 1:
            (k,) = tuple(S)
            res = self._ext(k) if self.itype[k] == X else []
            self.memo[key] = res
            return res
        res = []
        items = sorted(S)
        subsets = [frozenset(c) for r in range(1, len(items)) for c in itertools.combinations(items, r)]
        if X in ("g", "a"):
            # fermion pair -> vector
            for f in FERMIONS:
                if X not in _vertex_bosons(f, self.bosons):
                    continue
                for S1 in subsets:
                    S2 = S - S1
                    for r in self.subtrees(S1, ANTI[f]):
                        for c in self.subtrees(S2, f):
                            res.append(self._mk("ffv_vec", S, X, [r, c], boson=X, flav=f))
            if X == "g" and "g" in self.bosons:
                lo = min(items)
                for S1 in subsets:
                    if lo not in S1:
                        continue
                    S2 = S - S1
                    for a in self.subtrees(S1, "g"):
                        for b in self.subtrees(S2, "g"):
                            res.append(self._mk("vvv_vec", S, X, [a, b]))
                for parts in _three_partitions(items):
                    A = self.subtrees(parts[0], "g")
                    B = self.subtrees(parts[1], "g")
                    C = self.subtrees(parts[2], "g")
                    for a in A:
                        for b in B:
                            for c in C:
                                for k in range(3):
                                    res.append(self._mk("vvvv_vec%d" % k, S, X, [a, b, c]))
        elif is_fermion(X):
            # column current: this vertex sees it in the row slot; children column + vector
            for V in _vertex_bosons(X, self.bosons):
                for S1 in subsets:
                    S2 = S - S1
                    for c in self.subtrees(S1, X):
                        for v in self.subtrees(S2, V):
                            res.append(self._mk("ffv_col", S, X, [c, v], boson=V, flav=X))
        else:
            f = flavour(X)
            for V in _vertex_bosons(f, self.bosons):
                for S1 in subsets:
                    S2 = S - S1
                    for r in self.subtrees(S1, X):
                        for v in self.subtrees(S2, V):
                            res.append(self._mk("ffv_row", S, X, [r, v], boson=V, flav=f))
        self.memo[key] = res
        return res

    def _mk(self, kind, S, X, ch, boson=None, flav=None):
        n = Node(kind, S, X, ch)
        ph = sum(c.phase for c in ch)
        q = Fraction(1)
        gs = sum(c.ncoup[0] for c in ch)
        ee = sum(c.ncoup[1] for c in ch)
        for c in ch:
            q *= c.qfac
        if kind.startswith("ffv"):
            if boson == "g":
                ph += 1          # vertex i g
                gs += 1
            else:
                ph += 3          # vertex -i e Q
                ee += 1
                q *= FERMIONS[flav][1]
            if kind == "ffv_vec":
                ph += 3          # vector propagator -i
            else:
                ph += 1          # fermion propagator i
                n.mass = FERMIONS[flav][0]
        elif kind == "vvv_vec":
            ph += 3              # vertex g (no i), propagator -i
            gs += 1
        else:                    # four-gluon: vertex -i g^2, propagator -i
            ph += 3 + 3
            gs += 2
        n.phase = ph % 4
        n.qfac = q
        n.ncoup = (gs, ee)
        n.boson = boson
        return n

    def enumerate(self):
        root = self.npart - 1
        X = self.itype[root]
        rest = frozenset(range(self.npart - 1))
        items = sorted(rest)
        subsets = [frozenset(c) for r in range(1, len(items)) for c in itertools.combinations(items, r)]
        L = self._ext(root)[0]
        amps = []
        diag = 0

        def add(kind, ch, boson=None, flav=None):
            nonlocal diag
            ph = sum(c.phase for c in ch) + L.phase
            q = Fraction(1)
            gs = sum(c.ncoup[0] for c in ch)
            ee = sum(c.ncoup[1] for c in ch)
            for c in ch:
                q *= c.qfac
            if kind.startswith("ffv"):
                if boson == "g":
                    ph += 1
                    gs += 1
                else:
                    ph += 3
                    ee += 1
                    q *= FERMIONS[flav][1]
            elif kind == "vvv_amp":
                gs += 1
            else:
                ph += 3
                gs += 2
            a = Amp(kind, list(ch) + [L], ph % 4, q, (gs, ee), diag)
            a.boson = boson
            amps.append(a)

        if X in ("g", "a"):
            for f in FERMIONS:
                if X not in _vertex_bosons(f, self.bosons):
                    continue
                for S1 in subsets:
                    for r in self.subtrees(S1, ANTI[f]):
                        for c in self.subtrees(rest - S1, f):
                            add("ffv_amp", [r, c], boson=X, flav=f)
                            diag += 1
            if X == "g" and "g" in self.bosons:
                lo = min(items)
                for S1 in subsets:
                    if lo not in S1:
                        continue
                    for a in self.subtrees(S1, "g"):
                        for b in self.subtrees(rest - S1, "g"):
                            add("vvv_amp", [a, b])
                            diag += 1
                for parts in _three_partitions(items):
                    for a in self.subtrees(parts[0], "g"):
                        for b in self.subtrees(parts[1], "g"):
                            for c in self.subtrees(parts[2], "g"):
                                for k in range(3):
                                    add("vvvv_amp%d" % k, [a, b, c])
                                diag += 1
        elif is_fermion(X):
            # root is a column spinor: children row + vector
            for V in _vertex_bosons(X, self.bosons):
                for S1 in subsets:
                    for r in self.subtrees(S1, ANTI[X]):
                        for v in self.subtrees(rest - S1, V):
                            a = [r, v]
                            add("ffv_amp_rootcol", a, boson=V, flav=X)
                            diag += 1
        else:
            f = flavour(X)
            for V in _vertex_bosons(f, self.bosons):
                for S1 in subsets:
                    for c in self.subtrees(S1, f):
                        for v in self.subtrees(rest - S1, V):
                            add("ffv_amp_rootrow", [c, v], boson=V, flav=f)
                            diag += 1
        self.amps = amps

        # Feynman-diagram count: a four-gluon vertex contributes three colour
        # structures (three terms) but is one diagram
        def sig(n):
            if n.kind == "ext":
                return ("e", min(n.legs))
            k = "vvvv" if n.kind.startswith("vvvv") else n.kind
            return (k,) + tuple(sig(c) for c in n.children)

        self.ndiagrams = len({sig(Node(a.kind, [], None, a.children)) for a in amps})
        # collect nodes in dependency order
        order = []
        seen = set()

        def visit(n):
            if id(n) in seen:
                return
            for c in n.children:
                visit(c)
            seen.add(id(n))
            order.append(n)

        for a in amps:
            for c in a.children:
                visit(c)
        for i, n in enumerate(order):
            n.id = i
        self.nodes = order
        return self

    # -- colour ---------------------------------------------------------------
    def coloured_legs(self):
        return [k for k in range(self.npart) if coloured(self.itype[k])]

    def colour(self):
        legs = self.coloured_legs()
        pos = {k: i for i, k in enumerate(legs)}
        dims = [cdim(self.itype[k]) for k in legs]
        full_shape = tuple(dims)

        def expand(n):
            """Colour tensor of node n over (its coloured external legs, off-shell axis)."""
            if n.ctens is not None:
                return n.ctens, n.caxes
            if n.kind == "ext":
                t = n.ptype
                if coloured(t):
                    n.ctens, n.caxes = np.eye(cdim(t), dtype=complex), [min(n.legs), None]
                else:
                    n.ctens, n.caxes = np.ones((), complex), []
                return n.ctens, n.caxes
            ch = [expand(c) for c in n.children]
            n.ctens, n.caxes = _combine(n.kind, n.children, ch, n.boson)
            return n.ctens, n.caxes

        for a in self.amps:
            ch = [expand(c) for c in a.children]
            t, axes = _combine(a.kind, a.children, ch, a.boson)
            # reorder to the canonical leg order
            if axes:
                perm = [axes.index(k) for k in legs]
                t = np.transpose(t, perm)
            a.ctens = t.reshape(full_shape) if legs else t.reshape(())
        # flow basis
        self.flows = _flow_basis(self)
        B = np.array([b.ravel() for b in self.flows])
        self.colour_matrix = np.real(np.conj(B) @ B.T)
        assert np.allclose(np.imag(np.conj(B) @ B.T), 0, atol=1e-12)
        for a in self.amps:
            d = a.ctens.ravel()
            c, res, rank, _ = np.linalg.lstsq(B.T, d, rcond=None)
            assert np.allclose(B.T @ c, d, atol=1e-12), (self.name, a.kind)
            a.coef = [_crational(x) for x in c]
        self.colour_matrix = np.array([[float(Fraction(x).limit_denominator(10000)) for x in row]
                                       for row in self.colour_matrix])
        return self

    # -- helicities -------------------------------------------------------------
    def good_helicities(self):
        """Helicity combinations not identically zero: on every massless
        fermion line the row and column spinors must sit in opposite chiral
        blocks (an odd number of gamma matrices connects them)."""
        lines = []
        for k in range(self.npart):
            t = self.itype[k]
            if is_antifermion(t) and FERMIONS[flavour(t)][0] == "0":
                cols = [j for j in range(self.npart) if self.itype[j] == flavour(t)]
                assert len(cols) == 1
                lines.append((k, cols[0]))
        good = []
        for h in range(1 << self.npart):
            lam = [1 if (h >> (self.npart - 1 - k)) & 1 else -1 for k in range(self.npart)]
            ok = True
            for r, c in lines:
                out_r = r >= len(self.incoming)     # row is an outgoing fermion (ubar) or incoming antifermion (vbar)
                rb = (1 if lam[r] > 0 else 2) if out_r else (2 if lam[r] > 0 else 1)
                out_c = c >= len(self.incoming)     # column is an outgoing antifermion (v) or incoming fermion (u)
                cb = (1 if lam[c] > 0 else 2) if out_c else (2 if lam[c] > 0 else 1)
                if rb == cb:
                    ok = False
            if ok:
                good.append(h)
        return good

    def coupling_powers(self):
        p = {a.ncoup for a in self.amps}
        assert len(p) == 1, p
        return p.pop()


def _three_partitions(items):
    """Unordered partitions of items into three nonempty blocks (canonical:
    blocks ordered by their smallest element)."""
    out = []
    n = len(items)
    for labels in itertools.product(range(3), repeat=n):
        blocks = [frozenset(items[i] for i in range(n) if labels[i] == b) for b in range(3)]
        if any(len(b) == 0 for b in blocks):
            continue
        mins = [min(b) for b in blocks]
        if mins[0] < mins[1] < mins[2]:
            out.append(blocks)
    return out


def _combine(kind, children, ch, boson):
    """Contract the children's colour tensors with the vertex colour factor.
    Each child tensor has its external axes (labelled by leg) and, last, its
    off-shell axis.  Returns (tensor, axis labels) where the off-shell axis
    (if any) is last and labelled None."""
    letters = iter("abcdefghijklmnopqrstuvwxyz")
    ext_axes = []
    specs = []
    ops = []
    offs = []
    for (t, axes), c in zip(ch, children):
        s = ""
        for ax in axes:
            if ax is None:
                continue
            L = next(letters)
            s += L
            ext_axes.append((ax, L))
        if t.ndim > len([a for a in axes if a is not None]):
            o = next(letters)
            s += o
            offs.append(o)
        else:
            offs.append(None)
        specs.append(s)
        ops.append(t)
    out_off = next(letters)
    vs = ""
    vops = []
    k = kind
    if k in ("ffv_vec", "ffv_col", "ffv_row", "ffv_amp", "ffv_amp_rootcol", "ffv_amp_rootrow"):
        # slots: row index i, column index j, gluon a ; photon: delta_ij
        if k == "ffv_vec":
            r, c = offs
            if boson == "g":
                vs, vops, off = "%s%s%s" % (out_off, r, c), [TGEN], out_off   # T^a_{ij}
            elif r:
                vs, vops, off = "%s%s" % (r, c), [np.eye(3)], None
            else:
                vs, vops, off = "", [], None
        elif k == "ffv_col":          # children: column c, vector v ; result index = row slot
            c, v = offs
            if boson == "g":
                vs, vops, off = "%s%s%s" % (v, out_off, c), [TGEN], out_off
            else:
                if c:
                    vs, vops, off = "%s%s" % (out_off, c), [np.eye(3)], out_off
                else:
                    vs, vops, off = "", [], None
        elif k == "ffv_row":          # children: row r, vector v ; result index = column slot
            r, v = offs
            if boson == "g":
                vs, vops, off = "%s%s%s" % (v, r, out_off), [TGEN], out_off
            else:
                if r:
                    vs, vops, off = "%s%s" % (r, out_off), [np.eye(3)], out_off
                else:
                    vs, vops, off = "", [], None
        else:
            # amplitude: children (row, col, vector) in some order
            if k == "ffv_amp":
                r, c, v = offs[0], offs[1], offs[2]
            elif k == "ffv_amp_rootcol":
                r, v, c = offs[0], offs[1], offs[2]
            else:
                c, v, r = offs[0], offs[1], offs[2]
            if boson == "g":
                vs, vops = "%s%s%s" % (v, r, c), [TGEN]
            else:
                vs, vops = ("%s%s" % (r, c), [np.eye(3)]) if r else ("", [])
            off = None
    elif k in ("vvv_vec", "vvv_amp"):
        a, b = offs[0], offs[1]
        if k == "vvv_vec":
            vs, vops, off = "%s%s%s" % (a, b, out_off), [FSTR], out_off
        else:
            vs, vops, off = "%s%s%s" % (a, b, offs[2]), [FSTR], None
    else:
        idx = int(k[-1])
        a, b, c = offs[0], offs[1], offs[2]
        d = out_off if "vec" in k else offs[3]
        e = next(letters)
        F = FSTR
        if idx == 0:
            vs = "%s%s%s,%s%s%s" % (a, b, e, c, d, e)
        elif idx == 1:
            vs = "%s%s%s,%s%s%s" % (a, c, e, b, d, e)
        else:
            vs = "%s%s%s,%s%s%s" % (a, d, e, b, c, e)
        vops = [F, F]
        off = out_off if "vec" in k else None
    out_spec = "".join(L for _, L in ext_axes) + (off or "")
    all_specs = [s for s in specs]
    all_ops = list(ops)
    if vs:
        all_specs += vs.split(",")
        all_ops += vops
    t = np.einsum(",".join(all_specs) + "->" + out_spec, *all_ops, optimize=True)
    axes = [ax for ax, _ in ext_axes] + ([None] if off else [])
    return t, axes


def _flow_basis(proc):
    """Colour-flow basis: for every pairing of row-type and column-type
    coloured external quarks, and every distribution of the external gluons
    into ordered strings along those pairings, the product of generator
    strings.  Returns tensors over the coloured legs in leg order."""
    legs = proc.coloured_legs()
    if not legs:
        return [np.ones(())]
    rows = [k for k in legs if is_antifermion(proc.itype[k])]
    cols = [k for k in legs if is_fermion(proc.itype[k])]
    gls = [k for k in legs if proc.itype[k] == "g"]
    letter = {k: chr(ord("a") + i) for i, k in enumerate(legs)}
    out_spec = "".join(letter[k] for k in legs)
    basis = []
    nl = len(rows)
    for pairing in itertools.permutations(cols):
        for assign in itertools.product(range(nl), repeat=len(gls)):
            groups = [[g for g, a in zip(gls, assign) if a == l] for l in range(nl)]
            for orders in itertools.product(*[list(itertools.permutations(gr)) for gr in groups]):
                specs, ops = [], []
                extra = iter("zyxwvutsrq")
                for l in range(nl):
                    seq = list(orders[l])
                    if not seq:
                        specs.append(letter[rows[l]] + letter[pairing[l]])
                        ops.append(np.eye(3))
                        continue
                    prev = letter[rows[l]]
                    for j, g in enumerate(seq):
                        nxt = letter[pairing[l]] if j == len(seq) - 1 else next(extra)
                        specs.append(letter[g] + prev + nxt)
                        ops.append(TGEN)
                        prev = nxt
                basis.append(np.einsum(",".join(specs) + "->" + out_spec, *ops, optimize=True))
    return basis


def _crational(x):
    r = Fraction(float(np.real(x))).limit_denominator(2000)
    i = Fraction(float(np.imag(x))).limit_denominator(2000)
    assert abs(float(r) - np.real(x)) < 1e-12 and abs(float(i) - np.imag(x)) < 1e-12, x
    return (r, i)


# ---------------------------------------------------------------------------
# process list
# ---------------------------------------------------------------------------
LEPTONS = ("e-", "e+", "mu-", "mu+")


def process_list():
    return [
        Process("ee_mumu", ["e-", "e+"], ["mu-", "mu+"], {"a"}, 0.25),
        Process("ee_uu", ["e-", "e+"], ["u", "u~"], {"a"}, 0.25),
        Process("ee_uug", ["e-", "e+"], ["u", "u~", "g"], {"a", "g"}, 0.25),
        Process("gg_tt", ["g", "g"], ["t", "t~"], {"g"}, 1.0 / 256.0),
        Process("uu_tt", ["u", "u~"], ["t", "t~"], {"g"}, 1.0 / 36.0),
        Process("gg_ttg", ["g", "g"], ["t", "t~", "g"], {"g"}, 1.0 / 256.0),
        Process("uu_ttg", ["u", "u~"], ["t", "t~", "g"], {"g"}, 1.0 / 36.0),
        Process("ug_ttu", ["u", "g"], ["t", "t~", "u"], {"g"}, 1.0 / 96.0),
        Process("gg_ttgg", ["g", "g"], ["t", "t~", "g", "g"], {"g"}, 1.0 / 256.0, ident=0.5),
    ]


# ---------------------------------------------------------------------------
# HIP emission
# ---------------------------------------------------------------------------
def _cplx_lit(fr):
    return "%.17g" % float(fr)


def _phase_coef(coef, phase, qfac):
    """coef (re, im) * i^phase * qfac as a complex Fraction pair."""
    re, im = coef
    for _ in range(phase % 4):
        re, im = -im, re
    return (re * qfac, im * qfac)


def _acc_code(J, c, a):
    """J += c * a for a rational complex constant c."""
    re, im = c
    out = []
    if re == 0 and im == 0:
        return out
    def term(k, x):
        if k == 1:
            return " + " + x
        if k == -1:
            return " - " + x
        return " + T(%s) * %s" % (_cplx_lit(k), x)
    if im == 0:
        out.append("%s.r = %s.r%s;" % (J, J, term(re, a + ".r")))
        out.append("%s.i = %s.i%s;" % (J, J, term(re, a + ".i")))
    elif re == 0:
        out.append("%s.r = %s.r%s;" % (J, J, term(-im, a + ".i")))
        out.append("%s.i = %s.i%s;" % (J, J, term(im, a + ".r")))
    else:
        out.append("%s.r = %s.r%s%s;" % (J, J, term(re, a + ".r"), term(-im, a + ".i")))
        out.append("%s.i = %s.i%s%s;" % (J, J, term(re, a + ".i"), term(im, a + ".r")))
    return out


def cholesky_lower(C):
    return np.linalg.cholesky(C)


FKS_BORNS = ("ee_uu", "gg_tt", "uu_tt", "gg_ttg")


def _charge(t, pos, kind, a):
    """Colour charge T^a of one leg applied to a colour tensor: T^a on a
    fundamental (row) index, -(T^a)^T on an antifundamental (column) index,
    -i f^{a..} on an adjoint index."""
    if kind == "r":
        M = TGEN[a]
    elif kind == "c":
        M = -TGEN[a].T
    else:
        M = -1j * FSTR[a]
    t = np.moveaxis(t, pos, 0)
    return np.moveaxis(np.tensordot(M, t, axes=([1], [0])), 0, pos)


def colour_correlators(p):
    """C^(kl)_{ab} = <flow a| T_k . T_l |flow b> over the coloured legs."""
    legs = p.coloured_legs()
    kinds = ["g" if p.itype[k] == "g" else ("r" if is_antifermion(p.itype[k]) else "c") for k in legs]
    nl, nf = len(legs), len(p.flows)
    C = np.zeros((nl, nl, nf, nf), complex)
    for k in range(nl):
        for l in range(nl):
            for b in range(nf):
                for a8 in range(8):
                    t2 = _charge(_charge(p.flows[b], l, kinds[l], a8), k, kinds[k], a8)
                    for a in range(nf):
                        C[k, l, a, b] += np.vdot(p.flows[a], t2)
    assert np.abs(C.imag).max() < 1e-12
    C = C.real
    assert np.abs(C.sum(axis=1)).max() < 1e-11          # colour conservation
    return legs, C


def emit_colour_corr(p):
    """Code for B_kl = sum_ab C^(kl)_ab rho_ab from the helicity-summed real
    symmetric density rho (packed upper triangle, row-major)."""
    legs, C = colour_correlators(p)
    nf = len(p.flows)
    L = ["  static constexpr int NCL = %d;" % len(legs),
         "  static constexpr int CLEG[NCL] = {%s};" % ", ".join(str(k) for k in legs),
         "  static constexpr int NRHO = %d;" % (nf * (nf + 1) // 2),
         "  template <class D> NLO_HD static void colour_corr(const D (&rho)[NRHO], D (&bkl)[NCL][NCL]) {"]
    for k in range(len(legs)):
        for l in range(len(legs)):
            if l < k:
                L.append("    bkl[%d][%d] = bkl[%d][%d];" % (k, l, l, k))
                continue
            terms = []
            idx = 0
            for a in range(nf):
                for b in range(a, nf):
                    c = C[k, l, a, b] * (1.0 if a == b else 2.0)
                    if abs(c) > 1e-14:
                        terms.append("D(%.17g) * rho[%d]" % (c, idx))
                    idx += 1
            L.append("    bkl[%d][%d] = %s;" % (k, l, " + ".join(terms) if terms else "D(0)"))
    L.append("  }")
    return L


# rough flops of each routine, for choosing the order of the helicity loops
_NODE_COST = {"ffv_vec": 128, "ffv_col": 132, "ffv_row": 132, "vvv_vec": 166, "vvvv_vec0": 124,
              "vvvv_vec1": 124, "vvvv_vec2": 124, "ext": 8}


def _massless_lines(p):
    lines = []
    for k in range(p.npart):
        t = p.itype[k]
        if is_antifermion(t) and FERMIONS[flavour(t)][0] == "0":
            c = [j for j in range(p.npart) if p.itype[j] == flavour(t)][0]
            lines.append((k, c))
    return lines


def helicity_order(p):
    """Order of the nested helicity loops (outermost first).  A sub-current over
    leg set S is evaluated once per helicity assignment of the loops down to
    the innermost of its legs, i.e. 2^(level+1) times; the root leg takes part
    in no sub-current and goes innermost.  Exhaustive search over the other
    legs minimises the estimated flops."""
    root = p.npart - 1
    others = list(range(p.npart - 1))
    best = None
    for perm in itertools.permutations(others):
        order = list(perm) + [root]
        lev = {k: i for i, k in enumerate(order)}
        cost = 0
        for n in p.nodes:
            l = max(lev[k] for k in n.legs)
            cost += _NODE_COST.get(n.kind, 130) * (2 ** (l + 1))
        if best is None or cost < best[0]:
            best = (cost, order)
    return best[1]


# Every vertex of the model is a real multiple of a vector coupling and no
# propagator carries a width.  At real momenta, complex conjugation then maps
# each external wavefunction to its opposite-helicity partner up to a phase
# (for spinors through the charge-conjugation-like matrix that leaves every
# gamma^mu invariant, for vectors eps_-lambda ~ eps_lambda^*), and each tree
# diagram picks up the same overall phase.  The flow vector of the reversed
# helicity set is thus a phase times J^*, and with a real colour matrix
# J^+ C J is unchanged: |M_h|^2 = |M_-h|^2.  The nested helicity sum therefore
# runs over the half in which one leg (a fermion where there is one) has bit 0
# and is doubled by the caller (HEL_SYM).  An axial coupling or a width would
# break this.
HEL_SYMMETRY = True

# External vector legs are summed over their two real linear polarisations
# instead of their two helicities: for each leg the helicity states are a
# unitary combination of them, so the summed |A|^2 is the same, and currents
# and amplitudes with a real vector need fewer multiplications.  The one
# exception is a vector leg that the helicity-reversal halving holds at one
# helicity (only when the process has no fermion): that argument needs a
# helicity state there (the sum over all the other legs does not depend on
# their basis).
LINEAR_POLARISATIONS = True


def _fixed_leg(p, order):
    """The leg the helicity-reversal halving holds at one helicity: a fermion
    if the loops have one (then every vector leg can take linear
    polarisations), else the outermost leg."""
    if not HEL_SYMMETRY:
        return -1
    for k in order[:-1]:
        if p.itype[k] not in ("g", "a"):
            return k
    return order[0]


def _linear(p, leg, fixed):
    return LINEAR_POLARISATIONS and p.itype[leg] in ("g", "a") and leg != fixed

# processes whose sub-currents one level above the deepest loop are also
# evaluated lazily inside it (more flops, far fewer live registers)
JIT_EXTRA_LEVELS = {"gg_ttgg": 1}
# the same for the FP64 instantiation where it differs.  Measured per 2^20
# g g -> t tbar g g events: FP64 with 0, 1, 2 and 3 extra lazy levels 54.6,
# 60, 48.2 and 40.8 ms (FP64 values take twice the registers; with three,
# every sub-current is evaluated in the deepest loop, which spills least:
# 1.3 against 4.7 KB per lane); FP32 with 1, 2 and 3 levels 11.0, 12.0 and
# 11.9 ms.  FP64 g g -> t tbar g: with one level 2.35, without 2.44 ms per
# 2^22 events.
JIT_EXTRA_LEVELS_FP64 = {"gg_ttgg": 3, "gg_ttg": 1}
# the same for the BF16 pair kernels (bf16x2: every operation is widened to
# FP32 and rounded back, so their code is the longest): g g -> t tbar g g
# with three levels 104 against 131 ms per 2^20 events (FP16 gains nothing:
# 8.4 against 8.1 ms)
JIT_EXTRA_LEVELS_BF16 = {"gg_ttgg": 3}
# the helicity sums of those FP64 instantiations order the amplitudes with
# ties broken towards the amplitude that is the last user of the most
# sub-currents already evaluated: FP64 g g -> t tbar g g 40.7 -> 38.5 ms per
# 2^20 events, g g -> t tbar g 2.38 -> 2.29 ms per 2^22 (the same order made
# the FP32 g g -> t tbar g kernel 16 % slower, so FP32 keeps the plain one)
FP64_FREE_FIRST = True
# stop the compiler from hoisting those lazily emitted sub-currents back out
KEEP_LAZY_IN_LOOP = True
# processes whose helicity loops read the internal momenta through the
# optimisation barrier at every use.  The momenta are the same for every
# helicity, so loop-invariant code motion would otherwise hoist every
# momentum-only factor of the vertices (Pslash's components, the momentum
# differences of the three-gluon vertex) out of all the loops and keep them
# live across the whole helicity sum.
OPAQUE_MOMENTA = ("gg_ttgg",)
# of those, processes whose FP64 helicity loops form each internal momentum
# from the external ones where it is used (same legs, same order of the sum
# as the prologue, so the same bits), instead of holding all of them in
# registers: 31 momenta cost 248 registers in FP64
FP64_MOMENTUM_SUMS = ("gg_ttgg",)
# waves per SIMD the FP32 |M|^2 kernel (default schedule) and the FP16/BF16
# pair kernels are compiled for: the register budget then is 512 / waves per
# lane (g g -> t tbar g needs 266 for one wave and spills 11 dwords at two;
# its FP64 kernel, 472 registers, spills 1.1 KB at two waves and ran 2.1x
# slower, so the FP64 kernels keep one)
WAVES_F32 = {"gg_ttg": 2}
# processes that also get the other lazy depth as a run-time schedule
# variant (kernel configuration `schedule` = 1), for the autotuner
SCHEDULE_ALTS = ("gg_ttg", "gg_ttgg")


def _qref(S, mslot, opq):
    """the momentum of leg set S: the stored slot, through the barrier if opq;
    opq == 2: FP64 sums the external momenta at each use instead"""
    if opq == 2 and len(S) > 1:
        return "qlegs<T, %s>(s.Q, %d)" % (", ".join(str(mslot[frozenset([k])]) for k in sorted(S)), mslot[S])
    return ("oq(s.Q[%d])" if opq else "s.Q[%d]") % mslot[S]


def _node_call(n, mslot, dslot, den="s.den", opq=False, wrap=None):
    """C++ expression evaluating sub-current n from its children (opq: read
    the momenta through the optimisation barrier; wrap(c): also child c)."""
    ch = [("ow(v%d)" if wrap and wrap(c) else "v%d") % c.id for c in n.children]
    Q = _qref(n.legs, mslot, opq)
    dk = dslot[(n.legs, n.mass if n.kind in ("ffv_col", "ffv_row") else "0")]
    D = "%s(s.den[%d])" % (den[1:], dk) if den.startswith("@") else "%s[%d]" % (den, dk)
    if n.kind == "ffv_vec":
        return "ffv_vec(%s, %s, %s)" % (ch[0], ch[1], D)
    if n.kind in ("ffv_col", "ffv_row"):
        if n.mass == "MT":
            return "%s(%s, %s, %s, %s, mt)" % (n.kind, ch[0], ch[1], Q, D)
        return "%s0(%s, %s, %s, %s)" % (n.kind, ch[0], ch[1], Q, D)
    if n.kind == "vvv_vec":
        QA = _qref(n.children[0].legs, mslot, opq)
        QB = _qref(n.children[1].legs, mslot, opq)
        return "vvv_vec(%s, %s, %s, %s, %s)" % (ch[0], QA, ch[1], QB, D)
    return "%s(%s, %s, %s, %s)" % (n.kind, ch[0], ch[1], ch[2], D)


def _ext_call(p, k, bit, nin):
    t = p.itype[k]
    out = k >= nin
    if t in ("g", "a"):
        return "wf_eps(s.x%d, %s, %s)" % (k, bit, "true" if out else "false")
    if is_fermion(t):
        return "%s(s.x%d, %s)" % ("wf_v" if out else "wf_u", k, bit)
    return "wf_bar(%s(s.x%d, %s))" % ("wf_u" if out else "wf_v", k, bit)


def _amp_call(a, ch, mslot, rootv, opq=False):
    """C++ expression of amplitude a with the root wavefunction rootv."""
    ch = ch[:-1] + [rootv]
    if a.kind == "ffv_amp":
        return "ffv_amp(%s, %s, %s)" % (ch[0], ch[2], ch[1])
    if a.kind == "ffv_amp_rootcol":
        return "ffv_amp(%s, %s, %s)" % (ch[0], ch[1], ch[2])
    if a.kind == "ffv_amp_rootrow":
        return "ffv_amp(%s, %s, %s)" % (ch[2], ch[1], ch[0])
    if a.kind == "vvv_amp":
        Qs = [_qref(c.legs, mslot, opq) for c in a.children]
        return "vvv_amp(%s, %s, %s, %s, %s, %s)" % (ch[0], Qs[0], ch[1], Qs[1], ch[2], Qs[2])
    return "%s(%s, %s, %s, %s)" % (a.kind, ch[0], ch[1], ch[2], ch[3])


def emit_nested(p, mslot, dslot, N, nin, jit_extra=None, fname="helicity_sum", free_first=False):
    """helicity_sum: nested loops over the states of all legs but the root
    (the leg taking part in no sub-current): helicities for fermions, linear
    polarisations for vectors, one helicity for the leg the reversal halving
    fixes.  A sub-current is evaluated at the loop level of its innermost leg
    and reused by all inner iterations; in the deepest loop the remaining
    sub-currents are evaluated just before their first use, amplitude by
    amplitude, and every amplitude is formed for both root states at once,
    giving two flow vectors and two calls of body.  jit_extra overrides the
    number of extra lazy levels, fname the function's name.  free_first
    breaks ties in the amplitude order towards the amplitude that is the last
    user of the most sub-currents already evaluated (shorter live ranges)."""
    order = helicity_order(p)
    lev = {k: i for i, k in enumerate(order)}
    root = order[-1]
    opq = (2 if p.name in FP64_MOMENTUM_SUMS else 1) if p.name in OPAQUE_MOMENTA else 0
    fixed = _fixed_leg(p, order)                    # held at one helicity (HEL_SYM)
    deep = N - 2                                    # deepest emitted loop
    if jit_extra is None:
        jit_extra = JIT_EXTRA_LEVELS.get(p.name, 0)
    jit_from = deep - jit_extra
    L = ["  // helicity loops, outermost first: legs %s (root leg %d folded into the amplitudes)"
         % (", ".join(str(k) for k in order[:-1]), root),
         "  template <class T, class F> NLO_HD static void %s(const Pre<T>& s, T mt, F&& body) {" % fname]
    checks = {}
    for r, c in _massless_lines(p):
        out_r, out_c = r >= nin, c >= nin
        rb = "(b%d ? %d : %d)" % (lev[r], 1 if out_r else 2, 2 if out_r else 1)
        cb = "(b%d ? %d : %d)" % (lev[c], 1 if out_c else 2, 2 if out_c else 1)
        checks.setdefault(max(lev[r], lev[c]), []).append("%s == %s" % (rb, cb))
    nodes = [n for n in p.nodes if not (n.kind == "ext" and min(n.legs) == root)]
    level_of = {id(n): max(lev[k] for k in n.legs) for n in nodes}
    ind = "    "
    for level in range(deep + 1):
        # the leg fixed by the helicity-reversal halving runs one helicity
        trips = 1 if order[level] == fixed else 2
        L.append(ind + "#pragma unroll 1")
        L.append(ind + "for (int b%d = 0; b%d < %d; ++b%d) {" % (level, level, trips, level))
        ind += "  "
        for cond in checks.get(level, []):
            L.append(ind + "if (%s) continue;" % cond)
        for n in nodes:
            if level_of[id(n)] != level or (level >= jit_from and n.kind != "ext"):
                continue
            if n.kind == "ext" and _linear(p, min(n.legs), fixed):
                L.append(ind + "const w4<T> v%d = wf_lin(s.x%d, b%d);" % (n.id, min(n.legs), level))
            elif n.kind == "ext":
                L.append(ind + "const w4<T> v%d = %s;" % (n.id, _ext_call(p, min(n.legs), "b%d" % level, nin)))
            else:
                L.append(ind + "const w4<T> v%d = %s;" % (n.id, _node_call(n, mslot, dslot, opq=opq)))
    # deepest loop: root wavefunctions, then amplitudes with just-in-time
    # sub-currents.  A massless-fermion root whose chirality partner is fixed
    # has one allowed helicity: evaluate only that one.
    root_checks = checks.get(N - 1, [])
    root_linear = not root_checks and _linear(p, root, fixed)
    if root_checks:
        assert len(root_checks) == 1
        bad0 = root_checks[0].replace("b%d" % (N - 1), "0")
        L.append(ind + "const int rbit = (%s) ? 1 : 0;" % bad0)
        L.append(ind + "const w4<T> r0 = %s;" % _ext_call(p, root, "rbit", nin))
        roots = (("r0", "J0"),)
        L.append(ind + "cx<T> J0[NFLOW];")
        L.append(ind + "for (int f = 0; f < NFLOW; ++f) J0[f] = czero<T>();")
    else:
        if root_linear:
            # a vector root takes its two real linear polarisations in place
            # of its helicities (same sum of |A|^2, cheaper amplitudes)
            L.append(ind + "const w4<T> r0 = wf_lin(s.x%d, 0);" % root)
            L.append(ind + "const w4<T> r1 = wf_lin(s.x%d, 1);" % root)
        else:
            L.append(ind + "const w4<T> r0 = %s;" % _ext_call(p, root, "0", nin))
            L.append(ind + "const w4<T> r1 = %s;" % _ext_call(p, root, "1", nin))
        roots = (("r0", "J0"), ("r1", "J1"))
        L.append(ind + "cx<T> J0[NFLOW], J1[NFLOW];")
        L.append(ind + "for (int f = 0; f < NFLOW; ++f) { J0[f] = czero<T>(); J1[f] = czero<T>(); }")
    lazy_den = "s.den"
    if jit_from < deep and KEEP_LAZY_IN_LOOP:
        # Sub-currents emitted lazily one or more levels above their own would
        # be hoisted back out of the deepest loop by loop-invariant code motion
        # (they do not depend on its helicity), undoing the trade of flops for
        # registers.  Their propagator factors are read through a copy that the
        # compiler must treat as changing every iteration.
        if opq:
            # each factor read through the barrier where it is used
            lazy_den = "@oval"
        else:
            lazy_den = "dl"
            L.append(ind + "T dl[NDEN];")
            L.append(ind + "#pragma unroll")
            L.append(ind + "for (int q = 0; q < NDEN; ++q) { dl[q] = s.den[q]; opaque(dl[q]); }")
    done = set()

    def need(n):
        """sub-currents still to emit for node n (children first)"""
        if n.kind == "ext" or id(n) in done or level_of[id(n)] < jit_from:
            return []
        out = []
        for c in n.children:
            out += need(c)
        done.add(id(n))
        return out + [n]

    # greedy amplitude order: next the one needing the fewest new sub-currents
    pending = list(p.amps)
    lazy_uses = {}
    users = {}
    if free_first:
        for b in pending:
            u = set()

            def walk(n):
                if n.kind == "ext" or level_of[id(n)] < jit_from:
                    return
                u.add(id(n))
                for c in n.children:
                    walk(c)
            for c in b.children[:-1]:
                walk(c)
            lazy_uses[id(b)] = u
            for x in u:
                users[x] = users.get(x, 0) + 1

    def frees(a):
        """sub-currents already evaluated whose last user a is"""
        return sum(1 for x in lazy_uses[id(a)] if x in done and users[x] == 1)
    nflow = len(p.flows)
    k = 0
    while pending:
        def newcount(a):
            seen = set()
            def cnt(n):
                if n.kind == "ext" or id(n) in done or level_of[id(n)] < jit_from or id(n) in seen:
                    return 0
                seen.add(id(n))
                return 1 + sum(cnt(c) for c in n.children)
            return sum(cnt(c) for c in a.children[:-1])
        if free_first:
            a = min(pending, key=lambda b: (newcount(b), -frees(b)))
            for x in lazy_uses[id(a)]:
                users[x] -= 1
        else:
            a = min(pending, key=newcount)
        pending.remove(a)
        for c in a.children[:-1]:
            for n in need(c):
                # a sub-current from above the deepest loop has only operands
                # that do not change in it: read them through the barrier too
                wrap = (lambda c: True) if opq and level_of[id(n)] < deep else None
                L.append(ind + "const w4<T> v%d = %s;" % (n.id, _node_call(n, mslot, dslot, lazy_den, opq, wrap)))
        ch = ["v%d" % c.id for c in a.children]
        kcur = None
        if root_linear and a.kind == "ffv_amp":
            # the fermion current once, contracted with both (real) root
            # vectors: cheaper than two full amplitudes
            kcur = "k%d" % k
            L.append(ind + "const w4<T> %s = ffv_cur(%s, %s);" % (kcur, ch[0], ch[1]))
        for rv, J in roots:
            av = "a%d_%s" % (k, rv)
            expr = "mdot(%s, %s)" % (kcur, rv) if kcur else _amp_call(a, ch, mslot, rv, opq)
            L.append(ind + "const cx<T> %s = %s;" % (av, expr))
            for f in range(nflow):
                c = _phase_coef(a.coef[f], a.phase, a.qfac)
                for line in _acc_code("%s[%d]" % (J, f), c, av):
                    L.append(ind + line)
        k += 1
    for _, J in roots:
        L.append(ind + "body(%s);" % J)
    for level in range(deep + 1):
        ind = ind[:-2]
        L.append(ind + "}")
    L.append("  }")
    return L


def emit_process(p):
    """HIP source for one process (a struct with static device functions)."""
    good = p.good_helicities()
    gs, ee = p.coupling_powers()
    nflow = len(p.flows)
    N = p.npart
    # the good set is closed under reversing every helicity, so in ascending
    # order its first half (leg 0 at bit 0) holds one of each pair
    assert sorted((1 << N) - 1 - h for h in good) == good
    assert all(h < (1 << (N - 1)) for h in good[:len(good) // 2])
    nin = len(p.incoming)
    # momentum slots: one per distinct leg set
    msets = []
    for n in p.nodes:
        if n.legs not in msets:
            msets.append(n.legs)
    root = p.npart - 1
    if frozenset([root]) not in msets:
        msets.append(frozenset([root]))
    mslot = {s: i for i, s in enumerate(msets)}
    # denominators: internal nodes by (leg set, mass)
    dens = []
    for n in p.nodes:
        if n.kind == "ext":
            continue
        key = (n.legs, n.mass if n.kind in ("ffv_col", "ffv_row") else "0")
        if key not in dens:
            dens.append(key)
    dslot = {k: i for i, k in enumerate(dens)}
    L = []
    nm = p.name
    L.append("// %s: %d diagrams, %d amplitude terms, %d off-shell currents, %d colour flows, %d/%d helicities"
             % (nm, p.ndiagrams, len(p.amps), len([n for n in p.nodes if n.kind != "ext"]), nflow,
                len(good), 1 << N))
    L.append("static __constant__ unsigned char %s_good[%d] = {%s};" % (nm, len(good), ", ".join(str(h) for h in good)))
    L.append("struct %s {" % nm)
    L.append("  static constexpr int NPART = %d, NIN = %d, NFLOW = %d, NHEL = %d, NGOOD = %d;" % (N, nin, nflow, 1 << N, len(good)))
    L.append("  static constexpr int NDIAG = %d, NTERM = %d, NCUR = %d, GS_POW = %d, E_POW = %d;"
             % (p.ndiagrams, len(p.amps), len([n for n in p.nodes if n.kind != "ext"]), gs, ee))
    L.append("  static constexpr double AVG = %.17g, IDENT = %.17g;" % (p.avg, p.ident))
    # helicity_sum (and the first NGOOD / HEL_SYM entries of good()) cover one
    # helicity of each pair (h, -h); callers multiply their sums by HEL_SYM
    L.append("  static constexpr int HEL_SYM = %d;" % (2 if HEL_SYMMETRY else 1))
    L.append("  static constexpr int WAVES_F32 = %d;   // waves per SIMD of the FP32 and pair kernels" % WAVES_F32.get(p.name, 1))
    L.append("  static constexpr int NMOM = %d, NDEN = %d;" % (len(msets), len(dens)))
    L.append("  static constexpr const char* NAME = \"%s\";" % nm)
    L.append("  static constexpr unsigned TOP_LEGS = 0x%x;   // bit k: leg k is a top quark"
             % sum(1 << k for k, x in enumerate(list(p.incoming) + list(p.outgoing)) if x in ("t", "t~")))
    L.append("  static constexpr unsigned LEP_LEGS = 0x%x;   // bit k: leg k is a charged lepton"
             % sum(1 << k for k, x in enumerate(list(p.incoming) + list(p.outgoing)) if x in LEPTONS))
    L.append("  __device__ static int good(int i) { return %s_good[i]; }" % nm)
    # per-event data
    L.append("  template <class T> struct Pre {")
    L.append("    r4<T> Q[NMOM];")
    L.append("    T den[NDEN];")
    for k in range(N):
        t = p.itype[k]
        if t in ("g", "a"):
            L.append("    vec_data<T> x%d;" % k)
        else:
            L.append("    ferm_data<T> x%d;" % k)
    L.append("  };")
    # prologue
    L.append("  // ov: exact values of up to two pairwise invariants (an FKS pair's,")
    L.append("  // from the radiation variables) that replace the ones formed here")
    L.append("  template <class T> NLO_HD static void prologue(const double (&p)[NPART][4], Pre<T>& s, double mt,")
    L.append("                                                const PairOv& ov = PairOv()) {")
    L.append("    double q[NPART][4];")
    for k in range(N):
        sgn = "" if k < nin else "-"
        L.append("    for (int m = 0; m < 4; ++m) q[%d][m] = %sp[%d][m];" % (k, sgn, k))
    # pairwise invariants 2 q_a.q_b of the legs that some denominator needs
    massive = [FERMIONS[flavour(p.itype[k])][0] == "MT" if p.itype[k] not in ("g", "a") else False
               for k in range(N)]
    full = frozenset(range(N))

    def small_side(S):
        C = full - S
        if len(C) < len(S) or (len(C) == len(S) and 0 in C):
            return C
        return S
    pairs = set()
    for (S, mass) in dens:
        Sp = sorted(small_side(S))
        pairs.update((a, b) for ia, a in enumerate(Sp) for b in Sp[ia + 1:])
    pairs = sorted(pairs)
    for a, b in pairs:
        L.append("    double s%d_%d = 2.0 * (q[%d][0] * q[%d][0] - q[%d][1] * q[%d][1] - q[%d][2] * q[%d][2] - "
                 "q[%d][3] * q[%d][3]);" % (a, b, a, b, a, b, a, b, a, b))
    if pairs:
        L.append("    if (ov.a0 >= 0) {")
        for a, b in pairs:
            L.append("      if (ov.a0 == %d && ov.b0 == %d) s%d_%d = ov.v0;" % (a, b, a, b))
            L.append("      if (ov.a1 == %d && ov.b1 == %d) s%d_%d = ov.v1;" % (a, b, a, b))
        L.append("    }")
    else:
        L.append("    (void)ov;")
    for k in range(N):
        t = p.itype[k]
        if t in ("g", "a"):
            L.append("    { vec_data<double> d; vec_setup(p[%d], d); s.x%d = cast<T>(d); }" % (k, k))
        else:
            mass = FERMIONS[flavour(t)][0]
            L.append("    { ferm_data<double> d; ferm_setup(p[%d], %s, d); s.x%d = cast<T>(d); }"
                     % (k, "mt" if mass == "MT" else "0.0", k))
    for S, i in mslot.items():
        legs = sorted(S)
        expr = " + ".join("q[%d][m]" % k for k in legs)
        L.append("    { double Q[4]; for (int m = 0; m < 4; ++m) Q[m] = %s;" % expr)
        L.append("      for (int m = 0; m < 4; ++m) s.Q[%d].v[m] = T(Q[m]);" % i)
        L.append("    }")
    # denominators P^2 - m^2 = sum_a m_a^2 + sum_{a<b} 2 q_a.q_b - m^2 over the
    # smaller of the line's leg set and its complement (external particles on
    # shell by definition): the near-singular invariant of a soft or
    # collinear emission is then one pairwise product, never a difference of
    # O(s) squares
    for (S, mass), j in dslot.items():
        Sp = sorted(small_side(S))
        terms = ["s%d_%d" % (a, b) for ia, a in enumerate(Sp) for b in Sp[ia + 1:]]
        cm = sum(1 for a in Sp if massive[a]) - (1 if mass == "MT" else 0)
        if cm:
            terms.append("%.1f * (mt * mt)" % cm)
        L.append("    s.den[%d] = T(1.0 / (%s));" % (j, " + ".join(terms)))
    L.append("  }")
    # exact power-of-two rescaling of the external wavefunctions (used by the
    # half-width kernels to keep intermediate values inside the FP16 range)
    L.append("  // multiply the external wavefunctions by powers of two with product 2^-b;")
    L.append("  // |M|^2 then scales by exactly 2^-2b")
    L.append("  template <class T> NLO_HD static void scale_legs(Pre<T>& s, int b) {")
    L.append("    const int q = b / NPART, r = b % NPART;")
    for k in range(N):
        L.append("    scale_leg(s.x%d, T(ldexpf(1.0f, -(q + (%d < r ? 1 : 0)))));" % (k, k))
    L.append("  }")
    # amplitudes for one helicity
    L.append("  // OVR >= 0: the external wavefunction of leg OVR is replaced by *ov")
    L.append("  template <class T, int OVR = -1> NLO_HD static void amplitudes(const Pre<T>& s, int h, T mt, cx<T> (&J)[NFLOW],")
    L.append("                                                       const w4<T>* ov = nullptr) {")
    L.append("    for (int f = 0; f < NFLOW; ++f) J[f] = czero<T>();")
    for n in p.nodes:
        v = "v%d" % n.id
        if n.kind == "ext":
            k = min(n.legs)
            bit = "((h >> %d) & 1)" % (N - 1 - k)
            t = n.ptype
            out = k >= nin
            if t in ("g", "a"):
                expr = "wf_eps(s.x%d, %s, %s)" % (k, bit, "true" if out else "false")
            elif is_fermion(t):
                # column spinor: incoming fermion u(p) or outgoing antifermion v(p)
                expr = "%s(s.x%d, %s)" % ("wf_v" if out else "wf_u", k, bit)
            else:
                # row spinor: outgoing fermion ubar(p) or incoming antifermion vbar(p)
                expr = "wf_bar(%s(s.x%d, %s))" % ("wf_u" if out else "wf_v", k, bit)
            L.append("    const w4<T> %s = (OVR == %d) ? *ov : %s;" % (v, k, expr))
            continue
        ch = ["v%d" % c.id for c in n.children]
        Q = "s.Q[%d]" % mslot[n.legs]
        dkey = (n.legs, n.mass if n.kind in ("ffv_col", "ffv_row") else "0")
        D = "s.den[%d]" % dslot[dkey]
        if n.kind == "ffv_vec":
            L.append("    const w4<T> %s = ffv_vec(%s, %s, %s);" % (v, ch[0], ch[1], D))
        elif n.kind in ("ffv_col", "ffv_row"):
            if n.mass == "MT":
                L.append("    const w4<T> %s = %s(%s, %s, %s, %s, mt);" % (v, n.kind, ch[0], ch[1], Q, D))
            else:
                L.append("    const w4<T> %s = %s0(%s, %s, %s, %s);" % (v, n.kind, ch[0], ch[1], Q, D))
        elif n.kind == "vvv_vec":
            QA = "s.Q[%d]" % mslot[n.children[0].legs]
            QB = "s.Q[%d]" % mslot[n.children[1].legs]
            L.append("    const w4<T> %s = vvv_vec(%s, %s, %s, %s, %s);" % (v, ch[0], QA, ch[1], QB, D))
        else:
            L.append("    const w4<T> %s = %s(%s, %s, %s, %s);" % (v, n.kind, ch[0], ch[1], ch[2], D))
    for i, a in enumerate(p.amps):
        ch = ["v%d" % c.id for c in a.children]
        av = "a%d" % i
        if a.kind == "ffv_amp":
            L.append("    const cx<T> %s = ffv_amp(%s, %s, %s);" % (av, ch[0], ch[2], ch[1]))
        elif a.kind == "ffv_amp_rootcol":
            L.append("    const cx<T> %s = ffv_amp(%s, %s, %s);" % (av, ch[0], ch[1], ch[2]))
        elif a.kind == "ffv_amp_rootrow":
            L.append("    const cx<T> %s = ffv_amp(%s, %s, %s);" % (av, ch[2], ch[1], ch[0]))
        elif a.kind == "vvv_amp":
            Qs = ["s.Q[%d]" % mslot[c.legs] for c in a.children]
            L.append("    const cx<T> %s = vvv_amp(%s, %s, %s, %s, %s, %s);" % (av, ch[0], Qs[0], ch[1], Qs[1], ch[2], Qs[2]))
        else:
            L.append("    const cx<T> %s = %s(%s, %s, %s, %s);" % (av, a.kind, ch[0], ch[1], ch[2], ch[3]))
        for f in range(nflow):
            c = _phase_coef(a.coef[f], a.phase, a.qfac)
            for line in _acc_code("J[%d]" % f, c, av):
                L.append("    " + line)
    L.append("  }")
    j_def = JIT_EXTRA_LEVELS.get(p.name, 0)
    j_f64 = JIT_EXTRA_LEVELS_FP64.get(p.name, j_def)
    if p.name in SCHEDULE_ALTS:
        # each lazy depth in use under its own name; schedule 0 takes each
        # precision's default depth, schedule 1 an alternative: no extra lazy
        # level where the default has some, else one
        alt = lambda d: 0 if d else 1
        depths = sorted({j_def, alt(j_def), j_f64, alt(j_f64)})
        for d in depths:
            L.extend(emit_nested(p, mslot, dslot, N, nin, d, "helicity_sum_lazy%d" % d,
                                 FP64_FREE_FIRST and d == j_f64 != j_def))
        L.append("  static constexpr int NSCHED = 2;")
        L.append("  template <int SCHED, class T, class F> NLO_HD static void helicity_sum_sched(const Pre<T>& s, T mt, "
                 "F&& body) {")
        L.append("    constexpr int def = std::is_same<T, double>::value ? %d : %d;" % (j_f64, j_def))
        if depths == [0, 1]:
            L.append("    if constexpr ((SCHED == 0 ? def : 1 - def) == 0) helicity_sum_lazy0(s, mt, body);")
            L.append("    else helicity_sum_lazy1(s, mt, body);")
        else:
            L.append("    constexpr int depth = SCHED == 0 ? def : (def ? 0 : 1);")
            for i, d in enumerate(depths):
                L.append("    %sif constexpr (depth == %d) helicity_sum_lazy%d(s, mt, body);"
                         % ("else " if i else "", d, d))
        L.append("  }")
    else:
        L.append("  static constexpr int NSCHED = 1;")
        L.append("  template <int SCHED, class T, class F> NLO_HD static void helicity_sum_sched(const Pre<T>& s, T mt, "
                 "F&& body) { helicity_sum(s, mt, body); }")
    j_bf16 = JIT_EXTRA_LEVELS_BF16.get(p.name, j_def)
    special = []
    if j_f64 != j_def:
        special.append(("double", j_f64, "helicity_sum_fp64", FP64_FREE_FIRST))
    if j_bf16 != j_def:
        special.append(("bf16x2", j_bf16, "helicity_sum_bf16", False))
    if not special:
        L.extend(emit_nested(p, mslot, dslot, N, nin))
    else:
        # the FP64 (and BF16) instantiations take their own lazy depths; the
        # others run the default schedule in helicity_sum itself
        for ty, d, name, ff in special:
            L.extend(emit_nested(p, mslot, dslot, N, nin, d, name, ff))
        main = emit_nested(p, mslot, dslot, N, nin, j_def)
        L.append(main[0])
        L.append(main[1])
        for ty, d, name, _ in special:
            L.append("    if constexpr (std::is_same<T, %s>::value) {" % ty)
            L.append("      %s(s, mt, body);" % name)
            L.append("      return;")
            L.append("    }")
        L.extend(main[2:])
    # colour sum: J^dagger C J = |L^T Re J|^2 + |L^T Im J|^2, C = L L^T
    Lc = cholesky_lower(p.colour_matrix)
    L.append("  // colour matrix (rows):")
    for row in p.colour_matrix:
        L.append("  //   " + " ".join("%9.5f" % x for x in row))
    L.append("  template <class T> NLO_HD static T colour_sum(const cx<T> (&J)[NFLOW]) {")
    L.append("    T m2 = T(0), y;")
    for part in ("r", "i"):
        for k in range(nflow):
            terms = ["T(%.17g) * J[%d].%s" % (Lc[j, k], j, part) for j in range(k, nflow) if abs(Lc[j, k]) > 1e-15]
            if not terms:
                continue
            L.append("    y = %s; m2 += y * y;" % " + ".join(terms))
    L.append("    return m2;")
    L.append("  }")
    # transposed Cholesky factor for the matrix-core colour contraction: LT[k][j] = L[j][k]
    if p.name in FKS_BORNS:
        L.extend(emit_colour_corr(p))
    L.append("  static constexpr float LT[%d][%d] = {%s};" % (
        nflow, nflow, ", ".join("{" + ", ".join("%.9ef" % Lc[j, k] for j in range(nflow)) + "}" for k in range(nflow))))
    L.append("};")
    return "\n".join(L)


VARIANTS = ("VAR_F64", "VAR_F32", "VAR_MFMA", "VAR_F16", "VAR_BF16", "VAR_F64_ALT", "VAR_F32_ALT")
ALT_VARIANTS = (5, 6)   # compiled only for SCHEDULE_ALTS; elsewhere the table repeats variants 0 and 1


def _write_if_changed(path, src):
    old = open(path).read() if os.path.exists(path) else None
    if old != src:
        with open(path, "w") as f:
            f.write(src)


# FKS sectors: (real process, Born process, I, J (-1: both beams), all FKS pairs of
# the real process, Born at the y -> -1 end when it differs from the one at y -> +1)
FKS_SECTORS = [
    ("ee_uug", "ee_uu", 4, 2, [(4, 2), (4, 3)], None),
    ("ee_uug", "ee_uu", 4, 3, [(4, 2), (4, 3)], None),
    ("gg_ttg", "gg_tt", 4, -1, [(4, -1)], None),
    ("uu_ttg", "uu_tt", 4, -1, [(4, -1)], None),
    ("ug_ttu", "gg_tt", 4, -1, [(4, -1)], "uu_tt"),
    ("gg_ttgg", "gg_ttg", 4, 5, [(4, 5), (5, 4), (4, -1), (5, -1)], None),
    ("gg_ttgg", "gg_ttg", 5, 4, [(4, 5), (5, 4), (4, -1), (5, -1)], None),
    ("gg_ttgg", "gg_ttg", 4, -1, [(4, 5), (5, 4), (4, -1), (5, -1)], None),
    ("gg_ttgg", "gg_ttg", 5, -1, [(4, 5), (5, 4), (4, -1), (5, -1)], None),
]


def sector_name(real, i, j):
    return "fks_%s_%d_%s" % (real, i, "0" if j < 0 else str(j))


def emit_sector(procs, real, born, i, j, pairs, bornm=None):
    R = procs[real]
    B = procs[born]
    nr, nb = R.npart, B.npart
    bmap = []
    b = 0
    for r in range(nr):
        if r == i:
            bmap.append(-1)
        else:
            bmap.append(b)
            b += 1
    gluon = [R.itype[r] == "g" for r in range(nr)]
    name = sector_name(real, i, j)
    L = ["struct %s {" % name,
         "  using Real = %s;" % real,
         "  using Born = %s;" % born,
         "  using BornM = %s;   // Born at the y -> -1 end" % (bornm or born),
         "  // FKS parton I is a quark: no soft singularity, and the incoming parton",
         "  // changes flavour at each collinear end (Born and BornM)",
         "  static constexpr bool QUARK_I = %s;" % ("true" if bornm else "false"),
         "  static constexpr int I = %d, J = %d, JB = %d, NR = %d, NB = %d, NPAIR = %d;"
         % (i, j, bmap[j] if j >= 0 else -1, nr, nb, len(pairs)),
         "  static constexpr int BMAP[NR] = {%s};" % ", ".join(str(x) for x in bmap),
         "  static constexpr int PI[NPAIR] = {%s};" % ", ".join(str(a) for a, _ in pairs),
         "  static constexpr int PJ[NPAIR] = {%s};" % ", ".join(str(c) for _, c in pairs),
         "  static constexpr bool GLUON[NR] = {%s};" % ", ".join("true" if g else "false" for g in gluon),
         "  static constexpr bool J_GLUON = %s;" % ("true" if j >= 0 and gluon[j] else "false"),
         "  static constexpr bool BEAM_GLUON0 = %s, BEAM_GLUON1 = %s;"
         % ("true" if B.itype[0] == "g" else "false", "true" if B.itype[1] == "g" else "false"),
         "};"]
    return name, "\n".join(L)


def generate(out_dir):
    """Write one header per process, one translation unit per (process,
    kernel variant) and an index consumed by the C ABI.  Returns the list of
    translation units."""
    procs = process_list()
    os.makedirs(out_dir, exist_ok=True)
    tus = []
    index = ["// GENERATED by codegen.py -- do not edit.", "#pragma once", '#include "../launch.hpp"',
             '#include "../fks.hpp"', "namespace nlo {"]
    for p in procs:
        p.enumerate()
        p.colour()
        incs = ["#include <type_traits>", '#include "../helas.hpp"']
        if JIT_EXTRA_LEVELS.get(p.name, 0) or p.name in SCHEDULE_ALTS or p.name in OPAQUE_MOMENTA:
            incs.append('#include "../opaque.hpp"')
        hdr = "\n".join(["// GENERATED by codegen.py -- do not edit.", "#pragma once"] + incs +
                         ["namespace nlo {", emit_process(p), "}  // namespace nlo", ""])
        _write_if_changed(os.path.join(out_dir, p.name + ".hpp"), hdr)
        for v, var in enumerate(VARIANTS):
            if v in ALT_VARIANTS and p.name not in SCHEDULE_ALTS:
                continue
            tu = "\n".join(["// GENERATED by codegen.py -- do not edit.", '#include "../kernels.hpp"',
                             '#include "%s.hpp"' % p.name, "namespace nlo {",
                             "hipError_t me2_%s_%d(const LaunchArgs& a) { return launch_me2<%s, %s>(a); }"
                             % (p.name, v, p.name, var), "}  // namespace nlo", ""])
            path = os.path.join(out_dir, "tu_%s_%d.hip" % (p.name, v))
            _write_if_changed(path, tu)
            tus.append(path)
            index.append("hipError_t me2_%s_%d(const LaunchArgs&);" % (p.name, v))
    index.append("constexpr int NPROC = %d;" % len(procs))
    index.append("static const ProcStatic PROC_STATIC[NPROC] = {")
    for p in procs:
        gs, ee = p.coupling_powers()
        tops = sum(1 << k for k, x in enumerate(list(p.incoming) + list(p.outgoing)) if x in ("t", "t~"))
        leps = sum(1 << k for k, x in enumerate(list(p.incoming) + list(p.outgoing)) if x in LEPTONS)
        index.append('  {"%s", %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %.17g, %.17g, %du, %du},' % (
            p.name, p.npart, len(p.incoming), len(p.flows), 1 << p.npart, len(p.good_helicities()), p.ndiagrams,
            len(p.amps), len([n for n in p.nodes if n.kind != "ext"]), gs, ee, p.avg, p.ident, tops, leps))
    index.append("};")
    index.append("static const me2_launcher ME2_LAUNCH[NPROC][NVAR] = {")
    for p in procs:
        index.append("  {%s}," % ", ".join("me2_%s_%d" % (p.name, v if (v not in ALT_VARIANTS or p.name in SCHEDULE_ALTS)
                                                             else v - 5) for v in range(len(VARIANTS))))
    index.append("};")
    # FKS sectors
    byname = {p.name: p for p in procs}
    index.append("struct FksSector {")
    index.append("  const char* name; int real, born, bornm, i, j;")
    index.append("  hipError_t (*map)(const FksArgs&, int, hipStream_t);")
    index.append("  hipError_t (*born_fn[2])(const FksArgs&, int, int, hipStream_t);   // [0] double, [1] float")
    index.append("  hipError_t (*cuts)(const FksCutArgs&, hipStream_t);")
    index.append("};")
    decl, rows = [], []
    pid = {p.name: k for k, p in enumerate(procs)}
    for real, born, i, j, pairs, bornm in FKS_SECTORS:
        name, struct = emit_sector(byname, real, born, i, j, pairs, bornm)
        incs = ['#include "%s.hpp"' % x for x in dict.fromkeys([real, born, bornm or born])]
        hdr = "\n".join(["// GENERATED by codegen.py -- do not edit.", "#pragma once"] + incs +
                         ["namespace nlo {", struct, "}  // namespace nlo", ""])
        _write_if_changed(os.path.join(out_dir, name + ".hpp"), hdr)
        for v, T in enumerate(("double", "float")):
            body = ['#include "../fks.hpp"', '#include "%s.hpp"' % name, "namespace nlo {"]
            if v == 0:
                body.append("hipError_t %s_map(const FksArgs& a, int block, hipStream_t st) { return launch_fks_map<%s>(a, block, st); }" % (name, name))
                body.append("hipError_t %s_cuts(const FksCutArgs& a, hipStream_t st) { return launch_fks_cuts<%s>(a, st); }" % (name, name))
            body.append("hipError_t %s_born%d(const FksArgs& a, int which, int block, hipStream_t st) { return launch_fks_born<%s, %s>(a, which, block, st); }" % (name, v, name, T))
            body.append("}  // namespace nlo")
            path = os.path.join(out_dir, "tu_%s_%d.hip" % (name, v))
            _write_if_changed(path, "\n".join(["// GENERATED by codegen.py -- do not edit."] + body + [""]))
            tus.append(path)
        decl.append("hipError_t %s_map(const FksArgs&, int, hipStream_t);" % name)
        decl.append("hipError_t %s_born0(const FksArgs&, int, int, hipStream_t);" % name)
        decl.append("hipError_t %s_born1(const FksArgs&, int, int, hipStream_t);" % name)
        decl.append("hipError_t %s_cuts(const FksCutArgs&, hipStream_t);" % name)
        rows.append('  {"%s", %d, %d, %d, %d, %d, %s_map, {%s_born0, %s_born1}, %s_cuts},' % (
            name, pid[real], pid[born], pid[bornm or born], i, j, name, name, name, name))
    index.extend(decl)
    index.append("constexpr int NFKS = %d;" % len(FKS_SECTORS))
    index.append("static const FksSector FKS_TABLE[NFKS] = {")
    index.extend(rows)
    index.append("};")
    index.append("}  // namespace nlo")
    _write_if_changed(os.path.join(out_dir, "index.hpp"), "\n".join(index) + "\n")
    stale = os.path.join(out_dir, "processes.hpp")
    if os.path.exists(stale):
        os.remove(stale)
    return tus

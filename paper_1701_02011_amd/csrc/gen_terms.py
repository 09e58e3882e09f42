#!/usr/bin/env python3
"""Generate the spin-integrated contraction table of the DSRG-MRPT3 hot path.

Run:  python paper_1701_02011_amd/csrc/gen_terms.py  (writes dsrg_terms.inc beside it)

What it derives (Sec. II-III):  the scalar, one- and two-body parts of the commutator
[X, T]_{1,2} of a Hermitian operator X (one- and two-body) with an excitation operator
T = T1 + T2, for operators normal ordered with respect to a multideterminantal
reference (MK-GNO).  The paper evaluates these commutators with the generalised Wick
theorem and does not reprint the term list (Sec. III); this script re-derives it.

1. Generalised Wick patterns of {X}{T}: pairwise contractions X-creator/T-annihilator
   (gamma) and X-annihilator/T-creator (eta), plus at most one density-cumulant group
   (lambda2 or lambda3) touching both operators.  In the commutator {X}{T} - {T}{X} every
   pattern with n pair contractions carries the weight
       prod g - (-1)^n prod (delta - g) = sum_{S proper subset} (-1)^|S| kappa_S delta_rest,
   with kappa = gammaA on eta pairs and etaA = 1 - gammaA on gamma pairs (both active-only),
   so patterns without pairs cancel and lambda4 never appears (it would need internal
   amplitudes, which are zero).
2. Terms equal by the tensors' symmetries are merged numerically (proportional values on
   random tensors that carry exactly those symmetries).
3. Each term is spin-integrated for restricted orbitals: spin blocks aa, ab, bb (and
   aaa, aab, abb, bbb for lambda3); other spin patterns map to these by index permutation
   and sign.  Antisymmetrised integrals become Coulomb blocks J[p,r,q,s] = (pr|qs) of the
   factorised integrals (Eq. int_fact): <pq||rs> = J[p,r,q,s] - J[p,s,q,r].
4. Products with identical factors are computed once and scattered to every output
   position (common-subexpression grouping).

Four uses are emitted:
  C0  the scalar <[X, T]> for X given by its de-excitation block (tensors E1, E2);
  W   the excitation block of [V, A]_{1,2} = [V,T] + [V,T]^+ for the two-body Hamiltonian V;
  Z   the excitation block of [Y, A]_{1,2} for the non-diagonal operator Y (Y1, Y2);
  R   the active block of [X, A]_{1,2} = [X,T] + [X,T]^+ for a Hermitian X given, as in C0,
      by its de-excitation block (outputs R1 [A][A], R2 [A]^4).  Every amplitude has a
      non-active index, which a contraction must remove when all output indices are
      active: a virtual one meets an annihilator of X, a core one a creator, so only the
      de-excitation block of X (creators in H, annihilators in P) enters.
Index spaces: C core, A active, V virtual, H = C+A, P = A+V, G all (orbital order
[C|A|V] makes each a contiguous range).  Storage (C-convention, excitation order):
T1/E1/Y1/O1 [P][H], T2/E2/Y2/O2 [P][P][H][H], gA/eA [A][A], L2 [A]^4, L3 [A]^6.
"""
from __future__ import annotations

import itertools
import os
import sys

import numpy as np

# ---------------------------------------------------------------------------
# 1. Wick patterns (spin-orbital)
# ---------------------------------------------------------------------------


def _parity(seq):
    inv = sum(1 for i in range(len(seq)) for j in range(i + 1, len(seq)) if seq[i] > seq[j])
    return -1 if inv % 2 else 1


class _Op:
    __slots__ = ("kind", "letter", "owner", "pos")

    def __init__(self, kind, letter, owner, pos):
        self.kind, self.letter, self.owner, self.pos = kind, letter, owner, pos


def _ops(rx, rt):
    if rx == 2:
        xs, xt = [("c", "p"), ("c", "q"), ("a", "s"), ("a", "r")], ("X", "pqrs", 0.25)
    else:
        xs, xt = [("c", "p"), ("a", "q")], ("X1", "pq", 1.0)
    if rt == 2:
        ts, tt = [("c", "A"), ("c", "B"), ("a", "J"), ("a", "I")], ("T", "ABIJ", 0.25)
    else:
        ts, tt = [("c", "A"), ("a", "I")], ("T1", "AI", 1.0)
    ops = [_Op(k, l, "X", i) for i, (k, l) in enumerate(xs)]
    ops += [_Op(k, l, "T", len(xs) + i) for i, (k, l) in enumerate(ts)]
    return ops, xt, tt


def wick_terms(rx, rt, max_out=2):
    """Plain-order terms (coef, [(tensor, letters)], out) of [X, T]."""
    ops, xt, tt = _ops(rx, rt)
    X = [o for o in ops if o.owner == "X"]
    T = [o for o in ops if o.owner == "T"]
    allpairs = ([(x, t) for x in X if x.kind == "c" for t in T if t.kind == "a"]
                + [(x, t) for x in X if x.kind == "a" for t in T if t.kind == "c"])
    terms = []
    for npair in range(1, len(ops) // 2 + 1):
        for pairs in itertools.combinations(allpairs, npair):
            used = [o.pos for pr in pairs for o in pr]
            if len(set(used)) != len(used):
                continue
            rest = [o for o in ops if o.pos not in used]
            groups = [None]
            for k in (2, 3):
                cs = [o for o in rest if o.kind == "c"]
                an = [o for o in rest if o.kind == "a"]
                for gc in itertools.combinations(cs, k):
                    for ga in itertools.combinations(an, k):
                        g = list(gc) + list(ga)
                        if len({o.owner for o in g}) == 2:
                            groups.append(g)
            for g in groups:
                gpos = set() if g is None else {o.pos for o in g}
                ext = [o for o in rest if o.pos not in gpos]
                nout = len(ext) // 2
                if nout > max_out or sum(1 for o in ext if o.kind == "c") != nout:
                    continue
                key = lambda o: (o.owner != "X", o.pos)
                target, lam = [], None
                if g is not None:
                    gc = sorted([o for o in g if o.kind == "c"], key=key)
                    ga = sorted([o for o in g if o.kind == "a"], key=key)
                    target += gc + ga
                    lam = ("L%d" % len(gc), "".join(o.letter for o in gc + ga))
                for (x, t) in pairs:
                    target += [x, t]
                ec = sorted([o for o in ext if o.kind == "c"], key=key)
                ea = sorted([o for o in ext if o.kind == "a"], key=key)
                target += ec + ea
                sign = _parity([o.pos for o in target])
                out = "".join(o.letter for o in ec + ea)
                for S in itertools.product((0, 1), repeat=len(pairs)):
                    if sum(S) == len(pairs):
                        continue
                    coef = xt[2] * tt[2] * sign * (-1) ** sum(S)
                    fac = [(xt[0], xt[1]), (tt[0], tt[1])] + ([lam] if lam else [])
                    merge = {}
                    for (x, t), k in zip(pairs, S):
                        if k:
                            fac.append(("eA", x.letter + t.letter) if x.kind == "c"
                                       else ("gA", t.letter + x.letter))
                        else:
                            merge[t.letter] = x.letter
                    fac = [(nm, "".join(merge.get(c, c) for c in ls)) for nm, ls in fac]
                    terms.append((coef, fac, "".join(merge.get(c, c) for c in out)))
    return terms


# ---------------------------------------------------------------------------
# random tensors carrying exactly the symmetries of the real ones
# ---------------------------------------------------------------------------


def _asym(x, pairs):
    for (i, j) in pairs:
        ax = list(range(x.ndim))
        ax[i], ax[j] = ax[j], ax[i]
        x = x - x.transpose(ax)
    return x


def _herm(x, k):
    ax = list(range(k, 2 * k)) + list(range(k))
    return x + x.transpose(ax)


def _asym3(x, off):
    for perm in [(1, 0, 2), (0, 2, 1)]:
        pass
    y = np.zeros_like(x)
    for pm in itertools.permutations(range(3)):
        ax = list(range(x.ndim))
        for i in range(3):
            ax[off + i] = off + pm[i]
        y = y + _parity(pm) * x.transpose(ax)
    return y


def _so_env(rng, nC=1, nA=3, nV=2):
    """Spin-orbital dense random tensors (space-major spin-orbital layout)."""
    n = 2 * (nC + nA + nV)
    A = slice(2 * nC, 2 * (nC + nA))
    P = np.zeros(n, bool); P[2 * nC:] = True
    H = np.zeros(n, bool); H[:2 * (nC + nA)] = True
    Am = np.zeros(n, bool); Am[A] = True
    X = _herm(_asym(rng.standard_normal((n,) * 4), [(0, 1), (2, 3)]), 2)
    X1 = rng.standard_normal((n, n)); X1 = X1 + X1.T
    m2 = (P[:, None, None, None] & P[None, :, None, None] & H[None, None, :, None] & H[None, None, None, :]
          & ~(Am[:, None, None, None] & Am[None, :, None, None] & Am[None, None, :, None] & Am[None, None, None, :]))
    m1 = P[:, None] & H[None, :] & ~(Am[:, None] & Am[None, :])
    T = np.where(m2, _asym(rng.standard_normal((n,) * 4), [(0, 1), (2, 3)]), 0.0)
    T1 = np.where(m1, rng.standard_normal((n, n)), 0.0)
    na = 2 * nA
    g = rng.standard_normal((na, na)); g = g + g.T
    e = rng.standard_normal((na, na)); e = e + e.T
    l2 = _herm(_asym(rng.standard_normal((na,) * 4), [(0, 1), (2, 3)]), 2)
    l3 = _herm(_asym3(_asym3(rng.standard_normal((na,) * 6), 0), 3), 3)
    gA = np.zeros((n, n)); gA[A, A] = g
    eA = np.zeros((n, n)); eA[A, A] = e
    L2 = np.zeros((n,) * 4); L2[A, A, A, A] = l2
    L3 = np.zeros((n,) * 6); L3[A, A, A, A, A, A] = l3
    # plain-order cumulants used by the Wick terms
    return dict(X=X, X1=X1, T=T, T1=T1, gA=gA, eA=eA,
                L2=L2.transpose(0, 1, 3, 2), L3=L3.transpose(0, 1, 2, 5, 4, 3))


def _c_from_plain(V):
    Kc = V.transpose(0, 1, 3, 2)
    return Kc - Kc.transpose(1, 0, 2, 3) - Kc.transpose(0, 1, 3, 2) + Kc.transpose(1, 0, 3, 2)


def _eval_term(term, env):
    coef, fac, out = term
    spec = ",".join(l for _, l in fac) + "->" + out
    V = np.einsum(spec, *[env[nm] for nm, _ in fac], optimize="greedy")
    if len(out) == 4:
        return _c_from_plain(np.asarray(V)).ravel()
    return np.atleast_1d(np.asarray(V, dtype=float)).ravel()


def _merge(items, fingerprint, key):
    """Sum coefficients of items whose fingerprints are proportional (same key)."""
    groups = []
    for it in items:
        V = fingerprint(it)
        nrm = np.linalg.norm(V)
        if nrm < 1e-12:
            continue
        for g in groups:
            if g[3] != key(it):
                continue
            ratio = V @ g[2] / (g[2] @ g[2])
            if np.linalg.norm(V - ratio * g[2]) < 1e-10 * nrm:
                g[1] += it[0] * ratio
                break
        else:
            groups.append([it, it[0], V, key(it)])
    out = []
    for it, c, V, k in groups:
        if abs(c) > 1e-12:
            c64 = round(c * 64) / 64
            out.append((c64 if abs(c64 - c) < 1e-8 else c,) + tuple(it[1:]))
    return out


def spin_orbital_terms(seed=7):
    rng = np.random.default_rng(seed)
    envs = [_so_env(rng) for _ in range(3)]
    res = {}
    for rx in (1, 2):
        for rt in (1, 2):
            raw = wick_terms(rx, rt)
            fp = lambda t: np.concatenate([_eval_term(t, e) for e in envs])
            res[(rx, rt)] = _merge(raw, fp, key=lambda t: len(t[2]))
    return res


# ---------------------------------------------------------------------------
# 3. spin integration into spatial blocks
# ---------------------------------------------------------------------------
SETS = {"C": {"C"}, "A": {"A"}, "V": {"V"}, "H": {"C", "A"}, "P": {"A", "V"}, "G": {"C", "A", "V"}}
CODE = {frozenset(v): k for k, v in SETS.items()}
STORAGE = {"T1": "PH", "T2": "PPHH", "E1": "PH", "E2": "PPHH", "Y1": "PH", "Y2": "PPHH",
           "L2": "AAAA", "L3": "AAAAAA", "gA": "AA", "eA": "AA", "v": "GGGG", "J": "GGGG",
           "O1": "PH", "O2": "PPHH", "R1": "AA", "R2": "AAAA"}


def _inter(a, b):
    s = SETS[a] & SETS[b]
    return CODE.get(frozenset(s)) if s else None


class _Fac:
    def __init__(self, tensor, letters, rank):
        self.tensor, self.letters, self.rank = tensor, letters, rank


def _resolve(rank, up, lo):
    if sorted(up) != sorted(lo):
        return None
    pu = sorted(range(rank), key=lambda i: (up[i], i))
    pl = sorted(range(rank), key=lambda i: (lo[i], i))
    return "".join("ab"[up[i]] for i in pu), pu, pl, _parity(pu) * _parity(pl)


def _spin_terms(coef, facs, ospins):
    letters = sorted({l for f in facs for l in f.letters})
    internal = [l for l in letters if l not in ospins]
    out = []
    for sp in itertools.product((0, 1), repeat=len(internal)):
        spin = dict(ospins)
        spin.update(zip(internal, sp))
        c, rf = coef, []
        for f in facs:
            k = f.rank
            r = _resolve(k, [spin[l] for l in f.letters[:k]], [spin[l] for l in f.letters[k:]])
            if r is None:
                break
            name, pu, pl, sg = r
            rf.append((f.tensor, name, "".join(f.letters[i] for i in pu)
                       + "".join(f.letters[k + i] for i in pl)))
            c *= sg
        else:
            out.append((c, rf))
    return out


def _xpieces(use):
    if use in ("C0", "R"):
        return {1: [lambda L: _Fac("E1", L[1] + L[0], 1)],
                2: [lambda L: _Fac("E2", L[2] + L[3] + L[0] + L[1], 2)]}
    if use == "W":
        return {1: [], 2: [lambda L: _Fac("v", L, 2)]}
    return {1: [lambda L: _Fac("Y1", L, 1), lambda L: _Fac("Y1", L[1] + L[0], 1)],
            2: [lambda L: _Fac("Y2", L, 2), lambda L: _Fac("Y2", L[2] + L[3] + L[0] + L[1], 2)]}


def _conv(nm, ls):
    if nm == "T1":
        return _Fac("T1", ls, 1)
    if nm == "T":
        return _Fac("T2", ls, 2)
    if nm == "L2":
        return _Fac("L2", ls[0] + ls[1] + ls[3] + ls[2], 2)
    if nm == "L3":
        return _Fac("L3", ls[:3] + ls[5] + ls[4] + ls[3], 3)
    return _Fac(nm, ls, 1)


def _out_entries(out, rank, blk, active=False):
    """Output positions of a term's plain-order output letters: the term itself ("exc") or
    its adjoint ("dex"), over the excitation block (creators P, annihilators H) or, with
    active=True, over the active block (every letter A)."""
    if rank == 0:
        return [("", 1.0, {})]
    up, lo = ("A", "A") if active else ("P", "H")
    if rank == 1:
        c, a = out
        return [(c + a, 1.0, {c: up, a: lo})] if blk == "exc" else [(a + c, 1.0, {c: lo, a: up})]
    c1, c2, a1, a2 = out
    if blk == "exc":
        req, (x1, x2, y1, y2) = {c1: up, c2: up, a1: lo, a2: lo}, (c1, c2, a2, a1)
    else:
        req, (x1, x2, y1, y2) = {c1: lo, c2: lo, a1: up, a2: up}, (a2, a1, c1, c2)
    return [(x1 + x2 + y1 + y2, 1.0, req), (x2 + x1 + y1 + y2, -1.0, req),
            (x1 + x2 + y2 + y1, -1.0, req), (x2 + x1 + y2 + y1, 1.0, req)]


OUT_BLOCKS = {0: [("", ())], 1: [("a", (0, 0)), ("b", (1, 1))],
              2: [("aa", (0, 0, 0, 0)), ("ab", (0, 1, 0, 1)), ("bb", (1, 1, 1, 1))]}


def spatial_entries(so_terms, use, ranks):
    """(coef, out_tensor, out_block, out_letters, [(tensor, block, letters)], spaces)."""
    ents = []
    xp = _xpieces(use)
    active = use == "R"
    otn = "R" if active else "O"
    for (rx, rt), terms in so_terms.items():
        for coef, fac, out in terms:
            rank = len(out) // 2
            if rank not in ranks:
                continue
            for xb in xp[rx]:
                for blk in (("exc", "dex") if rank else ("exc",)):
                    for olets, osign, req in _out_entries(out, rank, blk, active):
                        facs = [xb(ls) if nm in ("X", "X1") else _conv(nm, ls) for nm, ls in fac]
                        sp = dict(req)
                        ok = True
                        for f in facs:
                            for ax, l in zip(STORAGE[f.tensor], f.letters):
                                new = _inter(sp.get(l, "G"), ax)
                                if new is None:
                                    ok = False
                                sp[l] = new
                        if not ok:
                            continue
                        if rank:
                            for ax, l in zip(STORAGE["%s%d" % (otn, rank)], olets):
                                new = _inter(sp[l], ax)
                                if new is None:
                                    ok = False
                                sp[l] = new
                            if not ok:
                                continue
                        for bname, bsp in OUT_BLOCKS[rank]:
                            for c, rf in _spin_terms(coef * osign, facs, dict(zip(olets, bsp))):
                                # antisymmetrised integrals -> Coulomb blocks J[p,r,q,s]
                                pieces = [(c, [])]
                                for (tn, b, ls) in rf:
                                    if tn != "v":
                                        pieces = [(cc, fs + [(tn, b, ls)]) for cc, fs in pieces]
                                        continue
                                    p, q, r, s = ls
                                    if b == "ab":
                                        pieces = [(cc, fs + [("J", "", p + r + q + s)]) for cc, fs in pieces]
                                    else:
                                        pieces = ([(cc, fs + [("J", "", p + r + q + s)]) for cc, fs in pieces]
                                                  + [(-cc, fs + [("J", "", p + s + q + r)]) for cc, fs in pieces])
                                for cc, fs in pieces:
                                    ents.append((cc, "%s%d" % (otn, rank) if rank else "E", bname,
                                                 olets, fs, dict(sp)))
    return ents


# spatial random environment for merging -------------------------------------
class _Dims:
    def __init__(self, nC, nA, nV):
        self.off = {"C": 0, "A": nC, "V": nC + nA, "H": 0, "P": nC, "G": 0}
        self.len = {"C": nC, "A": nA, "V": nV, "H": nC + nA, "P": nA + nV, "G": nC + nA + nV}

    def rng(self, ls, ax):
        o = self.off[ls] - self.off[ax]
        return slice(o, o + self.len[ls])


def _sp_env(rng, nC=2, nA=3, nV=3, M=7):
    nH, nP, N = nC + nA, nA + nV, nC + nA + nV
    inAP = np.arange(nP) < nA
    inAH = np.arange(nH) >= nC
    i2 = inAP[:, None, None, None] & inAP[None, :, None, None] & inAH[None, None, :, None] & inAH[None, None, None, :]
    i1 = inAP[:, None] & inAH[None, :]

    def t2(zero):
        d = {"aa": _asym(rng.standard_normal((nP, nP, nH, nH)), [(0, 1), (2, 3)]),
             "bb": _asym(rng.standard_normal((nP, nP, nH, nH)), [(0, 1), (2, 3)]),
             "ab": rng.standard_normal((nP, nP, nH, nH))}
        return {k: np.where(i2, 0.0, x) for k, x in d.items()} if zero else d

    def t1(zero):
        d = {k: rng.standard_normal((nP, nH)) for k in "ab"}
        return {k: np.where(i1, 0.0, x) for k, x in d.items()} if zero else d
    sym = lambda x: x + x.T
    l2 = {"aa": _herm(_asym(rng.standard_normal((nA,) * 4), [(0, 1), (2, 3)]), 2),
          "bb": _herm(_asym(rng.standard_normal((nA,) * 4), [(0, 1), (2, 3)]), 2),
          "ab": _herm(rng.standard_normal((nA,) * 4), 2)}
    a3 = lambda: _asym3(_asym3(rng.standard_normal((nA,) * 6), 0), 3)

    def aab():
        x = _asym(rng.standard_normal((nA,) * 6), [(0, 1), (3, 4)])
        return _herm(x, 3)

    def abb():
        x = _asym(rng.standard_normal((nA,) * 6), [(1, 2), (4, 5)])
        return _herm(x, 3)
    l3 = {"aaa": _herm(a3(), 3), "bbb": _herm(a3(), 3), "aab": aab(), "abb": abb()}
    B = rng.standard_normal((M, N, N)); B = B + B.transpose(0, 2, 1)
    tens = dict(T1=t1(True), T2=t2(True), E1=t1(False), E2=t2(False), Y1=t1(True), Y2=t2(True),
                L2=l2, L3=l3, gA={k: sym(rng.standard_normal((nA, nA))) for k in "ab"},
                eA={k: sym(rng.standard_normal((nA, nA))) for k in "ab"})
    return _Dims(nC, nA, nV), B, tens


def _jblock(d, B, ls, sp):
    R = [slice(d.off[sp[l]], d.off[sp[l]] + d.len[sp[l]]) for l in ls]
    return np.einsum("Qpr,Qqs->prqs", B[:, R[0], R[1]], B[:, R[2], R[3]])


def eval_entry(ent, d, B, tens):
    coef, ot, ob, ol, facs, sp = ent
    ops, specs = [], []
    for (tn, blk, ls) in facs:
        if tn == "J":
            ops.append(_jblock(d, B, ls, sp))
        else:
            sl = tuple(d.rng(sp[l], ax) for l, ax in zip(ls, STORAGE[tn]))
            ops.append(tens[tn][blk][sl])
        specs.append(ls)
    return np.einsum(",".join(specs) + "->" + ol, *ops, optimize="greedy")


def merge_spatial(ents, seed=11):
    rng = np.random.default_rng(seed)
    envs = [_sp_env(rng) for _ in range(3)]

    def fp(ent):
        vals = []
        for d, B, tens in envs:
            val = eval_entry(ent, d, B, tens)
            ot, ol, sp = ent[1], ent[3], ent[5]
            if ot == "E":
                vals.append(np.atleast_1d(float(val)))
            else:
                full = np.zeros(tuple(d.len[ax] for ax in STORAGE[ot]))
                full[tuple(d.rng(sp[l], ax) for l, ax in zip(ol, STORAGE[ot]))] = val
                vals.append(full.ravel())
        return np.concatenate(vals)
    return _merge(ents, fp, key=lambda e: (e[1], e[2]))


# ---------------------------------------------------------------------------
# 4. common subexpressions and emission
# ---------------------------------------------------------------------------
def group_products(ents):
    """products: (factors, spaces, result letters, [(coef, out, block, out letters)])."""
    prods = {}
    order = []
    for coef, ot, ob, ol, facs, sp in ents:
        res = "".join(sorted(ol))
        key = (tuple(facs), tuple(sorted(sp.items())), res)
        if key not in prods:
            prods[key] = []
            order.append(key)
        prods[key].append((coef, ot, ob, ol))
    return [(list(k[0]), dict(k[1]), k[2], prods[k]) for k in order]


def emit(tables, path):
    lines = []
    for use, prods in tables.items():
        lines.append("U %s %d" % (use, len(prods)))
        for facs, sp, res, scat in prods:
            fs = " ".join("%s.%s:%s" % (tn, blk or "-", ls) for tn, blk, ls in facs)
            spc = " ".join("%s=%s" % (l, sp[l]) for l in sorted(sp))
            lines.append("P %d %s | %s | %s" % (len(facs), fs, spc, res or "-"))
            for coef, ot, ob, ol in scat:
                lines.append("S %.17g %s.%s:%s" % (coef, ot, ob or "-", ol or "-"))
    body = "\n".join(lines) + "\n"
    with open(path, "w") as f:
        f.write("// Generated by gen_terms.py: spin-integrated contraction table of the\n"
                "// DSRG-MRPT3 commutators [X, T]_{1,2} (see that script for the derivation).\n"
                "// Format: 'U use nprod', then per product 'P nfac tensor.block:letters ... |\n"
                "// letter=space ... | result letters' followed by 'S coef out.block:letters' lines.\n")
        f.write("static const char kDsrgTermTable[] =\n")
        for ln in body.splitlines():
            f.write('  "%s\\n"\n' % ln)
        f.write(";\n")


def build_tables():
    so = spin_orbital_terms()
    tables = {}
    for use, ranks in (("C0", (0,)), ("W", (1, 2)), ("Z", (1, 2)), ("R", (1, 2))):
        tables[use] = group_products(merge_spatial(spatial_entries(so, use, ranks)))
    return so, tables


def main():
    so, tables = build_tables()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dsrg_terms.inc")
    emit(tables, out)
    for use, prods in tables.items():
        print(use, "products:", len(prods), "scatters:", sum(len(p[3]) for p in prods))


if __name__ == "__main__":
    main()

"""Commutators of operators normal ordered with respect to a multideterminantal
reference (oracle; FP64).

The MR-DSRG evaluates commutators with the Mukherjee-Kutzelnigg generalised Wick
theorem and keeps the scalar, one- and two-body parts (the "1,2" truncation,
Sec. II.A, Eq. exactBCH and the text after it).  This engine reaches the same
unique decomposition by a route that needs no hand-derived term list:

1. an operator given in MK-GNO form is rewritten in true-vacuum order using the
   reference densities (a normal-ordered string equals the bare string minus all
   its internal contractions, each weighted by the density of the removed indices);
2. the commutator of the two bare operators is taken with the canonical
   anticommutation relation a_p a+_q = delta_pq - a+_q a_p only (rank <= 3);
3. the bare result is rewritten in MK-GNO form again (each removed index set is
   weighted by the full reference density of those indices), and the GNO
   three-body part is dropped.

Operators are held in *plain order*: ``(k0, K1, K2)`` means
    k0 + sum K1[p,q] {a+_p a_q} + sum K2[p,q,r,s] {a+_p a+_q a_r a_s}
(no 1/4 and no antisymmetry assumed).  ``to_plain`` / ``to_c`` convert from / to
the paper's antisymmetrised convention X2[p,q,r,s] * 1/4 {a+_p a+_q a_s a_r}.

Only output blocks that the caller requests are formed; every tensor is dense
over the spin-orbital range G of ``spaces.Spaces``.

Parity: pinned by ``hilbert`` (bare commutators and GNO projections against
matrices in the full Fock space) on micro inputs.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .spaces import Densities

EIN = dict(optimize="greedy")


def to_plain(k0, X1, X2):
    """C-convention (X1, X2 with 1/4) -> plain-order operator."""
    K2 = None if X2 is None else 0.25 * X2.transpose(0, 1, 3, 2)
    return (float(k0), X1, K2)


def c_from_plain2(K2):
    """Plain two-body coefficients -> antisymmetrised C-convention tensor."""
    Kc = K2.transpose(0, 1, 3, 2)
    return Kc - Kc.transpose(1, 0, 2, 3) - Kc.transpose(0, 1, 3, 2) + Kc.transpose(1, 0, 3, 2)


# ---------------------------------------------------------------------------
# Term lists: a tensor contribution R[out] = coef * sum prod_k F_k[letters_k]
# ---------------------------------------------------------------------------
class Term:
    __slots__ = ("coef", "factors", "out")

    def __init__(self, coef: float, factors: List[Tuple[np.ndarray, str]], out: str):
        self.coef = coef
        self.factors = factors
        self.out = out


def _slice_factor(T, letters, ranges):
    return T[tuple(ranges.get(l, slice(None)) for l in letters)]


def _eval(terms: Sequence[Term], out_map: Dict[str, str], extra: List[Tuple[np.ndarray, str]],
          out_letters: str, ranges: Dict[str, slice], sign_coef: float = 1.0):
    """Sum over terms of coef * einsum(factors (+ extra), renamed by out_map) -> out_letters."""
    acc = None
    for t in terms:
        ops, specs = [], []
        for (T, lets) in t.factors:
            lets2 = "".join(out_map.get(l, l) for l in lets)
            ops.append(_slice_factor(T, lets2, ranges))
            specs.append(lets2)
        for (T, lets) in extra:
            ops.append(_slice_factor(T, lets, ranges))
            specs.append(lets)
        spec = ",".join(specs) + "->" + out_letters
        val = np.einsum(spec, *ops, **EIN) * (t.coef * sign_coef)
        acc = val if acc is None else acc + val
    return acc


# ---------------------------------------------------------------------------
# GNO -> bare
# ---------------------------------------------------------------------------
def gno_to_bare(op, dens: Densities):
    """(k0, K1, K2) in MK-GNO form -> same operator in true-vacuum order."""
    k0, K1, K2 = op
    g = dens.gamma
    H = slice(0, dens.D1.shape[0])
    n = g.shape[0]
    B1 = np.zeros((n, n)) if K1 is None else K1.copy()
    b0 = k0
    if K1 is not None:
        b0 -= float(np.einsum("pq,pq->", K1[H, H], dens.D1))
    if K2 is not None:
        gH = dens.D1
        # {a+p a+q a_r a_s} = a+p a+q a_r a_s + g_pr a+q a_s - g_ps a+q a_r - g_qr a+p a_s
        #                     + g_qs a+p a_r + 2 (g_ps g_qr - g_pr g_qs) - D2[p,q,r,s]
        B1 += np.einsum("pxry,pr->xy", K2[H, :, H, :], gH, **EIN)
        B1 -= np.einsum("pxys,ps->xy", K2[H, :, :, H], gH, **EIN)
        B1 -= np.einsum("xqry,qr->xy", K2[:, H, H, :], gH, **EIN)
        B1 += np.einsum("xqys,qs->xy", K2[:, H, :, H], gH, **EIN)
        KH = K2[H, H, H, H]
        b0 += 2.0 * float(np.einsum("pqrs,ps,qr->", KH, gH, gH, **EIN)
                          - np.einsum("pqrs,pr,qs->", KH, gH, gH, **EIN))
        b0 -= float(np.einsum("pqrs,pqrs->", KH, dens.D2p))
    return (b0, B1, K2)


# ---------------------------------------------------------------------------
# Bare commutator -> lists of bare terms of rank 1, 2 and 3
# ---------------------------------------------------------------------------
def bare_commutator_terms(Xb, Yb):
    """[X, Y] for bare operators of rank <= 2.  Returns (R1 terms, R2 terms, R3 terms)
    with letters in plain order: R1 'cd', R2 'abcd' (a+a a+b a_c a_d),
    R3 'abcdef' (a+a a+b a+c a_d a_e a_f)."""
    _, X1, X2 = Xb
    _, Y1, Y2 = Yb
    R1: List[Term] = []
    R2: List[Term] = []
    R3: List[Term] = []

    def one_one(K1, L1, sgn):
        # a+p a_q a+t a_u = d_qt a+p a_u - a+p a+t a_q a_u; two-body parts cancel.
        R1.append(Term(sgn, [(K1, "aq"), (L1, "qb")], "ab"))

    def one_two(K1, L2, sgn):
        # [K1, L2]: K1 L2 gives d_qt a+p a+u a_v a_w - d_qu a+p a+t a_v a_w (+3-body, cancels)
        #           L2 K1 gives d_wp a+t a+u a_v a_q - d_vp a+t a+u a_w a_q
        R2.append(Term(sgn, [(K1, "aq"), (L2, "qbcd")], "abcd"))
        R2.append(Term(-sgn, [(K1, "aq"), (L2, "bqcd")], "abcd"))
        R2.append(Term(-sgn, [(L2, "abcp"), (K1, "pd")], "abcd"))
        R2.append(Term(sgn, [(L2, "abpc"), (K1, "pd")], "abcd"))

    def two_two(K2, L2, sgn):
        # a_r a_s a+t a+u = a+t a+u a_r a_s + d_st d_ru - d_rt d_su - d_st a+u a_r
        #                   + d_rt a+u a_s + d_su a+t a_r - d_ru a+t a_s
        R2.append(Term(sgn, [(K2, "abrs"), (L2, "srcd")], "abcd"))
        R2.append(Term(-sgn, [(K2, "abrs"), (L2, "rscd")], "abcd"))
        # three-body pieces, out letters a+a a+b a+c a_d a_e a_f
        R3.append(Term(-sgn, [(K2, "abds"), (L2, "scef")], "abcdef"))   # -d_st: u->c, r->d
        R3.append(Term(sgn, [(K2, "abrd"), (L2, "rcef")], "abcdef"))    # +d_rt: u->c, s->d
        R3.append(Term(sgn, [(K2, "abds"), (L2, "csef")], "abcdef"))    # +d_su: t->c, r->d
        R3.append(Term(-sgn, [(K2, "abrd"), (L2, "cref")], "abcdef"))   # -d_ru: t->c, s->d

    if X1 is not None and Y1 is not None:
        one_one(X1, Y1, 1.0)
        one_one(Y1, X1, -1.0)
    if X1 is not None and Y2 is not None:
        one_two(X1, Y2, 1.0)
    if X2 is not None and Y1 is not None:
        one_two(Y1, X2, -1.0)
    if X2 is not None and Y2 is not None:
        two_two(X2, Y2, 1.0)
        two_two(Y2, X2, -1.0)
    return R1, R2, R3


# ---------------------------------------------------------------------------
# Bare -> GNO projections
# ---------------------------------------------------------------------------
def _project(R1, R2, R3, dens: Densities, want0: bool, want1, want2, G: slice, H: slice):
    """GNO scalar, one-body block want1=(rc, rd) and two-body block want2=(rc1,rc2,rd1,rd2)
    of the bare operator R1 + R2 + R3 (plain order)."""
    gH = dens.D1
    out0 = 0.0
    out1 = None
    out2 = None
    if want2 is not None:
        rc1, rc2, rd1, rd2 = want2
        # rank-2 bare part maps to itself
        out2 = _eval(R2, {}, [], "abcd", dict(a=rc1, b=rc2, c=rd1, d=rd2))
        # rank-3: sum_{i,j} (-1)^(i+j) gamma[c_i, d_j] {rest}
        cre, ann = "abc", "def"
        for i in range(3):
            for j in range(3):
                ci, dj = cre[i], ann[j]
                rest_c = [x for x in cre if x != ci]
                rest_a = [x for x in ann if x != dj]
                # rename: remaining creators -> w,x ; annihilators -> y,z (output order)
                ren = {rest_c[0]: "w", rest_c[1]: "x", rest_a[0]: "y", rest_a[1]: "z",
                       ci: "m", dj: "n"}
                rng = dict(w=rc1, x=rc2, y=rd1, z=rd2, m=H, n=H)
                val = _eval(R3, ren, [(gH, "mn")], "wxyz", rng, (-1.0) ** (i + j))
                if val is not None:
                    out2 = val if out2 is None else out2 + val
    if want1 is not None:
        rc, rd = want1
        out1 = _eval(R1, {"a": "c", "b": "d"}, [], "cd", dict(c=rc, d=rd))
        # rank-2: a+a a+b a_c a_d -> -g_ac{b d} + g_ad{b c} + g_bc{a d} - g_bd{a c}
        for (ci, dj, sgn) in (("a", "c", -1.0), ("a", "d", 1.0), ("b", "c", 1.0), ("b", "d", -1.0)):
            rc_ = [x for x in "ab" if x != ci][0]
            ra_ = [x for x in "cd" if x != dj][0]
            ren = {rc_: "x", ra_: "y", ci: "m", dj: "n"}
            val = _eval(R2, ren, [(gH, "mn")], "xy", dict(x=rc, y=rd, m=H, n=H), sgn)
            if val is not None:
                out1 = val if out1 is None else out1 + val
        # rank-3: sum (-1)^(i1+i2+j1+j2) D2[c_i1, c_i2, d_j1, d_j2] {c_k d_l}
        cre, ann = "abc", "def"
        for (i1, i2) in itertools.combinations(range(3), 2):
            for (j1, j2) in itertools.combinations(range(3), 2):
                k = [x for x in range(3) if x not in (i1, i2)][0]
                l = [x for x in range(3) if x not in (j1, j2)][0]
                ren = {cre[i1]: "m", cre[i2]: "n", ann[j1]: "o", ann[j2]: "q",
                       cre[k]: "x", ann[l]: "y"}
                sgn = (-1.0) ** ((i1 + 1) + (i2 + 1) + (j1 + 1) + (j2 + 1))
                val = _eval(R3, ren, [(dens.D2p, "mnoq")], "xy",
                            dict(x=rc, y=rd, m=H, n=H, o=H, q=H), sgn)
                if val is not None:
                    out1 = val if out1 is None else out1 + val
    if want0:
        v = _eval(R1, {"a": "c", "b": "d"}, [(gH, "cd")], "", dict(c=H, d=H))
        out0 += 0.0 if v is None else float(v)
        v = _eval(R2, {}, [(dens.D2p, "abcd")], "", dict(a=H, b=H, c=H, d=H))
        out0 += 0.0 if v is None else float(v)
        if R3:
            v = _eval(R3, {}, [(dens.D3p, "abcdef")], "",
                      dict(a=H, b=H, c=H, d=H, e=H, f=H))
            out0 += float(v)
    return out0, out1, out2


def commutator(X, Y, dens: Densities, want0: bool = False, want1=None, want2=None):
    """GNO parts of [X, Y]_{1,2}; X, Y plain-order GNO operators (k0, K1, K2).

    Returns (scalar, one-body block, two-body block) in plain order; blocks not
    requested are None.  The scalar of a commutator is its reference expectation
    value.
    """
    n = dens.gamma.shape[0]
    G = slice(0, n)
    H = slice(0, dens.D1.shape[0])
    Xb = gno_to_bare(X, dens)
    Yb = gno_to_bare(Y, dens)
    R1, R2, R3 = bare_commutator_terms(Xb, Yb)
    return _project(R1, R2, R3, dens, want0, want1, want2, G, H)

"""DSRG-MRPT3 energies at the medium and large workloads (oracle level O2; FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The steps and readings are those of ``dsrg.run`` (Sec. II.B in the paper's order), with
every tensor held in the block form of ``blocked`` and the antisymmetrised integrals
built on the fly from the factorised tensor (Sec. III, Eq. int_fact), the (VV|VV)-type
blocks in batches of their first index (Eq. scaling_problem).  Two steps use closed forms
that the oracle's pins establish for the generic engine: the two-body part of
[H(0), A(1)] is -D * A(1) element by element (H(0) is a diagonal one-body operator, so
its commutator scales each normal-ordered two-body string by the difference of orbital
energies), and the densities of rank two and three enter through their cumulant
expansions.  ``tests/test_oracle_df.py`` compares every intermediate with ``dsrg.run`` on
micro and tiny inputs and the energies with the stored small-workload values.

Parity: pinned to ``dsrg`` (the generic engine) element by element.
"""
from __future__ import annotations

import dataclasses
import itertools
import time
from typing import Optional

import numpy as np

from .blocked import (BT, DFV, SETS, BlockDensities, Orb, Sum, beval, commutator, spin_ok, view)
from .dsrg import regulariser, source_factor, so_fock_offdiag
from .gno import Term
from .spaces import Spaces, build_densities


@dataclasses.dataclass
class Result:
    e2: float
    e3: float
    e3_a: float
    e3_b: float
    seconds: dict
    t1: Optional[BT] = None      # [P][H] blocks
    t2: Optional[BT] = None      # [P][P][H][H] blocks (C-convention)
    o1_1: Optional[BT] = None
    o1_2: Optional[BT] = None
    z1_1: Optional[BT] = None
    z1_2: Optional[BT] = None
    u1: Optional[BT] = None
    u2: Optional[BT] = None


def _eps_blocks(orb: Orb, eps: np.ndarray):
    return [eps[orb.spatial(b)] for b in range(6)]


def _D2(eb, key):
    a, b, i, j = key
    return (eb[i][None, None, :, None] + eb[j][None, None, None, :]
            - eb[a][:, None, None, None] - eb[b][None, :, None, None])


def _D1(eb, key):
    a, i = key
    return eb[i][None, :] - eb[a][:, None]


def _internal(key):
    return all(b in SETS["A"] for b in key)


def _plain2(X2, coef=1.0):
    """C-convention two-body X2 -> plain-order coefficients 1/4 X2[p,q,s,r] (as gno.to_plain)."""
    return view(X2, (0, 1, 3, 2), 0.25 * coef)


def _hermitian2(X2):
    """An excitation-block two-body tensor [P][P][H][H] plus its adjoint block [H][H][P][P];
    on the all-active blocks, which both contain, the adjoint's value (as in ``dsrg.run``,
    which writes the adjoint block last)."""
    outer = BT(X2.orb, 4, {k: b for k, b in X2.blocks.items() if not _internal(k)})
    return Sum([outer, view(X2, (2, 3, 0, 1))])


def _hermitian1(orb, X1):
    """One-body [P][H] plus its adjoint [H][P]; the adjoint's value on the active-active
    blocks (as ``_hermitian2``)."""
    out = BT(orb, 2)
    for (a, i), blk in X1.blocks.items():
        if not _internal((a, i)):
            out.add((a, i), blk)
        out.add((i, a), blk.T)
    return out


def _antihermitian1(orb, X1):
    """X - X^T of a one-body excitation tensor, as explicit blocks."""
    out = BT(orb, 2)
    for (a, i), blk in X1.blocks.items():
        out.add((a, i), blk)
        out.add((i, a), -blk.T)
    return out


def _c_from_plain2(orb, K):
    """Plain-order two-body coefficients -> antisymmetrised C-convention tensor (as
    gno.c_from_plain2), materialised block by block."""
    Kc = view(K, (0, 1, 3, 2))
    terms = [(1.0, Kc), (-1.0, view(Kc, (1, 0, 2, 3))), (-1.0, view(Kc, (0, 1, 3, 2))),
             (1.0, view(Kc, (1, 0, 3, 2)))]
    keys = set()
    for c, T in terms:
        for k in K.blocks:
            # keys of the view T that exist: apply the inverse of T's axes to k
            kk = [None] * 4
            for pos, ax in enumerate(T.axes):
                kk[pos] = k[ax]
            keys.add(tuple(kk))
    out = BT(orb, 4)
    for k in keys:
        acc = None
        for c, T in terms:
            if T.has(k):
                x = c * T.coef * T.get(k)
                acc = x if acc is None else acc + x
        if acc is not None:
            out.blocks[k] = np.ascontiguousarray(acc)
    return out


def _amplitudes(orb, eb, s, gam, f_exc: Optional[BT], v_exc, keys2):
    """t[a,b,i,j] = v R_s(D) and t[a,i] = [f + sum_{u,x in A} (e_x - e_u) t[a,x,i,u] g[x,u]]
    R_s(D) on the excitation blocks, internal amplitudes zero (Eqs. T1_1st, T2_1st,
    T1_2nd, T2_2nd).  v_exc(key) returns the driving block."""
    T2 = BT(orb, 4)
    for key in keys2:
        if _internal(key):
            continue
        v = v_exc(key)
        if v is None:
            continue
        T2.blocks[key] = v * regulariser(s, _D2(eb, key))
    # singles coupling: W[x,u] = (e_x - e_u) g[x,u] over the active blocks
    W = BT(orb, 2)
    for b in SETS["A"]:
        if orb.n[b] and (b, b) in gam.blocks:
            W.blocks[(b, b)] = (eb[b][:, None] - eb[b][None, :]) * gam.blocks[(b, b)]
    coup = BT(orb, 2)
    if W.blocks:
        beval(orb, [Term(1.0, [(T2, "axiu"), (W, "xu")], "ai")], "ai",
              dict(a=SETS["P"], i=SETS["H"], x=SETS["A"], u=SETS["A"]), out=coup)
    T1 = BT(orb, 2)
    for a in SETS["P"]:
        for i in SETS["H"]:
            if SPIN_OF(a) != SPIN_OF(i) or orb.n[a] == 0 or orb.n[i] == 0 or _internal((a, i)):
                continue
            src = np.zeros(orb.shape((a, i)))
            if f_exc is not None and (a, i) in f_exc.blocks:
                src = src + f_exc.blocks[(a, i)]
            if (a, i) in coup.blocks:
                src = src + coup.blocks[(a, i)]
            T1.blocks[(a, i)] = src * regulariser(s, _D1(eb, (a, i)))
    return T1, T2


def SPIN_OF(b):
    return b % 2


def _exc_keys2(orb):
    out = []
    for key in itertools.product(SETS["P"], SETS["P"], SETS["H"], SETS["H"]):
        if spin_ok(key) and all(orb.n[b] for b in key):
            out.append(key)
    return out


def run(prob, keep: bool = False, log=None, through: str = "e3") -> Result:
    """E^(2), E^(3) of the unrelaxed DSRG-MRPT3 (Eqs. E(2), E(3), E_unrelaxed).

    through = "first_order" stops after the first-order amplitudes (step a2) and "e2" after
    E^(2) (step a3); the later fields are then NaN.  Stage wall times are in .seconds."""
    if through not in ("first_order", "e2", "e3"):
        raise ValueError("through must be 'first_order', 'e2' or 'e3'")
    nan = float("nan")
    say = log or (lambda *a: None)
    t0 = time.time()
    secs = {}
    sp = Spaces(prob.n_core, prob.n_active, prob.n_virtual)
    orb = Orb(prob.n_core, prob.n_active, prob.n_virtual)
    s = prob.s
    H, P, G = SETS["H"], SETS["P"], SETS["G"]
    # step a0: densities and cumulants (the active-space arrays only)
    d0 = build_densities(sp, prob.gamma1, prob.gamma2, prob.gamma3, with_D3=False)
    A = sp.A
    dens = BlockDensities(orb, d0.gamma[A, A], d0.L2, d0.L3)
    del d0
    eb = _eps_blocks(orb, np.asarray(prob.eps, dtype=np.float64))
    F0 = BT(orb, 2)
    for b in G:
        if orb.n[b]:
            F0.blocks[(b, b)] = np.diag(eb[b])
    F0op = (0.0, F0, None)
    # step a1: antisymmetrised integrals, built on demand (Eq. int_fact)
    v = DFV(orb, np.asarray(prob.B, dtype=np.float64))
    f_off = getattr(prob, "f_offdiag", None)
    f1 = BT.from_dense(orb, so_fock_offdiag(sp, f_off), "GG") if f_off is not None else BT(orb, 2)
    f_exc = BT(orb, 2, {k: b for k, b in f1.blocks.items() if k[0] in P and k[1] in H})
    keys2 = _exc_keys2(orb)
    # step a2: first-order amplitudes (Eqs. T1_1st, T2_1st)
    t1, t2 = _amplitudes(orb, eb, s, dens.gamma, f_exc, lambda k: v.get(k), keys2)
    secs["first_order"] = time.time() - t0
    say("first order %.1fs" % secs["first_order"])
    if through == "first_order":
        return Result(nan, nan, nan, nan, secs, t1=t1, t2=t2)
    a1_1 = _antihermitian1(orb, t1)
    a1_2p = Sum([view(t2, (0, 1, 3, 2), 0.25), view(t2, (2, 3, 1, 0), -0.25)])   # plain order
    A1 = (0.0, a1_1, a1_2p)
    # Y1 = [H(0), A(1)]: one-body part from the engine, two-body part -D * A(1)
    _, y1_1, _ = commutator(orb, F0op, (0.0, a1_1, a1_2p), dens, want1="GG")
    y1_2 = BT(orb, 4)
    for key, blk in t2.blocks.items():
        y1_2.blocks[key] = -_D2(eb, key) * blk
    Y2h = _hermitian2(y1_2)
    ht1_1 = BT(orb, 2)
    for k, b in f1.blocks.items():
        ht1_1.add(k, 2.0 * b)
    for k, b in y1_1.blocks.items():
        ht1_1.add(k, b)
    Ht1 = (0.0, ht1_1, Sum([_plain2(v, 2.0), _plain2(Y2h)]))   # H~(1) = 2 H(1) + Y1
    T1op = (0.0, t1, _plain2(t2))
    # step a3: E(2) = <[H~(1), T(1)]>
    e2, _, _ = commutator(orb, Ht1, T1op, dens, want0=True)
    secs["e2"] = time.time() - t0
    say("E2 %.12g  %.1fs" % (e2, secs["e2"]))
    if through == "e2":
        return Result(float(e2), nan, nan, nan, secs, t1=t1, t2=t2)
    # steps a4-a5: O1 = [H~(1), A(1)]_{1,2}, excitation blocks (Eq. Hbar_2nd)
    _, o1_1, o1_2p = commutator(orb, Ht1, A1, dens, want1="PH", want2="PPHH")
    o1_2 = _c_from_plain2(orb, o1_2p)
    del o1_2p
    secs["o1"] = time.time() - t0
    say("O1 %.1fs" % secs["o1"])
    # step a6: Z1 = [Y1, A(1)]_{1,2}
    Y1op = (0.0, y1_1, _plain2(Y2h))
    _, z1_1, z1_2p = commutator(orb, Y1op, A1, dens, want1="PH", want2="PPHH")
    z1_2 = _c_from_plain2(orb, z1_2p)
    del z1_2p
    secs["z1"] = time.time() - t0
    say("Z1 %.1fs" % secs["z1"])
    # second-order amplitudes from the excitation blocks of O1 / 2 (Eqs. T1_2nd, T2_2nd)
    f2 = BT(orb, 2, {k: 0.5 * b for k, b in o1_1.blocks.items()})
    u1, u2 = _amplitudes(orb, eb, s, dens.gamma, f2,
                         lambda k: 0.5 * o1_2.blocks[k] if k in o1_2.blocks else None, keys2)
    # step a7: H~(2)_{1,2} = [H(0), A(2)] + O1 / 2 - Z1 / 6 on the excitation blocks
    a2_1 = _antihermitian1(orb, u1)
    a2_2p = Sum([view(u2, (0, 1, 3, 2), 0.25), view(u2, (2, 3, 1, 0), -0.25)])
    _, w1, w2p = commutator(orb, F0op, (0.0, a2_1, a2_2p), dens, want1="PH", want2="PPHH")
    w2 = _c_from_plain2(orb, w2p)
    h2_1 = BT(orb, 2)
    for src, c in ((w1, 1.0), (o1_1, 0.5), (z1_1, -1.0 / 6.0)):
        for k, b in src.blocks.items():
            h2_1.add(k, c * b)
    h2_2 = BT(orb, 4)
    for src, c in ((w2, 1.0), (o1_2, 0.5), (z1_2, -1.0 / 6.0)):
        for k, b in src.blocks.items():
            h2_2.add(k, c * b)
    del w2
    Ht2 = (0.0, _hermitian1(orb, h2_1), _plain2(_hermitian2(h2_2)))
    T2op = (0.0, u1, _plain2(u2))
    # E(3) = <[H~(1), T(2)]> + <[H~(2)_{1,2}, T(1)]>  (Eq. E(3))
    e3a, _, _ = commutator(orb, Ht1, T2op, dens, want0=True)
    secs["e3_a"] = time.time() - t0
    say("E3a %.12g  %.1fs" % (e3a, secs["e3_a"]))
    e3b, _, _ = commutator(orb, Ht2, T1op, dens, want0=True)
    secs["total"] = time.time() - t0
    say("E3b %.12g  %.1fs" % (e3b, secs["total"]))
    r = Result(float(e2), float(e3a + e3b), float(e3a), float(e3b), secs)
    if keep:
        r.t1, r.t2, r.o1_1, r.o1_2, r.z1_1, r.z1_2, r.u1, r.u2 = t1, t2, o1_1, o1_2, z1_1, z1_2, u1, u2
    return r

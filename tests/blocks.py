"""Map the oracle's spin-orbital tensors to the library's spin-block layout (tests only).

Oracle layout: spin orbitals ordered [core a | core b | active a | active b | virtual a |
virtual b].  Library layout: spatial hole indices H = [core | active] and particle indices
P = [active | virtual], one array per spin block.
"""
import numpy as np


def so_index_P(nC, nA, nV, spin):
    x = np.arange(nA + nV)
    return np.where(x < nA, 2 * nC + spin * nA + x, 2 * (nC + nA) + spin * nV + (x - nA))


def so_index_H(nC, nA, spin):
    i = np.arange(nC + nA)
    return np.where(i < nC, spin * nC + i, 2 * nC + spin * nA + (i - nC))


def one_body(T, nC, nA, nV, offP=0, offH=0):
    """[2][nP][nH] from a spin-orbital [..][..] array whose rows start at spin-orbital offP
    and columns at offH (0 for full arrays)."""
    out = np.zeros((2, nA + nV, nC + nA))
    for s in (0, 1):
        P = so_index_P(nC, nA, nV, s) - offP
        H = so_index_H(nC, nA, s) - offH
        out[s] = T[np.ix_(P, H)]
    return out


def two_body(T, nC, nA, nV, offP=0, offH=0):
    """[3][nP][nP][nH][nH] (aa, ab, bb) from a spin-orbital [P][P][H][H]-indexable array."""
    out = np.zeros((3, nA + nV, nA + nV, nC + nA, nC + nA))
    for b, (s1, s2) in enumerate(((0, 0), (0, 1), (1, 1))):
        P1 = so_index_P(nC, nA, nV, s1) - offP
        P2 = so_index_P(nC, nA, nV, s2) - offP
        H1 = so_index_H(nC, nA, s1) - offH
        H2 = so_index_H(nC, nA, s2) - offH
        out[b] = T[np.ix_(P1, P2, H1, H2)]
    return out


def oracle_blocks(r, p):
    """Spin blocks of the oracle intermediates that the library exports."""
    nC, nA, nV = p.n_core, p.n_active, p.n_virtual
    offP, offH = 2 * nC, 0
    o1 = one_body(r.o1_1, nC, nA, nV, offP, offH)
    o2 = two_body(r.o1_2, nC, nA, nV, offP, offH)
    z1 = one_body(r.z1_1, nC, nA, nV, offP, offH)
    z2 = two_body(r.z1_2, nC, nA, nV, offP, offH)
    return dict(t1=one_body(r.t1_1, nC, nA, nV), t2=two_body(r.t2_1, nC, nA, nV),
                w1=0.5 * (o1 - z1), w2=0.5 * (o2 - z2), z1=z1, z2=z2,
                u1=one_body(r.t1_2, nC, nA, nV), u2=two_body(r.t2_2, nC, nA, nV))

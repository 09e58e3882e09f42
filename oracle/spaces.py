"""Spin-orbital spaces, reference densities and cumulants (oracle; FP64).

Spin-orbital layout: space-major, then spin, then spatial index:
    [core a | core b | active a | active b | virtual a | virtual b]
so every orbital space of Sec. II.A is a contiguous range:
    C = [0, 2nC), A = [2nC, 2nH), V = [2nH, 2N), H = C u A = [0, 2nH),
    P = A u V = [2nC, 2N), G = [0, 2N).

Tensor conventions (C-convention, as in the paper):
    one-body    X1[p, q]        multiplies {a+_p a_q}
    two-body    X2[p, q, r, s]  multiplies 1/4 {a+_p a+_q a_s a_r}  (antisymmetric in pq and in rs)
    densities   gamma[p, q] = <a+_p a_q>,  G2[p,q,r,s] = <a+_p a+_q a_s a_r>,
                G3[p,q,r,s,t,u] = <a+_p a+_q a+_r a_u a_t a_s>.
The cumulants follow the Kutzelnigg-Mukherjee definitions that the MK-GNO Wick
theorem rests on (Sec. II.A): lambda2 = G2 - det(gamma gamma), and
lambda3 = G3 - det(gamma gamma gamma) - (antisymmetrised gamma x lambda2).

Parity: pinned by ``hilbert`` (densities of the full reference over the hole space
against brute-force expectation values, zero cumulants for a single determinant).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


def perm_sign(p) -> float:
    inv = sum(1 for i in range(len(p)) for j in range(i + 1, len(p)) if p[i] > p[j])
    return -1.0 if inv % 2 else 1.0


@dataclass
class Spaces:
    nC: int
    nA: int
    nV: int

    @property
    def N(self):
        return self.nC + self.nA + self.nV

    @property
    def nH(self):
        return self.nC + self.nA

    @property
    def G(self):
        return slice(0, 2 * self.N)

    @property
    def C(self):
        return slice(0, 2 * self.nC)

    @property
    def A(self):
        return slice(2 * self.nC, 2 * self.nH)

    @property
    def V(self):
        return slice(2 * self.nH, 2 * self.N)

    @property
    def H(self):
        return slice(0, 2 * self.nH)

    @property
    def P(self):
        return slice(2 * self.nC, 2 * self.N)

    def so_index(self):
        """(spatial index, spin) of every spin orbital, spin 0 = alpha."""
        spatial, spin = [], []
        for off, n in ((0, self.nC), (self.nC, self.nA), (self.nH, self.nV)):
            for s in (0, 1):
                spatial.extend(range(off, off + n))
                spin.extend([s] * n)
        return np.array(spatial), np.array(spin)

    def active_so(self):
        """Spin-orbital indices of the active alpha and beta orbitals."""
        a0 = 2 * self.nC
        return np.arange(a0, a0 + self.nA), np.arange(a0 + self.nA, a0 + 2 * self.nA)


def so_energies(sp: Spaces, eps: np.ndarray) -> np.ndarray:
    spatial, _ = sp.so_index()
    return eps[spatial].copy()


def so_integrals(sp: Spaces, B: np.ndarray) -> np.ndarray:
    """Antisymmetrised <pq||rs> = (pr|qs) d(sp,sr) d(sq,ss) - (ps|qr) d(sp,ss) d(sq,sr),
    with chemists' (pq|rs) = sum_Q B^Q_pq B^Q_rs (Sec. III, Eq. int_fact)."""
    spatial, spin = sp.so_index()
    Bs = B[:, spatial][:, :, spatial]                      # [Q][p][q] over spin orbitals
    same = (spin[:, None] == spin[None, :]).astype(float)  # d(sigma_p, sigma_q)
    J = np.einsum("Qpr,Qqs->pqrs", Bs, Bs, optimize=True)  # (pr|qs) at [p,q,r,s]
    J *= same[:, None, :, None] * same[None, :, None, :]
    return J - J.transpose(0, 1, 3, 2)


def expand_rdm_blocks(nA: int, g1, g2, g3):
    """Spin-block densities (input layout) -> spin-orbital tensors over the 2 nA
    active spin orbitals ordered [alpha | beta]."""
    n2 = 2 * nA
    sl = (slice(0, nA), slice(nA, 2 * nA))
    G1 = np.zeros((n2, n2))
    G1[sl[0], sl[0]] = g1[0]
    G1[sl[1], sl[1]] = g1[1]

    def fill(rank, canon):
        T = np.zeros((n2,) * (2 * rank))
        for up in itertools.product((0, 1), repeat=rank):
            for lo in itertools.product((0, 1), repeat=rank):
                if sorted(up) != sorted(lo):
                    continue
                nb = sum(up)
                if canon.get(nb) is None:
                    continue
                # permutations that sort spins (alpha first, stable)
                pu = sorted(range(rank), key=lambda i: (up[i], i))
                pl = sorted(range(rank), key=lambda i: (lo[i], i))
                sign = perm_sign(pu) * perm_sign(pl)
                block = canon[nb]                      # indices in canonical spin order
                # target axis k (upper) corresponds to canonical axis pu.index(k)
                inv_u = [pu.index(k) for k in range(rank)]
                inv_l = [pl.index(k) for k in range(rank)]
                axes = inv_u + [rank + i for i in inv_l]
                idx = tuple(sl[up[k]] for k in range(rank)) + tuple(sl[lo[k]] for k in range(rank))
                T[idx] = sign * np.transpose(block, axes)
        return T

    G2 = fill(2, {0: g2[0], 1: g2[1], 2: g2[2]})
    G3 = fill(3, {0: g3[0], 1: g3[1], 2: g3[2], 3: g3[3]}) if g3 is not None else None
    return G1, G2, G3


def det2(a, b):
    """Antisymmetrised product a^p_r b^q_s - a^p_s b^q_r as a [p,q,r,s] tensor."""
    return np.einsum("pr,qs->pqrs", a, b) - np.einsum("ps,qr->pqrs", a, b)


def det3(g):
    out = 0.0
    for pm in itertools.permutations(range(3)):
        lo = "stu"
        spec = "p%s,q%s,r%s->pqrstu" % (lo[pm[0]], lo[pm[1]], lo[pm[2]])
        out = out + perm_sign(pm) * np.einsum(spec, g, g, g)
    return out


def g_times_l2(g, l2):
    """sum_{i,j} (-1)^(i+j) g[P_i, S_j] l2[P\\i, S\\j] over upper P=(p,q,r), lower S=(s,t,u)."""
    up, lo = "pqr", "stu"
    out = 0.0
    for i in range(3):
        for j in range(3):
            ru = up[:i] + up[i + 1:]
            rl = lo[:j] + lo[j + 1:]
            spec = "%s%s,%s%s->pqrstu" % (up[i], lo[j], ru, rl)
            out = out + (-1.0) ** (i + j) * np.einsum(spec, g, l2)
    return out


def cumulants(G1, G2, G3):
    """Step a0: lambda2 and lambda3 from the active 1-, 2-, 3-body densities."""
    L2 = G2 - det2(G1, G1)
    L3 = None
    if G3 is not None:
        L3 = G3 - det3(G1) - g_times_l2(G1, L2)
    return L2, L3


@dataclass
class Densities:
    """Reference densities in the spin-orbital layout of ``Spaces``.

    gamma, eta: [2N][2N] over G.  L2: [2nA]^4 and L3: [2nA]^6 over A.
    D1, D2p, D3p: *plain-order* densities over H (used by the commutator engine):
        D1[p,q] = <a+_p a_q>, D2p[p,q,r,s] = <a+_p a+_q a_r a_s>,
        D3p[p,q,r,s,t,u] = <a+_p a+_q a+_r a_s a_t a_u>.
    """
    sp: Spaces
    gamma: np.ndarray
    eta: np.ndarray
    L2: np.ndarray
    L3: np.ndarray
    D1: np.ndarray
    D2p: np.ndarray
    D3p: np.ndarray


def build_densities(sp: Spaces, g1, g2, g3, with_D3: bool = True) -> Densities:
    n2N = 2 * sp.N
    gam = np.zeros((n2N, n2N))
    gam[sp.C, sp.C] = np.eye(2 * sp.nC)
    nA2 = 2 * sp.nA
    if sp.nA > 0:
        G1a, G2a, G3a = expand_rdm_blocks(sp.nA, g1, g2, g3)
        gam[sp.A, sp.A] = G1a
        L2a, L3a = cumulants(G1a, G2a, G3a)
        if L3a is None:
            L3a = np.zeros((nA2,) * 6)
    else:
        L2a = np.zeros((0,) * 4)
        L3a = np.zeros((0,) * 6)
    eta = np.eye(n2N) - gam
    # full densities over the hole space, from the cumulant expansion
    nH2 = 2 * sp.nH
    gH = gam[:nH2, :nH2]
    L2H = np.zeros((nH2,) * 4)
    a = slice(2 * sp.nC, nH2)
    L2H[a, a, a, a] = L2a
    G2H = det2(gH, gH) + L2H                       # C-convention <a+p a+q a_s a_r>
    D2p = G2H.transpose(0, 1, 3, 2).copy()         # plain <a+p a+q a_r a_s>
    D3p = None
    if with_D3:
        L3H = np.zeros((nH2,) * 6)
        L3H[a, a, a, a, a, a] = L3a
        G3H = det3(gH) + g_times_l2(gH, L2H) + L3H
        D3p = G3H.transpose(0, 1, 2, 5, 4, 3).copy()
    return Densities(sp, gam, eta, L2a, L3a, gH.copy(), D2p, D3p)

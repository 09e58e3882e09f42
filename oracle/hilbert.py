"""Brute force in the full Fock space for micro inputs (oracle; FP64).

Everything here is computed from matrices of creation/annihilation operators on
the 2^(2N) occupation-number states, with no normal ordering and no term lists:
expectation values, exact commutators of operator matrices and Rayleigh-Schroedinger
perturbation theory in the determinant basis.  It pins the engine in ``gno`` and
the densities in ``spaces`` on inputs with at most 12-14 spin orbitals.

Spin-orbital ordering and signs follow ``spaces.Spaces``: bit k of a state is spin
orbital k, and a+_k carries (-1)^(number of occupied orbitals below k).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sps

from paper_1701_02011_amd.synth import det_strings

from .spaces import Spaces


class FockSpace:
    def __init__(self, n_so: int):
        if n_so > 14:
            raise ValueError("brute force limited to 14 spin orbitals")
        self.n = n_so
        self.dim = 1 << n_so
        states = np.arange(self.dim)
        self.ann = []
        for k in range(n_so):
            occ = (states >> k) & 1
            src = states[occ == 1]
            dst = src ^ (1 << k)
            below = np.array([bin(s & ((1 << k) - 1)).count("1") for s in src])
            sgn = np.where(below % 2 == 1, -1.0, 1.0)
            self.ann.append(sps.csr_matrix((sgn, (dst, src)), shape=(self.dim, self.dim)))
        self.cre = [a.T.tocsr() for a in self.ann]

    def number_sector(self, n_el: int):
        states = np.arange(self.dim)
        pc = np.array([bin(s).count("1") for s in states])
        return np.nonzero(pc == n_el)[0]

    # -- operators from plain-order tensors --------------------------------
    def apply(self, op, vec):
        """Apply (k0, K1, K2[, K3]) in *bare* plain order to one vector."""
        k0, K1, K2 = op[0], op[1], op[2]
        K3 = op[3] if len(op) > 3 else None
        n = self.n
        out = k0 * vec
        if K1 is not None:
            A1 = np.array([self.ann[q] @ vec for q in range(n)])           # a_q |v>
            U = np.tensordot(K1, A1, axes=([1], [0]))                       # [p] vec
            out = out + sum(self.cre[p] @ U[p] for p in range(n))
        if K2 is not None or K3 is not None:
            A2 = np.empty((n, n, self.dim))
            for r in range(n):
                ar = self.ann[r]
                for s in range(n):
                    A2[r, s] = ar @ (self.ann[s] @ vec)                     # a_r a_s |v>
        if K2 is not None:
            U = np.tensordot(K2, A2, axes=([2, 3], [0, 1]))                 # [p][q] vec
            for p in range(n):
                for q in range(n):
                    out = out + self.cre[p] @ (self.cre[q] @ U[p, q])
        if K3 is not None:
            A3 = np.empty((n, n, n, self.dim))
            for s in range(n):
                for t in range(n):
                    for u in range(n):
                        A3[s, t, u] = self.ann[s] @ A2[t, u]
            U = np.tensordot(K3, A3, axes=([3, 4, 5], [0, 1, 2]))
            for p in range(n):
                for q in range(n):
                    for r in range(n):
                        out = out + self.cre[p] @ (self.cre[q] @ (self.cre[r] @ U[p, q, r]))
        return out

    def matrix(self, op, basis):
        """Dense matrix of a bare plain-order operator restricted to ``basis`` states."""
        M = np.empty((len(basis), len(basis)))
        for j, st in enumerate(basis):
            e = np.zeros(self.dim)
            e[st] = 1.0
            M[:, j] = self.apply(op, e)[basis]
        return M


def reference_vector(sp: Spaces, ci, n_alpha: int, n_beta: int, fs: FockSpace):
    """|Psi0> = core^2 x sum c_IJ |I_alpha J_beta> x virtual^0 in the full Fock space."""
    core = sum(1 << k for k in range(2 * sp.nC))
    vec = np.zeros(fs.dim)
    if sp.nA == 0:
        vec[core] = 1.0
        return vec
    a0 = 2 * sp.nC
    for ia, sa in enumerate(det_strings(sp.nA, n_alpha)):
        ma = sum(1 << (a0 + o) for o in sa)
        for ib, sb in enumerate(det_strings(sp.nA, n_beta)):
            mb = sum(1 << (a0 + sp.nA + o) for o in sb)
            vec[core | ma | mb] = ci[ia, ib]
    return vec


def rdm(fs: FockSpace, vec, order: int, idx):
    """Plain-order density <a+_p1..a+_pk a_q1..a_qk> over the index list ``idx``."""
    m = len(idx)
    if order == 1:
        W = np.array([fs.ann[q] @ vec for q in idx])
        return W @ W.T                                      # <a+_p a_q> = (a_p v).(a_q v)
    if order == 2:
        W = np.array([[fs.ann[q] @ (fs.ann[r] @ vec) for r in idx] for q in idx])
        W = W.reshape(m * m, -1)
        # <a+p a+q a_r a_s> = (a_q a_p v).(a_r a_s v)
        G = W @ W.T                                         # [(x,y),(r,s)] = (a_x a_y v).(a_r a_s v)
        G = G.reshape(m, m, m, m)                           # [x,y,r,s]
        return G.transpose(1, 0, 2, 3)                      # x=q,y=p -> [p,q,r,s]
    if order == 3:
        W = np.empty((m, m, m, fs.dim))
        for a, q in enumerate(idx):
            for b, r in enumerate(idx):
                for c, s in enumerate(idx):
                    W[a, b, c] = fs.ann[q] @ (fs.ann[r] @ (fs.ann[s] @ vec))   # a_q a_r a_s |v>
        W = W.reshape(m ** 3, -1)
        G = (W @ W.T).reshape(m, m, m, m, m, m)              # [x,y,z,q,r,s] = (a_x a_y a_z v).(a_q a_r a_s v)
        # <a+p a+q a+r a_s a_t a_u> = (a_r a_q a_p v).(a_s a_t a_u v)
        return G.transpose(2, 1, 0, 3, 4, 5)


def sector_basis(fs: FockSpace, sp: Spaces, n_alpha_tot: int, n_beta_tot: int):
    """States with the given numbers of alpha and beta electrons."""
    spatial, spin = sp.so_index()
    st = np.arange(fs.dim)
    na = np.zeros(fs.dim, dtype=int)
    nb = np.zeros(fs.dim, dtype=int)
    for k in range(fs.n):
        bit = (st >> k) & 1
        if spin[k] == 0:
            na += bit
        else:
            nb += bit
    return np.nonzero((na == n_alpha_tot) & (nb == n_beta_tot))[0]


def rspt_energies(Hmat0_diag: np.ndarray, Vmat: np.ndarray, ref: int):
    """Second- and third-order Rayleigh-Schroedinger energies for H = H0 + V with a
    diagonal H0 in the determinant basis; ``ref`` is the reference row."""
    E0 = Hmat0_diag[ref]
    others = np.array([k for k in range(len(Hmat0_diag)) if k != ref])
    d = E0 - Hmat0_diag[others]
    V0k = Vmat[ref, others]
    E1 = Vmat[ref, ref]
    E2 = float(np.sum(V0k * V0k / d))
    Vkl = Vmat[np.ix_(others, others)] - E1 * np.eye(len(others))
    E3 = float((V0k / d) @ Vkl @ (V0k / d))
    return E1, E2, E3


def active_rdm_blocks(ci, nA: int, n_alpha: int, n_beta: int):
    """The reference densities of a CAS vector in the library's spin-block input layout,
    from brute-force expectation values in the full Fock space of the 2 nA active spin
    orbitals (nA <= 7): gamma1[s][u][v] = <a+_{us} a_{vs}>, gamma2[b][u][v][x][y] =
    <a+_u a+_v a_y a_x> (blocks aa, ab, bb), gamma3[b][u][v][w][x][y][z] =
    <a+_u a+_v a+_w a_z a_y a_x> (blocks aaa, aab, abb, bbb)."""
    sp = Spaces(0, nA, 0)
    fs = FockSpace(2 * nA)
    vec = reference_vector(sp, ci, n_alpha, n_beta, fs)
    idx = list(range(2 * nA))
    D1 = rdm(fs, vec, 1, idx)
    D2 = rdm(fs, vec, 2, idx).transpose(0, 1, 3, 2)          # -> <a+p a+q a_s a_r> at [p,q,r,s]
    D3 = rdm(fs, vec, 3, idx).transpose(0, 1, 2, 5, 4, 3)    # -> <a+p a+q a+r a_u a_t a_s>
    a, b = slice(0, nA), slice(nA, 2 * nA)
    g1 = np.stack([D1[a, a], D1[b, b]])
    g2 = np.stack([D2[a, a, a, a], D2[a, b, a, b], D2[b, b, b, b]])
    g3 = np.stack([D3[a, a, a, a, a, a], D3[a, a, b, a, a, b], D3[a, b, b, a, b, b], D3[b, b, b, b, b, b]])
    return g1, g2, g3

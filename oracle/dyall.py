"""Active-to-virtual doubles under Dyall's zeroth-order Hamiltonian (oracle; FP64).

App. B ("other choices of zeroth-order Hamiltonian"): with H0 = E0 + F0 plus the
two-body interaction among the active orbitals, 1/4 sum_{uvxy in A} v^(0) {a+a+aa}, and
in the limit s -> inf, the first-order amplitudes that move two electrons from active
to virtual orbitals are no longer a driving term over a denominator: Eq. t2_aavv couples
t_{ef}^{uv} to every t_{ef}^{xy} of the same virtual pair,

    0 = v_{ef}^{uv} - Delta_{ef}^{uv} t_{ef}^{uv}
        - 1/2 sum_{xy in A} v_{xy}^{uv,(0)} t_{ef}^{xy}
        + sum_{xyz in A} v_{xy}^{uv,(0)} t_{ef}^{xz} gamma_z^y,

with Delta_{ef}^{uv} = e_u + e_v - e_e - e_f.  The index placement follows the paper's
tensor macro (lower = creation, upper = annihilation indices of the operator string; the
two-body coefficient multiplies 1/4 {a+_e a+_f a_v a_u}), and gamma_z^y = <a+_y a_z>.

In this package's spin-orbital arrays (``spaces``): t[e, f, u, v], v[p, q, r, s] =
<pq||rs>, gamma[y, z] = <a+_y a_z>.  For each virtual pair (e, f) the equation is a
linear system over the antisymmetric active pairs u < v; the system matrix differs
between pairs only by the shift e_e + e_f on its diagonal.  ``solve`` assembles each
block and calls numpy.linalg.solve on it.

Readings (each in the design notes):
* v^(1)_{ef}^{uv} is the ordinary antisymmetrised integral <ef||uv> (the active-only
  two-body part moves into H0; this block is not active-only).
* The shifted denominators of Eqs. full_preconditioner / no_preconditioner are the
  diagonal of this system.  The two printed forms disagree with each other in sign (the
  natural-orbital form of the first is 1/2 v (n_u + n_v - 1)) and, in the unique-pair
  representation, by a factor 2 from the system's diagonal; ``shifted_denominators``
  returns the system's own diagonal, Delta + v_{uv}^{uv}(1 - n_u - n_v) in natural
  orbitals.

Parity: the operator of Eq. t2_aavv is pinned against the generic commutator engine
(``gno``): the (VV|AA) block of [H0_Dyall, A]_{1,2} for arbitrary active-to-virtual
amplitudes (tests/test_oracle_dyall.py); the solution against the s -> inf limit of
Eq. T2_1st when the active interaction vanishes.
"""
from __future__ import annotations

import numpy as np

from paper_1701_02011_amd.synth import Problem

from .spaces import Spaces, build_densities, so_energies, so_integrals


def _pairs(n: int):
    """Unique pairs (u, v), u < v, of n indices, in row-major order."""
    iu = np.triu_indices(n, k=1)
    return iu[0], iu[1]


def operator_apply(t, v0, gamma):
    """The active-coupling part of Eq. t2_aavv acting on t[..., x, y] (antisymmetric):
        K(t)[..., u, v] = 1/2 sum_{xy} v0[x,y,u,v] t[..., x, y]
                          - sum_{xyz} v0[x,y,u,v] t[..., x, z] gamma[y, z]
    so that Eq. t2_aavv reads Delta t + K(t) = v."""
    a = 0.5 * np.einsum("xyuv,...xy->...uv", v0, t, optimize=True)
    b = np.einsum("xyuv,...xz,yz->...uv", v0, t, gamma, optimize=True)
    return a - b


def system_blocks(sp: Spaces, eps_so, v, gamma):
    """K as a matrix over the unique active pairs (rows: output pair, columns: input pair),
    and the active pair sums d[k] = e_u + e_v.  Active spin orbitals ordered [alpha | beta]."""
    A = sp.A
    n = 2 * sp.nA
    v0 = v[A, A, A, A]
    gA = gamma[A, A]
    iu, iv = _pairs(n)
    npair = len(iu)
    K = np.zeros((npair, npair))
    for c in range(npair):
        t = np.zeros((n, n))
        t[iu[c], iv[c]] = 1.0
        t[iv[c], iu[c]] = -1.0
        K[:, c] = operator_apply(t, v0, gA)[iu, iv]
    ea = eps_so[A]
    d = ea[iu] + ea[iv]
    return K, d, (iu, iv)


def solve(prob: Problem, v=None):
    """t[e, f, u, v] over virtual (e, f) and active (u, v) spin orbitals, solving Eq. t2_aavv
    block by block.  Returns (t, K, d): t as a [2nV][2nV][2nA][2nA] antisymmetric array."""
    sp = Spaces(prob.n_core, prob.n_active, prob.n_virtual)
    dens = build_densities(sp, prob.gamma1, prob.gamma2, prob.gamma3, with_D3=False)
    eps = so_energies(sp, prob.eps)
    if v is None:
        v = so_integrals(sp, prob.B)
    K, d, (iu, iv) = system_blocks(sp, eps, v, dens.gamma)
    V, A = sp.V, sp.A
    ev = eps[V]
    nv2, n = 2 * sp.nV, 2 * sp.nA
    rhs = v[V, V, A, A][:, :, iu, iv]                  # [e][f][pair]
    t = np.zeros((nv2, nv2, n, n))
    for e in range(nv2):
        for f in range(nv2):
            if e == f:
                continue
            M = K + np.diag(d - ev[e] - ev[f])         # Delta + K, Eq. t2_aavv
            x = np.linalg.solve(M, rhs[e, f])
            t[e, f, iu, iv] = x
            t[e, f, iv, iu] = -x
    return t, K, d


def residual(prob: Problem, t, v=None):
    """Right-hand side of Eq. t2_aavv evaluated at t (zero at the solution)."""
    sp = Spaces(prob.n_core, prob.n_active, prob.n_virtual)
    dens = build_densities(sp, prob.gamma1, prob.gamma2, prob.gamma3, with_D3=False)
    eps = so_energies(sp, prob.eps)
    if v is None:
        v = so_integrals(sp, prob.B)
    V, A = sp.V, sp.A
    ev, ea = eps[V], eps[A]
    D = (ea[None, None, :, None] + ea[None, None, None, :]
         - ev[:, None, None, None] - ev[None, :, None, None])
    return v[V, V, A, A] - D * t - operator_apply(t, v[A, A, A, A], dens.gamma[A, A])


def shifted_denominators(K, d, ev):
    """D[e, f, k] = d[k] - e_e - e_f + K[k, k]: the diagonal of each block of Eq. t2_aavv
    (the paper's shifted denominators, Eq. full_preconditioner, read as that diagonal)."""
    return d[None, None, :] - ev[:, None, None] - ev[None, :, None] + np.diag(K)[None, None, :]

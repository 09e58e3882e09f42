"""Pins of the oracle's one-step relaxed energy (oracle/relax.py; Sec. II.B Eq. E_relaxed,
App. A Eqs. Hbar_mb, Hbar_DNO, c0_cas), each against something other than the oracle's
own formulas: Fock-space normal products, the variational principle, homogeneity in the
perturbation and the structure of the zeroth-order Hamiltonian."""
import dataclasses

import numpy as np
import pytest

from paper_1701_02011_amd.synth import det_strings, make_problem
from oracle import dsrg, gno, relax
from oracle.dsrg import anti_hermitian
from oracle.hilbert import FockSpace, reference_vector, sector_basis
from oracle.spaces import Spaces, build_densities, so_energies

from fock_normal import normal_product_action

MICRO = [(1, 2, 1, 5), (1, 3, 2, 6), (0, 3, 2, 8), (2, 2, 1, 9)]


def _problem(nC, nA, nV, seed, s=0.5):
    p = make_problem(nC, nA, nV, 8, seed=seed, s=s, f_sigma=0.05)
    return dataclasses.replace(p, e0=-1.25)


def _ci_in_basis(p, basis):
    """The reference CI vector in the order of an active-only determinant basis."""
    nA = p.n_active
    v = np.zeros(1 << (2 * nA))
    for ia, sa in enumerate(det_strings(nA, p.n_alpha)):
        ma = sum(1 << o for o in sa)
        for ib, sb in enumerate(det_strings(nA, p.n_beta)):
            mb = sum(1 << (nA + o) for o in sb)
            v[ma | mb] = p.ci[ia, ib]
    return v[basis]


@pytest.mark.parametrize("nC,nA,nV,seed", MICRO)
def test_rayleigh_quotient_of_reference_is_unrelaxed_energy(nC, nA, nV, seed):
    """Every normal-ordered part of Hbar has zero reference expectation value, so the CAS
    matrix in true-vacuum order must give <Psi0|H_CAS|Psi0> = Hbar_0 = E0 + E(2) + E(3)
    of the unrelaxed series (computed by the pinned unrelaxed oracle); and its lowest
    eigenvalue lies at or below that quotient (variational principle).  A dropped or
    mis-signed term of the de-normal-ordering constant or of c^u_v breaks the equality."""
    p = _problem(nC, nA, nV, seed)
    r = relax.relaxed_energy(p)
    o = dsrg.run(p)
    e_u = p.e0 + o.e2 + o.e3
    assert abs(r.e_unrelaxed - e_u) < 1e-12
    M, basis, _ = relax.cas_matrix(r.const, r.c, r.w, nA, p.n_alpha, p.n_beta)
    c = _ci_in_basis(p, basis)
    assert abs(c @ c - 1.0) < 1e-12
    assert abs(c @ M @ c - e_u) < 1e-11
    assert np.abs(M - M.T).max() < 1e-12
    assert r.e_relaxed <= e_u + 1e-12


@pytest.mark.parametrize("nC,nA,nV,seed", [(1, 2, 1, 5), (1, 2, 2, 11)])
def test_cas_matrix_matches_full_space_normal_products(nC, nA, nV, seed):
    """App. A: restricted to determinants with the core doubly occupied and the virtuals
    empty, Hbar_{1,2} over every spin orbital (core, active, virtual blocks) equals the
    active-only H_CAS (const, c^u_v, Hbar^uv_xy): the core folding c0 cancels the core
    terms of the de-normal-ordered operator.  The left side is built in the full Fock
    space from normal products of brute-force reference expectation values."""
    p = _problem(nC, nA, nV, seed)
    sp = Spaces(nC, nA, nV)
    n = 2 * sp.N
    hb = relax.hbar3(p, "all")
    const, c, w = relax.cas_operator(hb)
    Mcas, basis_a, _ = relax.cas_matrix(const, c, w, nA, p.n_alpha, p.n_beta)
    fs = FockSpace(n)
    psi0 = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    # CAS determinants inside the full Fock space: core bits set, virtual bits clear
    core = sum(1 << k for k in range(2 * nC))
    basis = [core | (int(b) << (2 * nC)) for b in basis_a]
    entries1 = [(i, j, hb.h1[i, j]) for i in range(n) for j in range(n) if hb.h1[i, j] != 0.0]
    idx = np.argwhere(np.abs(hb.h2) > 0.0)
    Mfull = np.zeros((len(basis), len(basis)))
    for col, st in enumerate(basis):
        x = np.zeros(fs.dim)
        x[st] = 1.0
        memo = {}
        y = hb.h0 * x
        for i, j, val in entries1:
            y = y + val * normal_product_action(fs, psi0, [i], [j], x, memo)
        for (pp, q, r_, s_) in idx:
            # 1/4 Hbar^{pq}_{rs} {a+_p a+_q a_s a_r}
            y = y + 0.25 * hb.h2[pp, q, r_, s_] * normal_product_action(
                fs, psi0, [int(pp), int(q)], [int(s_), int(r_)], x, memo)
        Mfull[:, col] = y[basis]
    assert np.abs(Mfull - Mcas).max() < 1e-11


@pytest.mark.parametrize("nC,nA,nV,seed", MICRO)
def test_active_blocks_need_only_excitation_blocks_of_h2(nC, nA, nV, seed):
    """The reading that H~(2)_{1,2} enters the active blocks through its excitation and
    de-excitation blocks only: forming every block of every intermediate gives the same
    active blocks and the same relaxed energy."""
    p = _problem(nC, nA, nV, seed)
    a = relax.relaxed_energy(p, "active")
    f = relax.relaxed_energy(p, "all")
    A = Spaces(nC, nA, nV).A
    assert np.abs(f.hbar.h1[A, A] - a.hbar.h1).max() < 1e-12
    assert np.abs(f.hbar.h2[A, A, A, A] - a.hbar.h2).max() < 1e-12
    assert abs(f.e_relaxed - a.e_relaxed) < 1e-12


def test_h0_commutators_have_no_active_elements():
    """Sec. II.B: with the diagonal zeroth-order Hamiltonian, [H(0), A] has excitation and
    de-excitation elements only, for any anti-Hermitian A built from non-internal
    amplitudes; so its active blocks and its scalar vanish (the reading under which
    [H(0), A(3)] is not formed)."""
    nC, nA, nV = 1, 3, 2
    p = _problem(nC, nA, nV, 21)
    sp = Spaces(nC, nA, nV)
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    eps = so_energies(sp, p.eps)
    m1, m2 = dsrg._internal_mask(sp)
    rng = np.random.default_rng(3)
    t2 = rng.standard_normal((n,) * 4)
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    t2 = np.where(m2, t2, 0.0)
    t1 = np.where(m1, rng.standard_normal((n, n)), 0.0)
    A = gno.to_plain(0.0, *anti_hermitian(t1, t2))
    k0, k1, k2 = gno.commutator((0.0, np.diag(eps), None), A, dens, want0=True,
                                want1=(sp.A, sp.A), want2=(sp.A,) * 4)
    assert abs(k0) < 1e-12
    assert np.abs(k1).max() < 1e-12
    assert np.abs(k2).max() < 1e-12
    # and it is not zero elsewhere
    _, e1, _ = gno.commutator((0.0, np.diag(eps), None), A, dens, want1=(sp.P, sp.H))
    assert np.abs(e1).max() > 1e-3


def test_orders_are_homogeneous_in_the_perturbation():
    """Scaling H(1) by k (f(1) -> k f(1), B -> sqrt(k) B) scales A(n) by k^n and Hbar^(n)
    by k^n, with the zeroth-order Hamiltonian and the densities fixed: each order's
    active blocks must be homogeneous of its degree (a term assigned to the wrong order
    fails this)."""
    p = _problem(1, 3, 2, 6)
    k = 0.37
    q = dataclasses.replace(p, B=p.B * np.sqrt(k), f_offdiag=p.f_offdiag * k)
    a = relax.hbar3(p)
    b = relax.hbar3(q)
    for order in range(4):
        for xa, xb in ((a.orders1[order], b.orders1[order]), (a.orders2[order], b.orders2[order])):
            scale = max(np.abs(xa).max(), 1e-300)
            assert np.abs(xb - k ** order * xa).max() <= 1e-11 * scale + 1e-15
    assert abs(b.e2 - k ** 2 * a.e2) < 1e-12 * abs(a.e2)
    assert abs(b.e3 - k ** 3 * a.e3) < 1e-11 * abs(a.e3)
    # the second and third orders carry active elements
    assert np.abs(a.orders2[2]).max() > 1e-4 and np.abs(a.orders2[3]).max() > 1e-5


def test_hbar_active_blocks_are_hermitian():
    p = _problem(1, 3, 2, 6)
    hb = relax.hbar3(p)
    assert np.abs(hb.h1 - hb.h1.T).max() < 1e-12
    assert np.abs(hb.h2 - hb.h2.transpose(2, 3, 0, 1)).max() < 1e-12
    assert np.abs(hb.h2 + hb.h2.transpose(1, 0, 2, 3)).max() < 1e-12


@pytest.mark.parametrize("nC,nA,nV", [(2, 1, 2), (2, 0, 3)])
def test_one_determinant_space_is_not_relaxed(nC, nA, nV):
    """A CAS space of one determinant (one active orbital with one electron, or no active
    orbitals) leaves nothing to relax: E^[3] equals the unrelaxed energy."""
    p = _problem(nC, nA, nV, 31)
    r = relax.relaxed_energy(p)
    assert abs(r.e_relaxed - r.e_unrelaxed) < 1e-12

"""Pins of the oracle for the active-to-virtual doubles under Dyall's zeroth-order
Hamiltonian (App. B, Eq. t2_aavv), none of which reuses the oracle's own algebra for it:

* the printed equation against the generic MK-GNO commutator engine: the (VV|AA) block of
  [F0 + V0_active, T - T+]_{1,2} for arbitrary active-to-virtual amplitudes T;
* the s -> inf limit of Eq. T2_1st (t = v / Delta) when the active interaction is zero;
* in natural orbitals, the diagonal of each block is Delta + <uv||uv>(1 - n_u - n_v).
"""
import numpy as np
import pytest

from oracle import dyall, gno
from oracle.spaces import Spaces, build_densities, so_energies, so_integrals
from paper_1701_02011_amd.synth import make_problem


def _random_aavv(sp, rng, spin_conserving=True):
    n = 2 * sp.N
    t = np.zeros((n,) * 4)
    V, A = sp.V, sp.A
    blk = rng.standard_normal((2 * sp.nV, 2 * sp.nV, 2 * sp.nA, 2 * sp.nA))
    blk = blk - blk.transpose(1, 0, 2, 3)
    blk = blk - blk.transpose(0, 1, 3, 2)
    if spin_conserving:
        _, spin = sp.so_index()
        sv, sa = spin[V], spin[A]
        keep = ((sv[:, None, None, None] + sv[None, :, None, None])
                == (sa[None, None, :, None] + sa[None, None, None, :]))
        blk = np.where(keep, blk, 0.0)
    t[V, V, A, A] = blk
    return t


@pytest.mark.parametrize("shape,seed,spin_conserving",
                         [((1, 2, 2, 5), 11, True), ((1, 3, 2, 6), 12, True), ((0, 3, 1, 4), 13, False)])
def test_equation_matches_commutator_engine(shape, seed, spin_conserving):
    """0 = v - Delta t - 1/2 v0 t + v0 t gamma is v + [H0_Dyall, A]_{1,2} on (VV|AA)."""
    p = make_problem(*shape, seed=seed)
    sp = Spaces(p.n_core, p.n_active, p.n_virtual)
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    eps = so_energies(sp, p.eps)
    v = so_integrals(sp, p.B)
    n = 2 * sp.N
    A, V, P, H = sp.A, sp.V, sp.P, sp.H
    v0 = np.zeros((n,) * 4)
    v0[A, A, A, A] = v[A, A, A, A]
    H0 = gno.to_plain(0.0, np.diag(eps), v0)
    t = _random_aavv(sp, np.random.default_rng(seed), spin_conserving)
    Aop = gno.to_plain(0.0, np.zeros((n, n)), t - t.transpose(2, 3, 0, 1))
    _, _, c2p = gno.commutator(H0, Aop, dens, want2=(P, P, H, H))
    c2 = gno.c_from_plain2(c2p)
    vP = slice(2 * sp.nA, 2 * sp.nA + 2 * sp.nV)       # V inside P
    aH = slice(2 * sp.nC, 2 * sp.nH)                    # A inside H
    engine = c2[vP, vP, aH, aH]
    tb = t[V, V, A, A]
    ev, ea = eps[V], eps[A]
    D = (ea[None, None, :, None] + ea[None, None, None, :]
         - ev[:, None, None, None] - ev[None, :, None, None])
    printed = -D * tb - dyall.operator_apply(tb, v[A, A, A, A], dens.gamma[A, A])
    assert np.abs(engine - printed).max() < 1e-12 * max(1.0, np.abs(printed).max())
    # the pin fails for a plausible misreading: the gamma term with the transposed density
    wrong = -D * tb - dyall.operator_apply(tb, v[A, A, A, A], dens.gamma[A, A].T.copy() * 0.5)
    assert np.abs(engine - wrong).max() > 1e-6


def test_no_active_interaction_gives_first_order_limit():
    """With v0 = 0 each block is diagonal: t = v / Delta, Eq. T2_1st at s -> inf."""
    p = make_problem(1, 3, 3, 8, seed=21)
    sp = Spaces(p.n_core, p.n_active, p.n_virtual)
    v = so_integrals(sp, p.B)
    A, V = sp.A, sp.V
    v[A, A, A, A] = 0.0
    t, K, _ = dyall.solve(p, v=v)
    assert np.abs(K).max() == 0.0
    eps = so_energies(sp, p.eps)
    ev, ea = eps[V], eps[A]
    D = (ea[None, None, :, None] + ea[None, None, None, :]
         - ev[:, None, None, None] - ev[None, :, None, None])
    ref = np.where(D != 0.0, v[V, V, A, A] / np.where(D != 0.0, D, 1.0), 0.0)
    n2 = 2 * sp.nV
    off = ~np.eye(n2, dtype=bool)[:, :, None, None]
    np.testing.assert_allclose(np.where(off, t, 0.0), np.where(off, ref, 0.0), rtol=0, atol=1e-13)


def test_solution_solves_the_equation():
    p = make_problem(1, 4, 3, 10, seed=22)
    t, _, _ = dyall.solve(p)
    r = dyall.residual(p, t)
    assert np.abs(r).max() < 1e-11 * max(1.0, np.abs(t).max())
    # antisymmetric in both pairs
    assert np.abs(t + t.transpose(1, 0, 2, 3)).max() == 0.0
    assert np.abs(t + t.transpose(0, 1, 3, 2)).max() == 0.0


def test_diagonal_in_natural_orbitals():
    """gamma diagonal (occupations n_u): diag(K) = <uv||uv>(1 - n_u - n_v) per unique pair."""
    p = make_problem(0, 3, 2, 6, seed=23)
    sp = Spaces(p.n_core, p.n_active, p.n_virtual)
    eps = so_energies(sp, p.eps)
    v = so_integrals(sp, p.B)
    n = 2 * sp.N
    occ = np.array([0.9, 0.6, 0.2, 0.8, 0.5, 0.1])
    gamma = np.zeros((n, n))
    gamma[sp.A, sp.A] = np.diag(occ)
    K, d, (iu, iv) = dyall.system_blocks(sp, eps, v, gamma)
    vA = v[sp.A, sp.A, sp.A, sp.A]
    ref = vA[iu, iv, iu, iv] * (1.0 - occ[iu] - occ[iv])
    np.testing.assert_allclose(np.diag(K), ref, rtol=0, atol=1e-14)

"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test states what fixes the expected value: brute force in the full Fock space,
a closed form, a limit, or an exact invariance.  None of them reuses the oracle's
own formulas for the expected side.
"""
import itertools
import math

import dataclasses

import numpy as np
import pytest

from paper_1701_02011_amd import synth
from paper_1701_02011_amd.synth import make_problem, Problem
from oracle import dsrg, gno
from oracle.gno import Term, _project
from oracle.hilbert import (FockSpace, reference_vector, rdm, sector_basis, rspt_energies)
from fock_normal import fock_string as _fock_string, normal_product_action as _normal_product_action
from oracle.spaces import (Spaces, build_densities, so_energies, so_integrals,
                           expand_rdm_blocks, cumulants)


def _micro(nC=1, nA=2, nV=3, M=10, seed=11, s=0.5):
    return make_problem(nC, nA, nV, M, seed=seed, s=s)


# ---------------------------------------------------------------------------
# Densities and cumulants (step a0)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nC,nA,nV,seed", [(1, 3, 2, 7), (2, 2, 1, 8), (0, 4, 1, 9)])
def test_densities_match_fock_space(nC, nA, nV, seed):
    """gamma, <a+a+aa>, <a+a+a+aaa> over the hole space (core included), rebuilt from
    the cumulant expansion, equal brute-force expectation values of the full reference."""
    p = make_problem(nC, nA, nV, 6, seed=seed)
    sp = Spaces(nC, nA, nV)
    fs = FockSpace(2 * sp.N)
    vec = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    assert abs(vec @ vec - 1.0) < 1e-14
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    H = list(range(2 * sp.nH))
    np.testing.assert_allclose(rdm(fs, vec, 1, list(range(2 * sp.N))), dens.gamma, atol=1e-14)
    np.testing.assert_allclose(rdm(fs, vec, 2, H), dens.D2p, atol=1e-14)
    np.testing.assert_allclose(rdm(fs, vec, 3, H), dens.D3p, atol=1e-14)


def test_single_determinant_cumulants_vanish():
    """A one-determinant CAS vector has zero two- and three-body cumulants."""
    nA, na, nb = 4, 2, 2
    ci = np.zeros((math.comb(nA, na), math.comb(nA, nb)))
    ci[3, 1] = -1.0
    g1, g2, g3 = synth.active_rdms(ci, nA, na, nb)
    G1, G2, G3 = expand_rdm_blocks(nA, g1, g2, g3)
    L2, L3 = cumulants(G1, G2, G3)
    assert np.abs(L2).max() < 1e-15 and np.abs(L3).max() < 1e-15
    # and the cumulants of a correlated vector do not vanish
    p = make_problem(0, nA, 1, 4, seed=3)
    G1, G2, G3 = expand_rdm_blocks(nA, p.gamma1, p.gamma2, p.gamma3)
    L2, L3 = cumulants(G1, G2, G3)
    assert np.abs(L2).max() > 1e-3 and np.abs(L3).max() > 1e-3


def test_rdm_traces():
    """Partial traces fixed by the electron numbers."""
    p = synth.make_config("small")
    na, nb = p.n_alpha, p.n_beta
    assert abs(np.trace(p.gamma1[0]) - na) < 1e-12 and abs(np.trace(p.gamma1[1]) - nb) < 1e-12
    assert abs(np.einsum("uvuv->", p.gamma2[1]) - na * nb) < 1e-10
    assert abs(np.einsum("uvuv->", p.gamma2[0]) - na * (na - 1)) < 1e-10
    assert abs(np.einsum("uvwuvw->", p.gamma3[2]) - na * nb * (nb - 1)) < 1e-9


# ---------------------------------------------------------------------------
# Commutator engine
# ---------------------------------------------------------------------------
def _dense_terms(terms):
    acc = 0.0
    for t in terms:
        spec = ",".join(l for _, l in t.factors) + "->" + t.out
        acc = acc + t.coef * np.einsum(spec, *[T for T, _ in t.factors])
    return acc


def test_bare_commutator_equals_matrix_commutator():
    rng = np.random.default_rng(1)
    n = 8
    fs = FockSpace(n)
    X = (0.0, rng.standard_normal((n, n)), rng.standard_normal((n,) * 4))
    Y = (0.0, rng.standard_normal((n, n)), rng.standard_normal((n,) * 4))
    R1, R2, R3 = gno.bare_commutator_terms(X, Y)
    op = (0.0, _dense_terms(R1), _dense_terms(R2), _dense_terms(R3))
    phi = rng.standard_normal(fs.dim)
    lhs = fs.apply(X, fs.apply(Y, phi)) - fs.apply(Y, fs.apply(X, phi))
    rhs = fs.apply(op, phi)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(lhs).max()


def test_gno_expectation_and_round_trip():
    """<Psi0|{X}|Psi0> = 0 for normal-ordered X; GNO -> bare -> GNO is the identity."""
    p = _micro(1, 3, 2, 8, seed=7)
    sp = Spaces(p.n_core, p.n_active, p.n_virtual)
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    fs = FockSpace(n)
    vec = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    rng = np.random.default_rng(3)
    X = (0.0, rng.standard_normal((n, n)), rng.standard_normal((n,) * 4))
    Xb = gno.gno_to_bare(X, dens)
    assert abs(vec @ fs.apply(Xb, vec)) < 1e-12
    G, H = slice(0, n), slice(0, 2 * sp.nH)
    R1 = [Term(1.0, [(Xb[1], "ab")], "ab")]
    R2 = [Term(1.0, [(Xb[2], "abcd")], "abcd")]
    c0, c1, c2 = _project(R1, R2, [], dens, True, (G, G), (G, G, G, G), G, H)
    assert abs(c0 + Xb[0]) < 1e-12
    assert np.abs(c1 - X[1]).max() < 1e-13 and np.abs(c2 - X[2]).max() < 1e-13


def test_generalised_wick_pair_product():
    """<{a+p a_q}{a+r a_s}> = gamma_ps eta_rq + lambda^{pr}_{qs}: the MK-GNO contraction
    rule for two one-body operators, read off from brute-force matrices."""
    p = _micro(0, 3, 1, 4, seed=21)
    sp = Spaces(0, 3, 1)
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    fs = FockSpace(n)
    vec = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    g = dens.gamma
    eta = np.eye(n) - g
    A = sp.A
    L2 = np.zeros((n,) * 4)
    L2[A, A, A, A] = dens.L2
    for (pp, q, r, s) in [(0, 1, 1, 0), (2, 0, 0, 2), (1, 4, 3, 0), (3, 3, 0, 0), (5, 2, 2, 5)]:
        Op = np.zeros((n, n)); Op[pp, q] = 1.0
        Or = np.zeros((n, n)); Or[r, s] = 1.0
        bp = gno.gno_to_bare((0.0, Op, None), dens)
        br = gno.gno_to_bare((0.0, Or, None), dens)
        val = vec @ fs.apply(bp, fs.apply(br, vec))
        ref = g[pp, s] * eta[r, q] + L2[pp, r, q, s]
        assert abs(val - ref) < 1e-13


def test_projection_single_determinant_excitations():
    """For a one-determinant reference, the GNO one- and two-body excitation parts of any
    operator are its matrix elements with singly / doubly excited determinants."""
    sp = Spaces(2, 0, 3)
    n = 2 * sp.N
    dens = build_densities(sp, None, None, None)
    fs = FockSpace(n)
    phi = reference_vector(sp, None, 0, 0, fs)
    rng = np.random.default_rng(5)
    K2 = rng.standard_normal((n,) * 4)
    K3 = rng.standard_normal((n,) * 6)
    G, H = slice(0, n), slice(0, 2 * sp.nH)
    c0, c1, c2 = _project([], [Term(1.0, [(K2, "abcd")], "abcd")],
                          [Term(1.0, [(K3, "abcdef")], "abcdef")], dens, True,
                          (G, G), (G, G, G, G), G, H)
    Ophi = fs.apply((0.0, None, K2, K3), phi)
    assert abs(c0 - phi @ Ophi) < 1e-12

    def exc(cre, ann):
        v = phi
        for q in ann:
            v = fs.ann[q] @ v
        for c in cre:
            v = fs.cre[c] @ v
        return v
    occ, vir = range(4), range(4, 10)
    for i in occ:
        for a in vir:
            assert abs(exc([a], [i]) @ Ophi - c1[a, i]) < 1e-12
    for i, j in itertools.combinations(occ, 2):
        for a, b in itertools.combinations(vir, 2):
            ref = c2[a, b, j, i] - c2[b, a, j, i] - c2[a, b, i, j] + c2[b, a, i, j]
            assert abs(exc([b, a], [i, j]) @ Ophi - ref) < 1e-12


def test_scalar_needs_only_deexcitation_block():
    """<[X, T]> depends only on X's elements with creators in H and annihilators in P
    (the restriction used for <[H~(2), T(1)]>)."""
    p = _micro(1, 2, 2, 6, seed=4)
    sp = Spaces(1, 2, 2)
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    rng = np.random.default_rng(9)
    X1 = rng.standard_normal((n, n)); X1 = X1 + X1.T
    X2 = rng.standard_normal((n,) * 4)
    X2 = X2 - X2.transpose(1, 0, 2, 3); X2 = X2 - X2.transpose(0, 1, 3, 2)
    X2 = X2 + X2.transpose(2, 3, 0, 1)
    r = dsrg.run(p)
    T = gno.to_plain(0.0, r.t1_1, r.t2_1)
    full, _, _ = gno.commutator(gno.to_plain(0.0, X1, X2), T, dens, want0=True)
    H, P = sp.H, sp.P
    Y1 = np.zeros_like(X1); Y1[H, P] = X1[H, P]
    Y2 = np.zeros_like(X2); Y2[H, H, P, P] = X2[H, H, P, P]
    part, _, _ = gno.commutator(gno.to_plain(0.0, Y1, Y2), T, dens, want0=True)
    assert abs(full - part) < 1e-12 * max(1.0, abs(full))


# ---------------------------------------------------------------------------
# DSRG-MRPT3 energies
# ---------------------------------------------------------------------------
def test_e2_matches_fock_space():
    """E^(2) = <Psi0|[H~(1), T(1)]|Psi0> with H~(1) = 2 H(1) + [H(0), A(1)] formed from
    brute-force operator matrices (no normal-ordered algebra beyond rank-2 conversion)."""
    p = _micro(1, 2, 3, 10, seed=11, s=0.5)
    r = dsrg.run(p)
    sp = r.sp
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    fs = FockSpace(n)
    vec = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    v = so_integrals(sp, p.B)
    H1 = gno.gno_to_bare(gno.to_plain(0.0, None, v), dens)
    F0 = gno.gno_to_bare((0.0, np.diag(r.eps), None), dens)
    a1, a2 = dsrg.anti_hermitian(r.t1_1, r.t2_1)
    A1 = gno.gno_to_bare(gno.to_plain(0.0, a1, a2), dens)
    T1 = gno.gno_to_bare(gno.to_plain(0.0, r.t1_1, r.t2_1), dens)

    def Ht(x):
        return 2.0 * fs.apply(H1, x) + fs.apply(F0, fs.apply(A1, x)) - fs.apply(A1, fs.apply(F0, x))
    e2 = vec @ Ht(fs.apply(T1, vec)) - vec @ fs.apply(T1, Ht(vec))
    assert abs(e2 - r.e2) < 1e-12


def test_e3_scalars_match_fock_space():
    """Both scalars of E^(3) equal brute-force expectation values of the commutators of
    the operators the oracle formed."""
    p = _micro(1, 2, 2, 8, seed=13, s=0.7)
    r = dsrg.run(p)
    sp = r.sp
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    fs = FockSpace(n)
    vec = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    H, P = sp.H, sp.P
    X1 = np.zeros((n, n)); X1[P, H] = r.h2_1; X1[H, P] = r.h2_1.T
    X2 = np.zeros((n,) * 4); X2[P, P, H, H] = r.h2_2; X2[H, H, P, P] = r.h2_2.transpose(2, 3, 0, 1)
    Xb = gno.gno_to_bare(gno.to_plain(0.0, X1, X2), dens)
    T1 = gno.gno_to_bare(gno.to_plain(0.0, r.t1_1, r.t2_1), dens)
    e3b = vec @ fs.apply(Xb, fs.apply(T1, vec)) - vec @ fs.apply(T1, fs.apply(Xb, vec))
    assert abs(e3b - r.e3_b) < 1e-12


@pytest.mark.parametrize("nC,nV,seed", [(2, 3, 5), (1, 4, 6), (2, 4, 8)])
def test_single_reference_infinite_s_is_mp2_mp3(nC, nV, seed):
    """n_A = 0 and s -> infinity: E^(2) = MP2 and E^(3) = MP3, both from brute-force
    Rayleigh-Schroedinger perturbation theory in the determinant basis with H0 = F0."""
    p = make_problem(nC, 0, nV, 9, seed=seed, s=float("inf"))
    r = dsrg.run(p)
    sp = Spaces(nC, 0, nV)
    n = 2 * sp.N
    dens = build_densities(sp, None, None, None)
    fs = FockSpace(n)
    eps = so_energies(sp, p.eps)
    v = so_integrals(sp, p.B)
    basis = sector_basis(fs, sp, nC, nC)
    ref = list(basis).index(sum(1 << k for k in range(2 * nC)))
    V = fs.matrix(gno.gno_to_bare(gno.to_plain(0.0, None, v), dens), basis)
    occ = np.array([[(st >> k) & 1 for k in range(n)] for st in basis])
    h0 = occ @ eps
    E1, E2, E3 = rspt_energies(h0, V, ref)
    assert abs(E1) < 1e-15
    assert abs(r.e2 - E2) < 1e-14 and abs(r.e3 - E3) < 1e-14


@pytest.mark.parametrize("s", [0.1, 0.7, 3.0])
def test_single_reference_e2_closed_form(s):
    """n_A = 0: E^(2) = 1/4 sum |v^ij_ab|^2 (1 - exp(-2 s D^2)) / D, the product of
    Eq. T2_1st and the non-diagonal H~(1) of Sec. III under Eq. E(2)."""
    p = make_problem(2, 0, 4, 9, seed=17, s=s)
    r = dsrg.run(p)
    sp = Spaces(2, 0, 4)
    eps = so_energies(sp, p.eps)
    v = so_integrals(sp, p.B)
    H, P = sp.H, sp.P
    D = (eps[H, None, None, None] + eps[None, H, None, None]
         - eps[None, None, P, None] - eps[None, None, None, P])
    ref = 0.25 * np.sum(v[H, H, P, P] ** 2 * (-np.expm1(-2.0 * s * D ** 2)) / D)
    assert abs(r.e2 - ref) < 1e-14


def test_small_s_orders():
    """s -> 0: E^(2) = O(s), E^(3) = O(s^2) (t(1) ~ s, O1 and Z1 ~ s, t(2) ~ s^2)."""
    p = _micro(1, 2, 3, 10, seed=19)
    ss = np.array([1e-6, 1e-5, 1e-4])
    e2 = np.array([dsrg.run(p.with_s(s)).e2 for s in ss])
    e3 = np.array([dsrg.run(p.with_s(s)).e3 for s in ss])
    k2 = np.polyfit(np.log(ss), np.log(np.abs(e2)), 1)[0]
    k3 = np.polyfit(np.log(ss), np.log(np.abs(e3)), 1)[0]
    assert abs(k2 - 1.0) < 1e-3 and abs(k3 - 2.0) < 1e-3


def test_homogeneity():
    """B -> 2B: E^(2) -> 2^4 E^(2) and E^(3) -> 2^6 E^(3) (powers of two scale exactly)."""
    p = _micro(1, 2, 3, 10, seed=23)
    r1 = dsrg.run(p)
    r2 = dsrg.run(p.scaled(2.0))
    assert r2.e2 == pytest.approx(16.0 * r1.e2, rel=1e-14)
    assert r2.e3 == pytest.approx(64.0 * r1.e3, rel=1e-14)


def _product_problem(pa: Problem, pb: Problem, s: float) -> Problem:
    """Union of two fragments with disjoint orbitals and auxiliary ranges, with the
    product reference Psi_A Psi_B (a fixed global sign does not matter)."""
    def blocks(p):
        return (p.eps[:p.n_core], p.eps[p.n_core:p.n_hole], p.eps[p.n_hole:])
    ca, aa, va = blocks(pa)
    cb, ab, vb = blocks(pb)
    nC, nA, nV = pa.n_core + pb.n_core, pa.n_active + pb.n_active, pa.n_virtual + pb.n_virtual
    eps = np.concatenate([ca, cb, aa, ab, va, vb])
    # orbital maps of each fragment into the union
    def omap(p, c_off, a_off, v_off):
        return ([c_off + i for i in range(p.n_core)] + [nC + a_off + i for i in range(p.n_active)]
                + [nC + nA + v_off + i for i in range(p.n_virtual)])
    ma = omap(pa, 0, 0, 0)
    mb = omap(pb, pa.n_core, pa.n_active, pa.n_virtual)
    M = pa.n_aux + pb.n_aux
    N = nC + nA + nV
    B = np.zeros((M, N, N))
    B[np.ix_(range(pa.n_aux), ma, ma)] = pa.B
    B[np.ix_(range(pa.n_aux, M), mb, mb)] = pb.B
    # product CI vector over the union's active space
    na, nb = pa.n_alpha + pb.n_alpha, pa.n_beta + pb.n_beta
    sa = synth.det_strings(nA, na)
    sb = synth.det_strings(nA, nb)
    A_a = {s_: i for i, s_ in enumerate(synth.det_strings(pa.n_active, pa.n_alpha))}
    A_b = {s_: i for i, s_ in enumerate(synth.det_strings(pa.n_active, pa.n_beta))}
    B_a = {s_: i for i, s_ in enumerate(synth.det_strings(pb.n_active, pb.n_alpha))}
    B_b = {s_: i for i, s_ in enumerate(synth.det_strings(pb.n_active, pb.n_beta))}
    ci = np.zeros((len(sa), len(sb)))
    k = pa.n_active
    for I, s1 in enumerate(sa):
        x1 = tuple(o for o in s1 if o < k); y1 = tuple(o - k for o in s1 if o >= k)
        if x1 not in A_a or y1 not in B_a:
            continue
        for J, s2 in enumerate(sb):
            x2 = tuple(o for o in s2 if o < k); y2 = tuple(o - k for o in s2 if o >= k)
            if x2 not in A_b or y2 not in B_b:
                continue
            ci[I, J] = pa.ci[A_a[x1], A_b[x2]] * pb.ci[B_a[y1], B_b[y2]]
    g1, g2, g3 = synth.active_rdms(ci, nA, na, nb)
    return Problem(nC, nA, nV, M, eps, B, g1, g2, g3, s, ci=ci, n_alpha=na, n_beta=nb)


def test_size_consistency():
    """Two non-interacting fragments with a product reference: E(A u B) = E(A) + E(B)."""
    pa = make_problem(1, 2, 2, 5, seed=31, s=0.6)
    pb = make_problem(1, 2, 1, 4, seed=32, s=0.6)
    pab = _product_problem(pa, pb, 0.6)
    ra, rb, rab = dsrg.run(pa), dsrg.run(pb), dsrg.run(pab)
    assert abs(rab.e2 - (ra.e2 + rb.e2)) < 1e-12
    assert abs(rab.e3 - (ra.e3 + rb.e3)) < 1e-12


def test_antisymmetry_and_internal_zero():
    p = _micro(1, 2, 3, 10, seed=29)
    r = dsrg.run(p)
    sp = r.sp
    for t in (r.t2_1, r.t2_2):
        assert np.abs(t + t.transpose(1, 0, 2, 3)).max() < 1e-15
        assert np.abs(t + t.transpose(0, 1, 3, 2)).max() < 1e-15
        A = sp.A
        assert np.abs(t[A, A, A, A]).max() == 0.0
    for o in (r.o1_2, r.z1_2, r.h2_2):
        assert np.abs(o + o.transpose(1, 0, 2, 3)).max() < 1e-13
        assert np.abs(o + o.transpose(0, 1, 3, 2)).max() < 1e-13


def test_first_order_closed_forms():
    """The generic [H(0), A(1)] reproduces the paper's closed forms: the two-body
    non-diagonal H~(1) is v (1 + exp(-s D^2)) and the one-body one is
    (sum_ux D^x_u t^iu_ax gamma^x_u) exp(-s D^2) for f(1) = 0 (Sec. III)."""
    p = _micro(1, 2, 3, 10, seed=37, s=0.8)
    sp = Spaces(1, 2, 3)
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    eps = so_energies(sp, p.eps)
    v = so_integrals(sp, p.B)
    m1, m2 = dsrg._internal_mask(sp)
    t1, t2 = dsrg.amplitudes(sp, eps, dens.gamma, p.s, np.zeros((n, n)), v, m1, m2)
    a1, a2 = dsrg.anti_hermitian(t1, t2)
    _, y1, y2p = gno.commutator((0.0, np.diag(eps), None), gno.to_plain(0.0, a1, a2), dens,
                                want1=(sp.G, sp.G), want2=(sp.G,) * 4)
    y2 = gno.c_from_plain2(y2p)
    D1, D2 = dsrg.denominators(eps)
    e2f = np.exp(-p.s * D2 ** 2)
    ht2 = 2.0 * v + y2
    np.testing.assert_allclose(np.where(m2, ht2, 0.0), np.where(m2, v * (1.0 + e2f), 0.0),
                               atol=1e-14)
    A = sp.A
    coup = np.einsum("axiu,ux,xu->ai", t2[:, A, :, A], eps[None, A] - eps[A, None],
                     dens.gamma[A, A])
    np.testing.assert_allclose(np.where(m1, y1, 0.0),
                               np.where(m1, coup * np.exp(-p.s * D1 ** 2), 0.0), atol=1e-14)


def test_second_order_source_closed_form():
    """[H(0), A(2)] + 1/2 O1 on the non-diagonal block equals the second-order source
    v(2) exp(-s D^2) (two-body) and (f(2) + sum D t(2) gamma) exp(-s D^2) (one-body):
    the 'analogous' expressions of Eqs. T1_2nd and T2_2nd."""
    p = _micro(1, 2, 2, 8, seed=41, s=0.9)
    r = dsrg.run(p)
    sp = r.sp
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    H, P, A = sp.H, sp.P, sp.A
    a1, a2 = dsrg.anti_hermitian(r.t1_2, r.t2_2)
    _, w1, w2p = gno.commutator((0.0, np.diag(r.eps), None), gno.to_plain(0.0, a1, a2), dens,
                                want1=(P, H), want2=(P, P, H, H))
    lhs2 = gno.c_from_plain2(w2p) + 0.5 * r.o1_2
    lhs1 = w1 + 0.5 * r.o1_1
    m1, m2 = dsrg._internal_mask(sp)
    D1, D2 = dsrg.denominators(r.eps)
    rhs2 = 0.5 * r.o1_2 * np.exp(-p.s * D2[P, P, H, H] ** 2)
    coup = np.einsum("axiu,ux,xu->ai", r.t2_2[:, A, :, A], r.eps[None, A] - r.eps[A, None],
                     dens.gamma[A, A])
    rhs1 = (0.5 * r.o1_1 + coup[P, H]) * np.exp(-p.s * D1[P, H] ** 2)
    mm2 = m2[P, P, H, H]
    mm1 = m1[P, H]
    assert np.abs(np.where(mm2, lhs2 - rhs2, 0.0)).max() < 1e-14
    assert np.abs(np.where(mm1, lhs1 - rhs1, 0.0)).max() < 1e-14


def test_spin_flip_and_orbital_permutation_invariance():
    """Swapping alpha and beta (CI transpose, n_alpha = n_beta) and permuting orbitals
    inside a block leave the energies unchanged."""
    p = make_problem(1, 2, 3, 10, seed=43, s=0.5)
    r = dsrg.run(p)
    g1, g2, g3 = synth.active_rdms(p.ci.T.copy(), p.n_active, p.n_beta, p.n_alpha)
    q = Problem(p.n_core, p.n_active, p.n_virtual, p.n_aux, p.eps, p.B, g1, g2, g3, p.s)
    rq = dsrg.run(q)
    assert abs(rq.e2 - r.e2) < 1e-13 and abs(rq.e3 - r.e3) < 1e-13
    perm = np.arange(p.N)
    perm[p.n_hole:] = p.n_hole + np.array([2, 0, 1])
    q2 = Problem(p.n_core, p.n_active, p.n_virtual, p.n_aux, p.eps[perm],
                 p.B[:, perm][:, :, perm], p.gamma1, p.gamma2, p.gamma3, p.s)
    r2 = dsrg.run(q2)
    assert abs(r2.e2 - r.e2) < 1e-13 and abs(r2.e3 - r.e3) < 1e-13


def test_pair_energies_partition_e3():
    """The core-pair parts of E(3) and the rest add up to E(3) (the amplitudes of the two
    final commutators are split into disjoint parts, Eq. E(3) is linear in them)."""
    p = _micro(3, 1, 3, 10, seed=29)
    pairs, rest, r = dsrg.pair_energies(p)
    assert len(pairs) == 6
    total = sum(pairs.values()) + rest
    assert abs(total - r.e3) <= 1e-12 * max(1.0, abs(r.e3))
    assert all(v != 0.0 for v in pairs.values())


def test_pair_energies_follow_core_permutation():
    """Relabelling the core orbitals relabels the pairs: e'_{pi(i) pi(j)} = e_{ij}."""
    p = _micro(3, 1, 3, 10, seed=31)
    perm = np.array([2, 0, 1])               # new core orbital k is old orbital perm[k]
    N = p.N
    full = np.concatenate([perm, np.arange(3, N)])
    q = dataclasses.replace(p, eps=p.eps[full], B=p.B[:, full][:, :, full])
    a, rest_a, _ = dsrg.pair_energies(p)
    b, rest_b, _ = dsrg.pair_energies(q)
    assert abs(rest_a - rest_b) <= 1e-12 * max(1.0, abs(rest_a))
    for (i, j), v in b.items():
        key = tuple(sorted((int(perm[i]), int(perm[j]))))
        assert abs(v - a[key]) <= 1e-12 * max(1.0, abs(v)), ((i, j), key)


# ---------------------------------------------------------------------------
# The integral builder and the multireference projection, pinned in Fock space
# ---------------------------------------------------------------------------
def _so_map(nC, nA, nV):
    """Spin-orbital index of (spatial p, spin sigma) in the space-major layout
    [core a | core b | active a | active b | virtual a | virtual b], written out here
    independently of the oracle's own layout helper."""
    idx = {}
    k = 0
    for off, n in ((0, nC), (nC, nA), (nC + nA, nV)):
        for sigma in (0, 1):
            for p in range(off, off + n):
                idx[(p, sigma)] = k
                k += 1
    return idx


def test_so_integrals_against_chemists_operator():
    """The two-electron operator written straight from the factorised chemists' integrals
    (Eq. int_fact), 1/2 sum_{pqrs} sum_{sigma tau} (pq|rs) a+_{p sigma} a+_{r tau} a_{s tau}
    a_{q sigma}, with explicit loops over spatial orbitals and spins, has the same Fock-space
    matrix as 1/4 sum <pq||rs> a+_p a+_q a_s a_r built from the oracle's antisymmetrised
    integrals.  A misplaced index in <pq||rs> (e.g. (pq|rs) - (pq|sr)) changes the matrix."""
    nC, nA, nV, M = 1, 1, 2, 5
    p = make_problem(nC, nA, nV, M, seed=61)
    N = nC + nA + nV
    eri = np.einsum("Qpq,Qrs->pqrs", p.B, p.B)       # (pq|rs), chemists' order
    so = _so_map(nC, nA, nV)
    n = 2 * N
    fs = FockSpace(n)
    rng = np.random.default_rng(62)
    vecs = rng.standard_normal((3, fs.dim))
    # explicit operator: accumulate its action on the test vectors
    lhs = np.zeros_like(vecs)
    for P_ in range(N):
        for Q_ in range(N):
            for R_ in range(N):
                for S_ in range(N):
                    g = 0.5 * eri[P_, Q_, R_, S_]
                    for sig in (0, 1):
                        for tau in (0, 1):
                            cp, cr = fs.cre[so[(P_, sig)]], fs.cre[so[(R_, tau)]]
                            as_, aq = fs.ann[so[(S_, tau)]], fs.ann[so[(Q_, sig)]]
                            for k in range(len(vecs)):
                                lhs[k] += g * (cp @ (cr @ (as_ @ (aq @ vecs[k]))))
    sp = Spaces(nC, nA, nV)
    v = so_integrals(sp, p.B)
    # 1/4 v[p,q,r,s] a+p a+q a_s a_r in the plain order a+p a+q a_r' a_s' of FockSpace.apply
    K2 = 0.25 * v.transpose(0, 1, 3, 2)
    rhs = np.array([fs.apply((0.0, None, K2), x) for x in vecs])
    assert np.abs(lhs).max() > 1e-3
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(lhs).max()


@pytest.mark.parametrize("nC,nA,nV,seed", [(1, 3, 1, 71), (0, 4, 1, 72)])
def test_multireference_projection_in_fock_space(nC, nA, nV, seed):
    """The oracle's bare -> GNO projection of rank-3 and rank-2 bare operators (scalar,
    one- and two-body parts; the "1,2" truncation of Sec. II.A) obeys the operator identity
        R3 + R2 = c0 + {c1} + {c2} + {R3}
    in the full Fock space of a correlated CAS reference (non-zero two- and three-body
    cumulants), with every normal product built recursively from brute-force reference
    expectation values; and <psi0|{R3}|psi0> = 0.  Weighting the two-index removals of the
    rank-3 part by gamma ^ gamma instead of the full two-body density (dropping lambda2), or
    a wrong sign in any branch, breaks the identity."""
    p = make_problem(nC, nA, nV, 6, seed=seed)
    sp = Spaces(nC, nA, nV)
    n = 2 * sp.N
    fs = FockSpace(n)
    psi0 = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    assert np.abs(dens.L2).max() > 1e-2 and np.abs(dens.L3).max() > 1e-2
    rng = np.random.default_rng(seed + 1)
    # sparse random bare operators: rank-3 strings mostly over the hole space, where the
    # reference densities are non-zero, and a few rank-2 strings
    H = list(range(2 * sp.nH))
    G_ = list(range(n))
    K3 = np.zeros((n,) * 6)
    strings3 = []
    for _ in range(24):
        pick = lambda: int(rng.choice(H)) if rng.random() < 0.8 else int(rng.choice(G_))
        c = [pick() for _ in range(3)]
        a = [pick() for _ in range(3)]
        val = rng.standard_normal()
        K3[tuple(c + a)] += val
        strings3.append((c, a, val))
    K2 = np.zeros((n,) * 4)
    strings2 = []
    for _ in range(8):
        c = [int(rng.choice(H)) for _ in range(2)]
        a = [int(rng.choice(H)) for _ in range(2)]
        val = rng.standard_normal()
        K2[tuple(c + a)] += val
        strings2.append((c, a, val))
    G, Hs = slice(0, n), slice(0, 2 * sp.nH)
    c0, c1, c2 = _project([], [Term(1.0, [(K2, "abcd")], "abcd")],
                          [Term(1.0, [(K3, "abcdef")], "abcdef")], dens, True,
                          (G, G), (G, G, G, G), G, Hs)
    # test vectors: the reference and random vectors in its particle-number sector
    ne = 2 * nC + p.n_alpha + p.n_beta
    sector = fs.number_sector(ne)
    tests = [psi0]
    for _ in range(2):
        x = np.zeros(fs.dim)
        x[sector] = rng.standard_normal(len(sector))
        tests.append(x)
    for x in tests:
        memo = {}
        lhs = np.zeros(fs.dim)
        for c, a, val in strings3 + strings2:
            lhs += val * _fock_string(fs, c, a, x)
        rhs = c0 * x
        for (i, j) in zip(*np.nonzero(np.abs(c1) > 0)):
            rhs += c1[i, j] * _normal_product_action(fs, psi0, [i], [j], x, memo)
        for idx in zip(*np.nonzero(np.abs(c2) > 0)):
            rhs += c2[idx] * _normal_product_action(fs, psi0, list(idx[:2]), list(idx[2:]), x, memo)
        r3 = np.zeros(fs.dim)
        for c, a, val in strings3:
            r3 += val * _normal_product_action(fs, psi0, c, a, x, memo)
        rhs += r3
        if x is psi0:
            assert abs(psi0 @ r3) < 1e-12
        assert np.abs(lhs).max() > 1e-3
        assert np.abs(lhs - rhs).max() < 1e-11 * max(1.0, np.abs(lhs).max())


# ---------------------------------------------------------------------------
# Inter-block Fock elements f(1) (H(1) = f(1) + V)
# ---------------------------------------------------------------------------
def test_e2_with_fock_offdiag_matches_fock_space():
    """With f(1): E^(2) = <Psi0|[H~(1), T(1)]|Psi0>, H~(1) = 2 (f(1) + V) + [H(0), A(1)],
    every operator a brute-force Fock-space matrix."""
    p = make_problem(1, 2, 3, 10, seed=81, s=0.6, f_sigma=0.08)
    r = dsrg.run(p)
    sp = r.sp
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    fs = FockSpace(2 * sp.N)
    vec = reference_vector(sp, p.ci, p.n_alpha, p.n_beta, fs)
    v = so_integrals(sp, p.B)
    # f(1) over spin orbitals written out here: equal spins, inter-block spatial elements
    so = _so_map(sp.nC, sp.nA, sp.nV)
    blk = [0] * sp.nC + [1] * sp.nA + [2] * sp.nV
    f_so = np.zeros((2 * sp.N, 2 * sp.N))
    for P_ in range(sp.N):
        for Q_ in range(sp.N):
            if blk[P_] != blk[Q_]:
                for sig in (0, 1):
                    f_so[so[(P_, sig)], so[(Q_, sig)]] = p.f_offdiag[P_, Q_]
    H1 = gno.gno_to_bare(gno.to_plain(0.0, f_so, v), dens)
    F0 = gno.gno_to_bare((0.0, np.diag(r.eps), None), dens)
    a1, a2 = dsrg.anti_hermitian(r.t1_1, r.t2_1)
    A1 = gno.gno_to_bare(gno.to_plain(0.0, a1, a2), dens)
    T1 = gno.gno_to_bare(gno.to_plain(0.0, r.t1_1, r.t2_1), dens)

    def Ht(x):
        return 2.0 * fs.apply(H1, x) + fs.apply(F0, fs.apply(A1, x)) - fs.apply(A1, fs.apply(F0, x))
    e2 = vec @ Ht(fs.apply(T1, vec)) - vec @ fs.apply(T1, Ht(vec))
    r0 = dsrg.run(dataclasses.replace(p, f_offdiag=None))
    assert abs(e2 - r0.e2) > 1e-4           # f(1) matters
    assert abs(e2 - r.e2) < 1e-12


@pytest.mark.parametrize("nC,nV,seed", [(2, 3, 85), (1, 4, 86)])
def test_single_reference_infinite_s_with_fock_offdiag_is_mp2_mp3(nC, nV, seed):
    """n_A = 0, s -> infinity, f(1) on the core-virtual block: E^(2) and E^(3) equal second-
    and third-order Rayleigh-Schroedinger energies (singles included) from brute force in
    the determinant basis, with H0 = sum_p eps_p n_p and V = f(1) + the normal-ordered
    two-electron operator."""
    p = make_problem(nC, 0, nV, 9, seed=seed, s=float("inf"), f_sigma=0.1)
    r = dsrg.run(p)
    sp = Spaces(nC, 0, nV)
    n = 2 * sp.N
    dens = build_densities(sp, None, None, None)
    fs = FockSpace(n)
    eps = so_energies(sp, p.eps)
    v = so_integrals(sp, p.B)
    so = _so_map(nC, 0, nV)
    f_so = np.zeros((n, n))
    for P_ in range(sp.N):
        for Q_ in range(sp.N):
            if (P_ < nC) != (Q_ < nC):
                for sig in (0, 1):
                    f_so[so[(P_, sig)], so[(Q_, sig)]] = p.f_offdiag[P_, Q_]
    basis = sector_basis(fs, sp, nC, nC)
    ref = list(basis).index(sum(1 << k for k in range(2 * nC)))
    V = fs.matrix(gno.gno_to_bare(gno.to_plain(0.0, f_so, v), dens), basis)
    occ = np.array([[(st >> k) & 1 for k in range(n)] for st in basis])
    h0 = occ @ eps
    E1, E2, E3 = rspt_energies(h0, V, ref)
    assert abs(E1) < 1e-15
    r0 = dsrg.run(dataclasses.replace(p, f_offdiag=None))
    assert abs(r.e2 - r0.e2) > 1e-4 and abs(r.e3 - r0.e3) > 1e-5
    assert abs(r.e2 - E2) < 1e-14 and abs(r.e3 - E3) < 1e-14


def test_first_order_closed_forms_with_fock_offdiag():
    """With f(1) the non-diagonal one-body H~(1) is f + (f + sum_ux D^x_u t^iu_ax gamma^x_u)
    exp(-s D^2) and t^i_a = (f + sum ...) R_s(D) (Eq. T1_1st and Sec. III)."""
    p = make_problem(1, 2, 3, 10, seed=87, s=0.8, f_sigma=0.1)
    sp = Spaces(1, 2, 3)
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    r = dsrg.run(p, keep_ops=True)
    eps = r.eps
    A = sp.A
    coup = np.einsum("axiu,ux,xu->ai", r.t2_1[:, A, :, A], eps[None, A] - eps[A, None],
                     dens.gamma[A, A])
    f_so = dsrg.so_fock_offdiag(sp, p.f_offdiag)
    m1, _ = dsrg._internal_mask(sp)
    D1, _ = dsrg.denominators(eps)
    Rs = np.where(D1 != 0, -np.expm1(-p.s * D1 ** 2) / np.where(D1 != 0, D1, 1.0), 0.0)
    np.testing.assert_allclose(np.where(m1, r.t1_1, 0.0), np.where(m1, (f_so + coup) * Rs, 0.0),
                               atol=1e-15)
    ht1 = r.ops["Ht1"][1]          # plain-order one-body part of H~(1)
    np.testing.assert_allclose(np.where(m1, ht1, 0.0),
                               np.where(m1, f_so + (f_so + coup) * np.exp(-p.s * D1 ** 2), 0.0),
                               atol=1e-14)


@pytest.mark.parametrize("nA,na,nb,seed", [(3, 2, 1, 1), (4, 2, 2, 2), (5, 3, 2, 3)])
def test_active_rdm_blocks_match_generator(nA, na, nb, seed):
    """The oracle's CAS densities (brute force in the Fock space of the active spin orbitals)
    equal the input generator's (Gram matrices of annihilated vectors): two constructions of
    the same expectation values, and the layout of the spin blocks."""
    rng = np.random.default_rng(seed)
    ci = synth.random_ci(rng, nA, na, nb)
    from oracle.hilbert import active_rdm_blocks
    a = active_rdm_blocks(ci, nA, na, nb)
    b = synth.active_rdms(ci, nA, na, nb)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-14

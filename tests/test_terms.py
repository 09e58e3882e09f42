"""The library's derived working equations against the oracle (CPU only).

* the spin-orbital MK-GNO commutator terms derived by ``gen_terms.py`` reproduce the
  oracle's definition-level commutator engine for every operator rank pair;
* the committed spin-integrated table, executed step by step in NumPy, reproduces the
  oracle's E^(2), E^(3) and intermediates.
"""
import importlib.util
import os

import numpy as np
import pytest

from paper_1701_02011_amd.synth import make_problem, make_config
from oracle import dsrg, gno
from oracle.spaces import Spaces, build_densities

import table_emulator
from table_emulator import load_table, pipeline

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gen():
    spec = importlib.util.spec_from_file_location(
        "gen_terms", os.path.join(ROOT, "paper_1701_02011_amd", "csrc", "gen_terms.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_derived_commutator_matches_engine():
    gen = _gen()
    so = gen.spin_orbital_terms()
    p = make_problem(1, 3, 2, 8, seed=7)
    sp = Spaces(1, 3, 2)
    n = 2 * sp.N
    dens = build_densities(sp, p.gamma1, p.gamma2, p.gamma3)
    rng = np.random.default_rng(2)
    X2 = rng.standard_normal((n,) * 4)
    X2 = X2 - X2.transpose(1, 0, 2, 3); X2 = X2 - X2.transpose(0, 1, 3, 2)
    X2 = X2 + X2.transpose(2, 3, 0, 1)
    X1 = rng.standard_normal((n, n)); X1 = X1 + X1.T
    m1, m2 = dsrg._internal_mask(sp)
    T2 = rng.standard_normal((n,) * 4)
    T2 = T2 - T2.transpose(1, 0, 2, 3); T2 = T2 - T2.transpose(0, 1, 3, 2)
    T2 = np.where(m2, T2, 0.0)
    T1 = np.where(m1, rng.standard_normal((n, n)), 0.0)
    A = sp.A
    gA = np.zeros((n, n)); gA[A, A] = dens.gamma[A, A]
    eA = np.zeros((n, n)); eA[A, A] = np.eye(2 * sp.nA) - dens.gamma[A, A]
    L2 = np.zeros((n,) * 4); L2[A, A, A, A] = dens.L2
    L3 = np.zeros((n,) * 6); L3[A, A, A, A, A, A] = dens.L3
    env = dict(X=X2, X1=X1, T=T2, T1=T1, gA=gA, eA=eA,
               L2=L2.transpose(0, 1, 3, 2), L3=L3.transpose(0, 1, 2, 5, 4, 3))
    G = slice(0, n)
    for (rx, rt), terms in so.items():
        Xop = (0.0, X1, None) if rx == 1 else (0.0, None, 0.25 * X2.transpose(0, 1, 3, 2))
        Top = (0.0, T1, None) if rt == 1 else (0.0, None, 0.25 * T2.transpose(0, 1, 3, 2))
        c0, c1, c2 = gno.commutator(Xop, Top, dens, want0=True, want1=(G, G), want2=(G, G, G, G))
        w = {0: 0.0, 1: np.zeros((n, n)), 2: np.zeros((n,) * 4)}
        for coef, fac, out in terms:
            spec = ",".join(l for _, l in fac) + "->" + out
            w[len(out) // 2] = w[len(out) // 2] + coef * np.einsum(spec, *[env[k] for k, _ in fac])
        assert abs(w[0] - c0) < 1e-11 * max(1.0, abs(c0))
        if c1 is not None:
            assert np.abs(w[1] - c1).max() < 1e-11 * max(1.0, np.abs(c1).max())
        if c2 is not None:
            d = gno.c_from_plain2(w[2]) - gno.c_from_plain2(c2)
            assert np.abs(d).max() < 1e-11 * max(1.0, np.abs(c2).max())


def test_committed_table_is_current():
    """dsrg_terms.inc is what gen_terms.py produces now."""
    gen = _gen()
    import tempfile
    _, tables = gen.build_tables()
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "t.inc")
        gen.emit(tables, path)
        assert open(path).read() == open(os.path.join(
            ROOT, "paper_1701_02011_amd", "csrc", "dsrg_terms.inc")).read()


@pytest.mark.parametrize("shape,seed,s", [((1, 2, 3, 10), 11, 0.5), ((1, 3, 2, 8), 7, 0.6),
                                          ((2, 2, 4, 9), 5, 1.3), ((2, 0, 4, 9), 17, 0.4),
                                          ((0, 3, 3, 7), 19, 0.8)])
def test_table_pipeline_matches_oracle(shape, seed, s):
    p = make_problem(*shape, seed=seed, s=s)
    e = pipeline(p, load_table())
    r = dsrg.run(p)
    assert abs(e["e2"] - r.e2) < 1e-12 * max(1.0, abs(r.e2))
    assert abs(e["e3"] - r.e3) < 1e-12 * max(1.0, abs(r.e3))
    assert abs(e["e3a"] - r.e3_a) < 1e-12 * max(1.0, abs(r.e3_a))


def test_table_pipeline_tiny_config():
    p = make_config("tiny")
    e = pipeline(p, load_table())
    r = dsrg.run(p)
    assert abs(e["e2"] - r.e2) < 1e-12 * max(1.0, abs(r.e2))
    assert abs(e["e3"] - r.e3) < 1e-12 * max(1.0, abs(r.e3))


@pytest.mark.parametrize("shape,seed,s", [((2, 2, 10, 40), 101, 0.5), ((3, 1, 5, 12), 23, 0.5),
                                          ((2, 2, 4, 9), 5, 1.3), ((2, 0, 4, 9), 17, 0.4)])
def test_pair_use_matches_oracle(shape, seed, s):
    """The library's derived pair use (C0 products differentiated by their doubles
    factor, core holes only), run by the emulator, gives the oracle's core-pair parts."""
    p = make_problem(*shape, seed=seed, s=s)
    e = pipeline(p)
    pairs, rest, r = dsrg.pair_energies(p)
    scale = max(1.0, max(abs(v) for v in pairs.values()))
    for k, v in pairs.items():
        assert abs(e["pairs"][k] - v) <= 1e-12 * scale, k
    assert abs(e["pair_rest"] - rest) <= 1e-12 * max(1.0, abs(rest))


def test_merged_products_give_the_same_commutators():
    """Products that read the same arrays (the beta doubles are the alpha ones in the first
    order; the first-order doubles are antisymmetric (same spin) or symmetric under the
    exchange of both pairs (opposite spin)) are computed once for all their scatters: the
    commutators W and Z, and so E(3), are unchanged."""
    p = make_problem(2, 2, 4, 9, seed=5, s=1.3)
    uses = table_emulator.load_table()
    ident = {("T2", "bb"): ("T2", "aa"), ("E2", "bb"): ("E2", "aa"), ("Y2", "bb"): ("Y2", "aa"),
             ("E1", "a"): ("Y1", "a"), ("E1", "b"): ("Y1", "b")}
    sym = {("T2", "aa"): 1, ("T2", "ab"): 2}
    merged = dict(uses)
    for name in ("W", "Z"):
        merged[name] = table_emulator.merge_equal(uses[name], ident, sym)
    assert len(merged["W"]) <= len(uses["W"]) - 30
    a = table_emulator.pipeline(p, uses)
    b = table_emulator.pipeline(p, merged)
    for k in ("aa", "ab", "bb"):
        assert np.abs(a["O2"][k] - b["O2"][k]).max() <= 1e-12 * max(1.0, np.abs(a["O2"][k]).max()), k
    assert abs(a["e3"] - b["e3"]) <= 1e-12 * max(1.0, abs(a["e3"]))


def test_collapsed_antisymmetriser_images_give_the_same_commutators():
    """Four scatters forming the pair-antisymmetriser images of one product collapse into
    one scatter into a pre-image, added as A(pre-image) afterwards: W and Z unchanged."""
    p = make_problem(2, 2, 4, 9, seed=5, s=1.3)
    uses = table_emulator.load_table()
    a = table_emulator.pipeline(p, uses)
    collapsed = {}
    for name in ("W", "Z"):
        prods = uses[name]
        col = table_emulator.collapse_images(prods, {"O2"})
        n_before = sum(len(x[3]) for x in prods)
        n_after = sum(len(x[3]) for x in col)
        assert n_after <= n_before - 3 * 30, (name, n_before, n_after)
        collapsed[name] = col
    # run with pre-images: the O2 outputs gain blocks "aa~", "ab~", "bb~" that are added
    # into their blocks through the antisymmetriser after the use
    orig_run_use = table_emulator.run_use

    def run_use_collapsed(prods, dd, B, tens, outs):
        if outs is None or not any(x[3] and any(bl.endswith("~") for _, _, bl, _ in x[3]) for x in prods):
            return orig_run_use(prods, dd, B, tens, outs)
        pre = {k + "~": np.zeros_like(v) for k, v in outs["O2"].items()}
        outs["O2"].update(pre)
        e = orig_run_use(prods, dd, B, tens, outs)
        for k in list(pre):
            outs["O2"][k[:-1]] += table_emulator.antisym(outs["O2"].pop(k))
        return e

    table_emulator.run_use = run_use_collapsed
    try:
        b = table_emulator.pipeline(p, dict(uses, W=collapsed["W"], Z=collapsed["Z"]))
    finally:
        table_emulator.run_use = orig_run_use
    for k in ("aa", "ab", "bb"):
        assert np.abs(a["O2"][k] - b["O2"][k]).max() <= 1e-12 * max(1.0, np.abs(a["O2"][k]).max()), k
    assert abs(a["e3"] - b["e3"]) <= 1e-12 * max(1.0, abs(a["e3"]))


@pytest.mark.parametrize("shape,seed,s", [((1, 2, 3, 10), 11, 0.6), ((1, 3, 2, 8), 7, 0.6),
                                          ((2, 2, 4, 9), 5, 1.3), ((0, 3, 3, 7), 19, 0.8),
                                          ((1, 4, 2, 8), 3, 0.5), ((2, 0, 4, 9), 17, 0.4)])
def test_relaxation_steps_match_oracle(shape, seed, s):
    """The library's relaxation steps (use R on H~(1), H~(2)_{1,2} and both orders of
    amplitudes, spin-blocked de-normal ordering, Slater-Condon determinant matrix), run by
    the emulator, give the oracle's active blocks of Hbar^[3]_{1,2}, CAS constant and
    relaxed energy (Sec. II.B Eq. E_relaxed; App. A)."""
    from oracle import relax
    p = make_problem(*shape, seed=seed, s=s)
    e = pipeline(p)
    r = table_emulator.relaxation(p, e)
    o = relax.relaxed_energy(p)
    assert abs(r["lam"] - o.e_relaxed) < 1e-12 * max(1.0, abs(o.e_relaxed))
    nA = p.n_active
    if nA == 0:
        return
    a, b = slice(0, nA), slice(nA, 2 * nA)
    hb = o.hbar
    for k, sl in (("a", a), ("b", b)):
        assert np.abs(r["h1"][k] - hb.h1[sl, sl]).max() < 1e-12
    for k, (x, y) in (("aa", (a, a)), ("ab", (a, b)), ("bb", (b, b))):
        assert np.abs(r["h2"][k] - hb.h2[x, y, x, y]).max() < 1e-12
    assert abs(r["const"] - o.const) < 1e-12

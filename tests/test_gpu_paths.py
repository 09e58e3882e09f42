"""GPU parity of the paths and inputs the main workloads do not reach: active spaces of
7 and 8 orbitals, a single-determinant reference, gamma3 = NULL, the unregularised
limit, inter-block Fock elements f(1), the paths the medium workload takes (forced on
the small one through workspace_cap, virt_batch and the grouping flag), and the
device-side input checks.  Every energy is compared with the FP64 oracle (or the stored
oracle values of the small workload) at 1e-10 relative, the bar of the other parity
tests."""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_1701_02011_amd import _lib, synth
from paper_1701_02011_amd.synth import make_problem, make_config
from oracle import dsrg

from blocks import oracle_blocks

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _close(x, ref, rel=1e-10):
    return abs(x - ref) <= rel * max(1.0, abs(ref))


def _check_oracle(p, g=None, rel=1e-10):
    g = g or _lib.dsrg_pt3_energy(p)
    r = dsrg.run(p)
    for k, ref in (("e2", r.e2), ("e3_a", r.e3_a), ("e3_b", r.e3_b)):
        assert _close(g[k], ref, rel), (k, g[k], ref)
    return g, r


@pytest.mark.parametrize("shape,seed", [((1, 7, 1, 5), 41), ((1, 8, 1, 4), 41), ((0, 8, 2, 5), 43)])
def test_large_active_micro_energies(shape, seed):
    """CAS(7,7) and CAS(8,8): the three-body cumulant over (2 nA)^6 elements, the singles
    kernel with up to 64 lanes of active terms and the density expansion at nA = 7, 8."""
    p = make_problem(*shape, seed=seed, s=0.5)
    say("large active micro", shape)
    _check_oracle(p)


def test_single_determinant_reference():
    """A CAS vector with one determinant: the cumulants vanish on both sides."""
    nA, na, nb = 4, 2, 2
    base = make_problem(1, nA, 3, 8, seed=51, s=0.7)
    ci = np.zeros((math.comb(nA, na), math.comb(nA, nb)))
    ci[2, 4] = 1.0
    g1, g2, g3 = synth.active_rdms(ci, nA, na, nb)
    p = synth.Problem(1, nA, 3, 8, base.eps, base.B, g1, g2, g3, 0.7, ci=ci, n_alpha=na, n_beta=nb)
    say("single determinant")
    _check_oracle(p)


def test_gamma3_null():
    """gamma3 = NULL sets lambda3 = 0 on both sides (an approximation the ABI allows)."""
    p = make_problem(1, 3, 3, 8, seed=53, s=0.6, with_gamma3=False)
    say("gamma3 null")
    g, _ = _check_oracle(p)
    full = _lib.dsrg_pt3_energy(make_problem(1, 3, 3, 8, seed=53, s=0.6))
    assert g["e2"] != full["e2"]        # lambda3 enters E(2)


@pytest.mark.parametrize("shape,seed", [((2, 0, 4, 9), 17), ((3, 0, 5, 12), 23)])
def test_infinite_s_single_reference(shape, seed):
    """s = +inf, nA = 0: the unregularised limit (E(2), E(3) = MP2, MP3 in the oracle's pins)."""
    p = make_problem(*shape, seed=seed, s=float("inf"))
    say("s = inf", shape)
    _check_oracle(p)


@pytest.mark.parametrize("shape,seed,s", [((1, 2, 3, 10), 61, 0.5), ((2, 0, 4, 9), 62, float("inf")),
                                          ((0, 3, 3, 7), 63, 0.8), ((2, 2, 10, 40), 64, 0.5)])
def test_fock_offdiag_energies(shape, seed, s):
    """Inter-block Fock elements f(1) (H(1) = f(1) + V): energies against the oracle, and
    they change the energies."""
    p = make_problem(*shape, seed=seed, s=s, f_sigma=0.08)
    say("f(1)", shape, s)
    g, _ = _check_oracle(p)
    g0 = _lib.dsrg_pt3_energy(make_problem(*shape, seed=seed, s=s))
    assert abs(g["e2"] - g0["e2"]) > 1e-6 * max(1.0, abs(g0["e2"]))


def test_fock_offdiag_intermediates_and_replay():
    """With f(1) at the tiny size: every intermediate elementwise against the oracle, and
    device inputs through a recorded plan and its replay give the eager energies."""
    base = make_config("tiny")
    p = make_problem(base.n_core, base.n_active, base.n_virtual, base.n_aux, seed=101, s=0.5, f_sigma=0.1)
    say("f(1) tiny intermediates")
    g = _lib.dsrg_pt3_energy_ex(p)
    r = dsrg.run(p)
    ref = oracle_blocks(r, p)
    for k in ("t1", "t2", "w1", "w2", "z1", "z2", "u1", "u2"):
        scale = max(1.0, np.abs(ref[k]).max())
        assert np.abs(g[k] - ref[k]).max() <= 1e-11 * scale, k
    _lib.release_cache()
    d = _lib.to_device(p)
    first = _lib.dsrg_pt3_energy(d)
    rep = _lib.dsrg_pt3_energy(d)
    assert first["plan"] == 1 and rep["plan"] == 2
    assert rep["e2"] == first["e2"] and rep["e3"] == first["e3"]
    assert _close(rep["e3"], r.e3) and _close(rep["e2"], r.e2)
    _lib.release_cache()


def test_result_fields():
    """e_total = e0 + E(2) + E(3); precision, batch size and the flop count are reported."""
    p = make_config("tiny")
    p.e0 = -75.25
    g = _lib.dsrg_pt3_energy(p)
    assert g["e_total"] == p.e0 + g["e2"] + g["e3"]
    assert g["precision_used"] == 0 and g["virt_batch_used"] == g["ladder_batch"] > 0
    assert g["alg_flops"] == g["gett_flops"] > 0
    g2 = _lib.dsrg_pt2_energy(p)
    assert g2["e_total"] == p.e0 + g2["e2"]
    g1 = _lib.dsrg_pt3_energy(p, precision=1)
    assert g1["precision_used"] == 1


def _small_gold(s=0.5):
    return json.load(open(os.path.join(GOLDEN, "small_s%g.json" % s)))


def test_small_virt_batch_option():
    """virt_batch = 5 at the small size: five values of the first particle index per
    (PP|PP) batch (11 batches, the last ragged); energies against the stored oracle values."""
    p = make_config("small")
    gold = _small_gold()
    say("small virt_batch 5")
    g = _lib.dsrg_pt3_energy(p, virt_batch=5, cache=False)
    assert g["virt_batch_used"] == 5
    for k in ("e2", "e3_a", "e3_b"):
        assert _close(g[k], gold[k]), (k, g[k], gold[k])


@pytest.mark.parametrize("mode", ["waves", "per_launch"])
def test_small_forced_medium_paths(mode):
    """The paths the medium workload takes, forced at the small size and checked against
    the stored oracle values: a workspace_cap that leaves the grouped commutators only part
    of their temporaries (small products in waves, large ones one launch each, ladder
    batches of 3 rows) and one launch per contraction (operand packing, 128 x 128 tiles and
    split-K on the contractions large enough for them).  Deterministic."""
    p = make_config("small")
    gold = _small_gold()
    nP = p.n_active + p.n_virtual
    kp = nP * (nP - 1) // 2
    row = 8 * (nP ** 3 + nP * (2 * kp + nP))
    say("small forced paths", mode)
    if mode == "waves":
        kw = dict(workspace_cap=3 * row, cache=False)
    else:
        kw = dict(grouping=False, cache=False, virt_batch=2)
    a = _lib.dsrg_pt3_energy(p, **kw)
    b = _lib.dsrg_pt3_energy(p, **kw)
    assert a["e3"] == b["e3"] and a["e2"] == b["e2"]
    for k in ("e2", "e3_a", "e3_b"):
        assert _close(a[k], gold[k]), (k, a[k], gold[k])
    full = _lib.dsrg_pt3_energy(p, cache=False)
    if mode == "waves":
        assert a["virt_batch_used"] == 3
        assert 0 < a["grouped_uses"] and a["n_launch"] > full["n_launch"]
    else:
        assert a["grouped_uses"] == 0 and a["virt_batch_used"] == 2


def test_device_density_check():
    """Device densities that break gamma1 symmetry are rejected with DSRG_E_RDM, eagerly and
    on a plan replay (the check runs beside the graph); a clean replay after it is unaffected."""
    p = make_problem(1, 2, 3, 7, seed=2)
    d = _lib.to_device(p)
    say("device density check")
    first = _lib.dsrg_pt3_energy(d)
    d["gamma1"][0, 0, 1] += 1e-3
    with pytest.raises(_lib.DsrgError) as e:
        _lib.dsrg_pt3_energy(d)
    assert e.value.code == _lib.DSRG_E_RDM
    with pytest.raises(_lib.DsrgError) as e:
        _lib.dsrg_pt3_energy(d, cache=False)
    assert e.value.code == _lib.DSRG_E_RDM
    d["gamma1"][0, 0, 1] -= 1e-3
    d["gamma1"][0, 0, 1] = float(p.gamma1[0, 0, 1])
    again = _lib.dsrg_pt3_energy(d)
    assert again["e2"] == first["e2"] and again["e3"] == first["e3"]


@pytest.mark.parametrize("mode", ["resident", "batched"])
def test_cas88_against_block_oracle(mode):
    """CAS(8,8) with 150 virtual orbitals (nP = 158) against the stored block-level oracle
    values: the (PP|PP) block either resident over particle pairs (the default) or built in
    batches of 16 rows (a workspace_cap below the resident block), 128 x 128 tiles on the
    large contractions."""
    with open(os.path.join(GOLDEN, "cas88_s0.5.json")) as f:
        gold = json.load(f)
    # the shape and seed tests/golden/make_golden.py cas88 uses
    p = make_problem(n_core=12, n_active=8, n_virtual=150, n_aux=600, seed=404, s=0.5, name="cas88")
    assert (gold["n_core"], gold["n_active"], gold["n_virtual"], gold["n_aux"]) == (
        p.n_core, p.n_active, p.n_virtual, p.n_aux)
    nP = p.n_active + p.n_virtual
    kp = nP * (nP - 1) // 2
    row = 8 * (nP ** 3 + nP * (2 * kp + nP))
    kw = dict(cache=False) if mode == "resident" else dict(cache=False, workspace_cap=16 * row)
    say("cas88", mode)
    g = _lib.dsrg_pt3_energy(p, **kw)
    if mode == "batched":
        assert g["virt_batch_used"] == 16
    for k in ("e2", "e3_a", "e3_b"):
        assert _close(g[k], gold[k]), (k, g[k], gold[k])

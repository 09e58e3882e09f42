"""The learned part on the GPU: the network's training kernels against the FP64 reference
(tests/mlp_reference.py, itself pinned by finite differences), training behaviour, the
pair features, and the surrogate energy path, whose exact part (the rest of E(3)) is
compared with the oracle's core-pair decomposition."""
import json
import os
import sys
import time

import numpy as np
import pytest

from paper_1701_02011_amd import _lib, surrogate
from paper_1701_02011_amd.synth import make_problem, make_config
from oracle import dsrg

import mlp_reference as ref

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _data(n=300, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 16)) * rng.uniform(0.5, 3.0, 16) + rng.standard_normal(16)
    y = np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2] - 0.2 * X[:, 5] ** 2 + 0.05 * rng.standard_normal(n)
    return X.astype(np.float32), y


def test_gradient_against_reference():
    """Loss and gradient of the training kernels (FP32 sums, BF16-rounded weights) against
    the FP64 reference with the same weights: relative 1e-4 of the largest gradient entry."""
    X, y = _data()
    blob = _lib.dsrg_mlp_train(X, y, epochs=20, seed=5)   # some trained, non-trivial weights
    say("mlp gradient check")
    loss_g, g = _lib.test_mlp_grad(blob, X, y)
    loss_r, gr = ref.loss_grad(blob, X.astype(np.float64), y)
    assert abs(loss_g - loss_r) <= 1e-5 * max(1.0, loss_r), (loss_g, loss_r)
    scale = np.abs(gr).max()
    assert np.abs(g - gr).max() <= 1e-4 * scale, np.abs(g - gr).max() / scale
    # every layer's block is non-trivially checked
    offs, _ = ref.layout()
    for (ow, ob) in offs:
        assert np.abs(gr[ow:ob]).max() > 1e-6 * scale


def test_predict_against_reference():
    X, y = _data(200, 4)
    blob = _lib.dsrg_mlp_train(X, y, epochs=50, seed=2)
    p = _lib.dsrg_mlp_predict(blob, X)
    pr = ref.predict(blob, X.astype(np.float64))
    assert np.abs(p - pr).max() <= 1e-5 * max(1.0, np.abs(pr).max())


def test_training_lowers_loss_and_is_deterministic():
    X, y = _data(400, 6)
    a = _lib.dsrg_mlp_train(X, y, epochs=400, seed=9)
    b = _lib.dsrg_mlp_train(X, y, epochs=400, seed=9)
    assert a == b
    l0, _ = _lib.test_mlp_grad(_lib.dsrg_mlp_train(X, y, epochs=0, seed=9), X, y)
    l1, _ = _lib.test_mlp_grad(a, X, y)
    say("mlp loss", l0, "->", l1)
    assert l1 < 0.3 * l0


def test_pair_features_against_numpy():
    """Features 0, 1, 5 (log |E2_ij|), 13 and 15 and the E2_ij proxy recomputed from B and
    eps one pair at a time (spatial (ai|bj), R_s, exp(-s D^2))."""
    p = make_problem(3, 2, 6, 12, seed=21, s=0.7)
    X, e2 = _lib.dsrg_pair_features(p)
    nC, nA, N = p.n_core, p.n_active, p.N
    P = np.arange(nC, N)
    k = 0
    for i in range(nC):
        for j in range(i, nC):
            V = np.einsum("Qa,Qb->ab", p.B[:, P, i], p.B[:, P, j])
            Xc = V.T
            D = p.eps[i] + p.eps[j] - p.eps[P][:, None] - p.eps[P][None, :]
            R = dsrg.regulariser(p.s, D)
            f = np.exp(-p.s * D ** 2)
            c = 0.5 if i == j else 1.0
            ref_e2 = c * (2 * np.sum(V * V * (1 + f) * R) + (0.0 if i == j else np.sum((V - Xc) ** 2 * (1 + f) * R)))
            assert abs(e2[k] - ref_e2) <= 1e-12 * abs(ref_e2)
            assert X[k, 0] == np.float32(p.eps[i]) and X[k, 1] == np.float32(p.eps[j])
            assert abs(X[k, 5] - np.log(abs(ref_e2))) <= 1e-6
            assert X[k, 13] == (1.0 if i == j else 0.0)
            ijij = np.sum(p.B[:, i, j] ** 2)
            assert abs(X[k, 15] - np.log(ijij)) <= 1e-5
            k += 1


@pytest.mark.parametrize("shape,seed,s", [((3, 1, 5, 12), 23, 0.5), ((2, 2, 10, 40), 101, 0.5),
                                          ((2, 0, 4, 9), 17, 0.4)])
def test_surrogate_exact_parts_against_oracle(shape, seed, s):
    """The surrogate path with every pair computed exactly (rel_threshold 0) gives the exact
    E(3); with none (rel_threshold huge) its exact part, E(3) minus the predicted pair
    parts, is the oracle's rest of the core-pair decomposition."""
    p = make_problem(*shape, seed=seed, s=s)
    say("surrogate exact parts", shape)
    X, y = _data(64, 8)
    blob = _lib.dsrg_mlp_train(X, y, epochs=5, seed=1)    # any weights: only exact parts are checked
    pairs, rest, r = dsrg.pair_energies(p)
    scale = max([1.0, abs(r.e3)] + [abs(v) for v in pairs.values()])
    allx = _lib.dsrg_pt3_energy_surrogate(p, blob, rel_threshold=0.0)
    assert abs(allx["e2"] - r.e2) <= 1e-10 * max(1.0, abs(r.e2))
    assert abs(allx["e3"] - r.e3) <= 1e-10 * scale, (allx["e3"], r.e3)
    none = _lib.dsrg_pt3_energy_surrogate(p, blob, rel_threshold=1e300)
    Xf, e2p = _lib.dsrg_pair_features(p)
    if len(Xf):
        z = (Xf - np.frombuffer(blob, np.float32)[8:24]) / np.frombuffer(blob, np.float32)[24:40]
        if np.abs(z).max() > 8:     # out of the toy training range: the path used exact pairs
            return
        pred = _lib.dsrg_mlp_predict(blob, Xf) * np.abs(e2p) ** 1.5
    else:
        pred = np.zeros(0)
    assert none["n_exact_pairs"] == 0
    assert abs((none["e3"] - pred.sum()) - rest) <= 1e-10 * scale, (none["e3"] - pred.sum(), rest)


def test_surrogate_gain_on_large_workload():
    """The large workload (nC = 43, nA = 2, nV = 185, naux = 920) with the trained network
    (paper_1701_02011_amd/pair_network.bin): time of the surrogate path against the exact
    energy and the error it makes in E(3).  A measurement: it asserts only that both paths
    run and that the exact parts stay exact."""
    if not os.path.exists(surrogate.WEIGHTS):
        pytest.skip("no trained weights (python -m paper_1701_02011_amd.surrogate)")
    blob = open(surrogate.WEIGHTS, "rb").read()
    p = make_config("large")
    d = _lib.to_device(p)
    import torch
    say("surrogate gain: large")
    exact = _lib.dsrg_pt3_energy(d, cache=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    exact = _lib.dsrg_pt3_energy(d, cache=False)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t0
    sur = _lib.dsrg_pt3_energy_surrogate(d, blob, rel_threshold=1e300)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur = _lib.dsrg_pt3_energy_surrogate(d, blob, rel_threshold=1e300)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    out = dict(t_exact=t_exact, t_surrogate=t_sur, e3_exact=exact["e3"], e3_surrogate=sur["e3"],
               abs_dE3=abs(sur["e3"] - exact["e3"]), rel_dE3=abs(sur["e3"] - exact["e3"]) / abs(exact["e3"]),
               n_exact_pairs=sur["n_exact_pairs"], e2_equal=sur["e2"] == exact["e2"])
    say("surrogate gain", json.dumps(out))
    assert np.isfinite(sur["e3"]) and abs(sur["e2"] - exact["e2"]) <= 1e-10 * abs(exact["e2"])

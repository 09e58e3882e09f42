"""Training data and training of the pair-energy network (argument marshalling around the
library's GPU entry points: features, exact pair energies, training kernels).

The network predicts the core-pair parts e3_ij of E(3) (the decomposition of
``dsrg_pt3_pair_energies``) from 16 first-order features of the pair
(``dsrg_pair_features``), as y_ij = e3_ij / |E2_ij|^{3/2}, which B -> kappa B leaves
unchanged.  Training pairs come from synthetic problems of the tiny, small and medium
shapes at s = 0.1, 0.5, 1.0 (seeds 1101-1356, 2201-2264, 3301-3304), validation pairs
from held-out seeds (1401-1432, 2301-2308); targets are the library's exact pair
energies.

    python -m paper_1701_02011_amd.surrogate [--epochs E] [--out PATH]

writes the weights blob (default: paper_1701_02011_amd/pair_network.bin) and a JSON
summary beside it (training and validation R^2, sizes, timings).
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import _lib
from .synth import CONFIGS, make_problem

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "pair_network.bin")
S_VALUES = (0.1, 0.5, 1.0)
TRAIN = (("tiny", range(1101, 1357)), ("small", range(2201, 2265)), ("medium", range(3301, 3305)))
VALID = (("tiny", range(1401, 1433)), ("small", range(2301, 2309)))


def shape_problem(name: str, seed: int, s: float):
    kw = dict(CONFIGS[name])
    kw.pop("seed")
    kw["s"] = s
    return make_problem(seed=seed, name="%s-%d" % (name, seed), **kw)


def pair_rows(p, device=True):
    """(features [npairs][16], targets y_ij, exact e3_ij, E2_ij) of one problem."""
    q = _lib.to_device(p) if device else p
    X, e2 = _lib.dsrg_pair_features(q)
    g = _lib.dsrg_pt3_pair_energies(q)
    nC = p.n_core
    keys = [(i, j) for i in range(nC) for j in range(i, nC)]
    e3 = np.array([g["pairs"][k] for k in keys])
    y = e3 / np.abs(e2) ** 1.5
    return X, y, e3, e2


def dataset(spec, device=True, log=None):
    Xs, ys = [], []
    for name, seeds in spec:
        t = time.time()
        for seed in seeds:
            for s in S_VALUES:
                X, y, _, _ = pair_rows(shape_problem(name, seed, s), device)
                Xs.append(X)
                ys.append(y)
        if log:
            log("%s: %d problems in %.1f s" % (name, len(seeds) * len(S_VALUES), time.time() - t))
    return np.concatenate(Xs), np.concatenate(ys)


def r2(pred, y):
    return 1.0 - float(np.sum((pred - y) ** 2) / np.sum((y - np.mean(y)) ** 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    say = lambda m: print(m, flush=True)
    t0 = time.time()
    Xt, yt = dataset(TRAIN, log=say)
    Xv, yv = dataset(VALID, log=say)
    t1 = time.time()
    blob = _lib.dsrg_mlp_train(Xt, yt, epochs=args.epochs, seed=args.seed)
    t2 = time.time()
    pt = _lib.dsrg_mlp_predict(blob, Xt)
    pv = _lib.dsrg_mlp_predict(blob, Xv)
    summary = dict(train_pairs=len(yt), valid_pairs=len(yv), epochs=args.epochs, seed=args.seed,
                   r2_train=r2(pt, yt), r2_valid=r2(pv, yv), data_seconds=t1 - t0,
                   train_seconds=t2 - t1)
    with open(args.out, "wb") as f:
        f.write(blob)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    say(json.dumps(summary))


if __name__ == "__main__":
    main()

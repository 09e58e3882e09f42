"""Tile autotuner for batches of uneven problems (the synthetic dissociation curve).

For each size class of the particle space n_P = n_active + n_virtual it times one
representative geometry of the 64-point curve under every candidate tile rule (the
large-tile threshold of the contraction launches and the (PP|PP) batch) and keeps the
fastest; the winners are written as the library's rule table (dsrg_set_tile_rules),
which _lib.load_tile_rules() installs.  The timed calls run the pipeline directly (no
cached plan), as a curve does: every geometry has its own shape.

    python -m paper_1701_02011_amd.autotune [--out PATH] [--repeats N]

Needs a GPU; prints one line per trial.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

# size classes of n_P (inclusive bounds) and the candidate settings
CLASSES = [(0, 159), (160, 239), (240, 319), (320, 1 << 30)]
BIG_TILE_MIN = [64, 128, 256, 512, 1 << 30]   # 1 << 30: 64 x 64 tiles only
VIRT_BATCH = [0, 8, 32]                       # 0: the largest batch workspace_cap allows


def representatives(geometries=64):
    """The curve geometry nearest the middle of each class (by n_P), or None."""
    from paper_1701_02011_amd.synth import make_batch_config, batch_sizes
    sizes = [(k, na + nv) for k, (nc, na, nv) in enumerate(batch_sizes(geometries))]
    reps = []
    for lo, hi in CLASSES:
        inside = sorted((nP, k) for k, nP in sizes if lo <= nP <= hi)
        if not inside:
            reps.append(None)
            continue
        nP, k = inside[len(inside) // 2]
        p = make_batch_config(1, first=k)[0]
        assert p.n_active + p.n_virtual == nP
        reps.append(p)
    return reps


def tune(out_path, repeats=3, log=print):
    import torch
    from paper_1701_02011_amd import _lib
    _lib.load()
    rules, trials = [], []
    for (lo, hi), p in zip(CLASSES, representatives()):
        if p is None:
            continue
        d = _lib.to_device(p)
        shape = dict(n_core=p.n_core, n_active=p.n_active, n_virtual=p.n_virtual, n_aux=p.n_aux)
        best = None
        ref = None
        for bt in BIG_TILE_MIN:
            for vb in VIRT_BATCH:
                rule = dict(np_min=lo, np_max=hi, big_tile_min=bt, virt_batch=vb)
                _lib.set_tile_rules([rule])
                try:
                    r = _lib.dsrg_pt3_energy(d, cache=False)      # warm-up
                except _lib.DsrgError as e:
                    if e.code != _lib.DSRG_E_OOM:
                        raise
                    log("class [%d, %d] big_tile_min=%d virt_batch=%d: does not fit workspace_cap"
                        % (lo, hi, bt, vb))
                    continue
                ts = []
                for _ in range(repeats):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r = _lib.dsrg_pt3_energy(d, cache=False)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                t = min(ts)   # direct runs allocate and free their buffers: noisy upwards
                if ref is None:
                    ref = r["e3"]
                rel = abs(r["e3"] - ref) / max(1.0, abs(ref))
                trials.append(dict(rule, seconds=t, shape=shape, e3_rel_change=rel))
                log("class [%d, %d] nP=%d big_tile_min=%d virt_batch=%d: %.1f ms (E3 rel. change %.1e)"
                    % (lo, hi, p.n_active + p.n_virtual, bt, vb, 1e3 * t, rel))
                if best is None or t < best[0]:
                    best = (t, rule)
        rules.append(dict(best[1], seconds=best[0], shape=shape))
        log("class [%d, %d]: big_tile_min=%d virt_batch=%d (%.1f ms)"
            % (lo, hi, best[1]["big_tile_min"], best[1]["virt_batch"], 1e3 * best[0]))
        del d
        torch.cuda.empty_cache()
    _lib.set_tile_rules([])
    props = torch.cuda.get_device_properties(0)
    doc = dict(device=props.name, gcn_arch=getattr(props, "gcnArchName", ""),
               library_version=int(_lib.load().dsrg_version()), repeats=repeats,
               rules=[{k: r[k] for k in ("np_min", "np_max", "big_tile_min", "virt_batch")} for r in rules],
               winners=rules, trials=trials)
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    log("wrote " + out_path)
    return doc


def main():
    from paper_1701_02011_amd import _lib
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=_lib.TILE_RULES_PATH)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args()
    tune(args.out, args.repeats, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()

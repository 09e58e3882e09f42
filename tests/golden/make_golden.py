"""Write oracle energies for workloads too slow to run inside a test.

Calls only ``oracle/`` (and the shared input generator).  Usage:
    python tests/golden/make_golden.py small          # energies and sampled intermediates
    python tests/golden/make_golden.py small-pairs    # core-pair parts of E(3), s = 0.5
    python tests/golden/make_golden.py medium         # energies from the block-sparse DF level
    python tests/golden/make_golden.py large          #   (oracle/dsrg_df.py; hours of CPU)
    python tests/golden/make_golden.py relax          # one-step relaxed energies (oracle/relax.py)
    python tests/golden/make_golden.py cas88          # CAS(8,8) with 150 virtuals, block-sparse DF
    python tests/golden/make_golden.py big-active     # active spaces of 9 to 16 orbitals
    python tests/golden/make_golden.py curve 36       # geometry 36 of the synthetic curve (block level)
Writes tests/golden/<name>_s<s>.json with E(2), E(3) and its two parts (and, for small,
sampled intermediates), or tests/golden/small_pairs_s0.5.json with the core-pair
decomposition of E(3).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1701_02011_amd.synth import make_config, SMALL_S_VALUES  # noqa: E402
from oracle import dsrg  # noqa: E402

sys.path.insert(0, os.path.join(ROOT, "tests"))
from blocks import oracle_blocks  # noqa: E402  (index mapping only)
import numpy as np  # noqa: E402


def samples(r, p, n=400, seed=12345):
    """Seeded random elements of each intermediate, in the library's spin-block layout."""
    rng = np.random.default_rng(seed)
    out = {}
    for k, arr in oracle_blocks(r, p).items():
        flat = rng.choice(arr.size, size=min(n, arr.size), replace=False)
        idx = np.array(np.unravel_index(flat, arr.shape)).T
        out[k] = dict(index=idx.tolist(), value=arr[tuple(idx.T)].tolist(),
                      scale=float(np.abs(arr).max()))
    return out


def main_df(name, shape=None):
    """Workloads beyond the dense engine: the block-sparse, density-fitted level."""
    import platform
    from oracle import dsrg_df
    from paper_1701_02011_amd.synth import make_problem
    p = make_config(name) if shape is None else make_problem(name=name, **shape)
    t = time.time()
    r = dsrg_df.run(p, log=lambda m: print(m, flush=True))
    out = dict(workload=name, s=p.s, n_core=p.n_core, n_active=p.n_active,
               n_virtual=p.n_virtual, n_aux=p.n_aux, e2=r.e2, e3=r.e3, e3_a=r.e3_a,
               e3_b=r.e3_b, oracle_seconds=time.time() - t, stage_seconds=r.seconds,
               host=dict(cpus=os.cpu_count(), machine=platform.machine(),
                         processor=platform.processor()),
               source="oracle/dsrg_df.py (FP64, block-sparse spin orbitals, DF integrals)")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "%s_s%g.json" % (name, p.s))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["e2"], out["e3"], "%.0fs" % out["oracle_seconds"], flush=True)


# CAS(8,8) at a size the block-sparse level finishes in minutes, large enough that the
# library runs its large-problem paths (ungrouped commutators, batched (PP|PP) ladder when
# asked for, 128 x 128 tiles)
CAS88 = dict(n_core=12, n_active=8, n_virtual=150, n_aux=600, seed=404, s=0.5)


# Active spaces beyond 8 orbitals: (name, make_problem arguments, oracle level).  The dense
# engine takes up to 10 active orbitals at these sizes; the block-sparse level goes further.
# The 16-orbital case holds three electrons (two alpha, one beta): a half-filled CAS(16,16)
# vector has 1.7e8 determinants, too many to draw.
BIG_ACTIVE = [("cas9", dict(n_core=0, n_active=9, n_virtual=1, n_aux=4, seed=91), "dense"),
              ("cas10", dict(n_core=1, n_active=10, n_virtual=1, n_aux=6, seed=92), "dense"),
              ("cas12", dict(n_core=1, n_active=12, n_virtual=1, n_aux=6, seed=93), "block"),
              ("cas16_3e", dict(n_core=1, n_active=16, n_virtual=2, n_aux=8, seed=94,
                                n_alpha=2, n_beta=1), "block")]


def main_big_active(only=None):
    """E(2), E(3) for active spaces of 9 to 16 orbitals (s = 0.5)."""
    from oracle import dsrg_df
    from paper_1701_02011_amd.synth import make_problem
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "big_active.json")
    cases = {}
    if os.path.exists(path):
        with open(path) as f:
            cases = {c["name"]: c for c in json.load(f)["cases"]}
    for name, args, level in BIG_ACTIVE:
        if only and name != only:
            continue
        p = make_problem(**args)
        t = time.time()
        r = dsrg.run(p) if level == "dense" else dsrg_df.run(p)
        cases[name] = dict(name=name, args=args, s=p.s, level=level, e2=r.e2, e3=r.e3,
                           e3_a=r.e3_a, e3_b=r.e3_b, oracle_seconds=time.time() - t)
        print(name, r.e2, r.e3, "%.0fs" % cases[name]["oracle_seconds"], flush=True)
        out = dict(cases=[cases[n] for n, _, _ in BIG_ACTIVE if n in cases],
                   source="oracle/dsrg.py (dense) or oracle/dsrg_df.py (block), FP64")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
    print(path, flush=True)


def main_curve(k):
    """One geometry of the 64-point synthetic dissociation curve, block-sparse level."""
    import platform
    from oracle import dsrg_df
    from paper_1701_02011_amd.synth import make_batch_config
    p = make_batch_config(1, first=k)[0]
    t = time.time()
    r = dsrg_df.run(p, log=lambda m: print(m, flush=True))
    out = dict(workload="curve%d" % k, geometry=k, s=p.s, n_core=p.n_core, n_active=p.n_active,
               n_virtual=p.n_virtual, n_aux=p.n_aux, e2=r.e2, e3=r.e3, e3_a=r.e3_a, e3_b=r.e3_b,
               oracle_seconds=time.time() - t,
               host=dict(cpus=os.cpu_count(), machine=platform.machine()),
               source="oracle/dsrg_df.py (FP64, block-sparse spin orbitals, DF integrals)")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "curve%d_s%g.json" % (k, p.s))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["e2"], out["e3"], "%.0fs" % out["oracle_seconds"], flush=True)


def main(name):
    if name in ("medium", "large"):
        return main_df(name)
    if name == "cas88":
        return main_df(name, CAS88)
    svals = SMALL_S_VALUES if name == "small" else (None,)
    for s in svals:
        p = make_config(name, s=s)
        t = time.time()
        r = dsrg.run(p)
        out = dict(workload=name, s=p.s, n_core=p.n_core, n_active=p.n_active,
                   n_virtual=p.n_virtual, n_aux=p.n_aux, e2=r.e2, e3=r.e3, e3_a=r.e3_a,
                   e3_b=r.e3_b, oracle_seconds=time.time() - t,
                   source="oracle/dsrg.py (FP64, spin-orbital, MK-GNO commutator engine)",
                   samples=samples(r, p))
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "%s_s%g.json" % (name, p.s))
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, out["e2"], out["e3"], "%.0fs" % out["oracle_seconds"], flush=True)


def main_pairs():
    p = make_config("small", s=0.5)
    t = time.time()
    pairs, rest, r = dsrg.pair_energies(p)
    out = dict(workload="small", s=p.s, e3=r.e3, rest=rest,
               pairs=[[i, j, v] for (i, j), v in sorted(pairs.items())],
               oracle_seconds=time.time() - t,
               source="oracle/dsrg.py pair_energies (FP64, spin-orbital, MK-GNO engine)")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_pairs_s0.5.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, len(pairs), rest, "%.0fs" % out["oracle_seconds"], flush=True)


# relaxed-energy cases: (name, make_problem arguments or a workload name, s, f_sigma, e0)
RELAX_CASES = [("cas77", dict(n_core=0, n_active=7, n_virtual=1, n_aux=6, seed=41), 0.5, 0.03, -1.5),
               ("cas66", dict(n_core=1, n_active=6, n_virtual=2, n_aux=8, seed=42), 0.5, 0.03, -2.0),
               ("small", "small", 0.5, 0.0, 0.0)]


def relax_problem(case):
    import dataclasses
    from paper_1701_02011_amd.synth import make_problem
    name, args, s, f_sigma, e0 = case
    if isinstance(args, str):
        p = make_config(args, s=s)
    else:
        p = make_problem(s=s, f_sigma=f_sigma, **args)
    return dataclasses.replace(p, e0=e0)


def main_relax():
    """Relaxed energies (Sec. II.B Eq. E_relaxed), the CAS constant, the one-body active block
    of Hbar^[3]_{1,2} and seeded samples of its two-body blocks, in the library's layout."""
    from oracle import relax
    cases = []
    for case in RELAX_CASES:
        p = relax_problem(case)
        t = time.time()
        r = relax.relaxed_energy(p)
        nA = p.n_active
        a, b = slice(0, nA), slice(nA, 2 * nA)
        h1 = np.stack([r.hbar.h1[a, a], r.hbar.h1[b, b]])
        h2 = np.stack([r.hbar.h2[a, a, a, a], r.hbar.h2[a, b, a, b], r.hbar.h2[b, b, b, b]])
        rng = np.random.default_rng(777)
        flat = rng.choice(h2.size, size=min(300, h2.size), replace=False)
        idx = np.array(np.unravel_index(flat, h2.shape)).T
        cases.append(dict(name=case[0], args=case[1], s=case[2], f_sigma=case[3], e0=case[4],
                          e_relaxed=r.e_relaxed, e_unrelaxed=r.e_unrelaxed, cas_const=r.const,
                          hbar1=h1.tolist(), hbar2_index=idx.tolist(),
                          hbar2_value=h2[tuple(idx.T)].tolist(), oracle_seconds=time.time() - t))
        print(case[0], r.e_relaxed, r.e_unrelaxed, "%.0fs" % cases[-1]["oracle_seconds"], flush=True)
    out = dict(cases=cases, source="oracle/relax.py (FP64, spin-orbital, MK-GNO engine, Fock-space CAS)")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "relax.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, flush=True)


if __name__ == "__main__":
    arg = sys.argv[1] if len(sys.argv) > 1 else "small"
    if arg == "small-pairs":
        main_pairs()
    elif arg == "relax":
        main_relax()
    elif arg == "curve":
        main_curve(int(sys.argv[2]))
    elif arg == "big-active":
        main_big_active(sys.argv[2] if len(sys.argv) > 2 else None)
    else:
        main(arg)

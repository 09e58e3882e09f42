#!/usr/bin/env python3
"""DSRG-MRPT3 energies/s on one MI355X, with the roofline of the dominant kernel and the
FP64 CPU oracle timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload small|tiny|medium|large]

One step = one pass of the whole hot path (cumulants, integral blocks, first-order
amplitudes, E(2), [V, A], [Y, A], second-order amplitudes, E(3)) over every problem of
the workload: the "small" workload is CAS(6,6) with nC=5, nV=49, naux=200 at
s = 0.1, 0.5 and 1.0 (three energies per step).  Inputs are resident in device memory
before the timed region; the library runs on torch's current stream.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix = vector)
PEAK_FP32_TFLOPS = 157.3     # MI355X dense FP32 MFMA
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 MFMA
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
METRIC = "DSRG-MRPT3 energies/sec and MFMA TFLOP/s vs peak at |ΔE|≤1e-6 Eh"


def workload_problems(name, geometries=4):
    from paper_1701_02011_amd.synth import make_config, make_batch_config, SMALL_S_VALUES
    if name == "small":
        return [make_config("small", s=s) for s in SMALL_S_VALUES]
    if name == "curve":
        # the first geometries of the 64-point synthetic dissociation curve (uneven sizes,
        # naux = 4N, gaps shrinking with the index)
        return make_batch_config(geometries)
    return [make_config(name)]




def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of the kernel from the committed rocprofv3 counter summaries
    (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or None when no summary
    covers this kernel and workload or the kernel source changed since it was taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1701_02011_amd", "csrc", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.txt")):
        kv = {}
        for line in open(path):
            if ": " in line and not line.startswith(" "):
                k, v = line.rstrip("\n").split(": ", 1)
                kv[k] = v
        if (kv.get("kernel") == kernel and kv.get("workload") == workload and
                kv.get("precision") == precision and kv.get("kernels_hip_sha256") == digest):
            return float(kv["traffic_bytes_per_launch"])
    return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        if n:
            return max(n)
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# kernel instance of each profile bucket (index 2 * role + 128x128-tile flag), FP64 names;
# the last template argument is the waves along m (2: 64 x 64 and 128 x 128 tiles, 4:
# 128 x 32 tiles, which share the bucket of the 64 x 64 ones)
KERNELS = ["gett_f64_kernel<0, 2, 2, 2|4>", "gett_f64_kernel<0, 4, 4, 2>",
           "gett_f64_kernel<1, 2, 2, 2|4>", "gett_f64_kernel<1, 4, 4, 2>",
           "gett_f64_kernel<2, 2, 2, 2|4> / coulomb_group_kernel<0>", "gett_f64_kernel<2, 4, 4, 2>",
           "gett_group_kernel<0>", "gett_group_big_kernel<0>"]
# a "launch" below is one contraction call of the library, timed by HIP events around all
# of its dispatches: a 128 x 128 launch whose last round is mostly empty is the whole rounds
# plus a k-split tail (two dispatches of the kernel and a reduction)
ROLE_NOTES = ["table products, one contraction call each", "(PP|PP) ladder contractions",
              "Coulomb-block builds B.B", "grouped table products"]


def kernel_name(k, prec):
    """Kernel symbol of slot k of the library's per-kernel profile at precision prec
    (0 FP64, 1 FP32 products, 2 split-BF16 x3 products)."""
    n = KERNELS[k]
    if prec:
        n = n.replace("gett_f64", "gett_f32" if prec == 1 else "gett_b3").replace("<0>", "<%d>" % prec)
    return n


def dominant_kernel(prof, prec, step_s):
    """The kernel instance with the most device time in a profiled pass: its algorithmic
    rate (the library's 2 M N K flop count over the HIP-event time of its launches) against
    the MFMA peak of the instruction it issues.  Split BF16 x3 issues three BF16 products
    per product, so its executed rate is three times the algorithmic one."""
    ksec = [sum(r["kernel_seconds"][k] for r in prof) for k in range(8)]
    kfl = [sum(r["kernel_flops"][k] for r in prof) for k in range(8)]
    kn = [sum(r["kernel_launches"][k] for r in prof) for k in range(8)]
    dom = max(range(8), key=lambda k: ksec[k])
    avg_s = ksec[dom] / max(1, kn[dom])
    flops_per_launch = kfl[dom] / max(1, kn[dom])
    achieved = flops_per_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    out = dict(kernel=kernel_name(dom, prec), note=ROLE_NOTES[dom // 2], alg_flops_per_launch=flops_per_launch,
               avg_launch_us=1e6 * avg_s, launches_per_energy=kn[dom] / max(1, len(prof)),
               share_of_step=ksec[dom] / len(prof) / step_s if step_s > 0 else None)
    if prec == 2:
        out.update(bound="mfma", achieved=3 * achieved, peak=PEAK_BF16_TFLOPS, unit="TFLOP/s",
                   frac=3 * achieved / PEAK_BF16_TFLOPS, alg_tflops=achieved,
                   instruction="v_mfma_f32_16x16x16bf16_1k, three per product")
    else:
        peak = PEAK_FP32_TFLOPS if prec else PEAK_FP64_TFLOPS
        out.update(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                   instruction="v_mfma_f32_16x16x4f32" if prec else "v_mfma_f64_16x16x4f64")
    return out, (ksec, kfl, kn)


def golden(workload, s):
    path = os.path.join(ROOT, "tests", "golden", "%s_s%g.json" % (workload, s))
    return json.load(open(path)) if os.path.exists(path) else None


def parity_of(probs, res, workload):
    """|dE| and |dE|/|E| of each energy against the stored oracle values (FP64 oracle)."""
    out = []
    for p, r in zip(probs, res):
        g = golden(workload, p.s)
        if g is None:
            return None
        item = dict(s=p.s)
        for k in ("e2", "e3"):
            d = abs(r[k] - g[k])
            item["abs_d" + k] = d
            item["rel_d" + k] = d / max(abs(g[k]), 1e-300)
        out.append(item)
    return dict(items=out, max_abs_dE=max(max(x["abs_de2"], x["abs_de3"]) for x in out),
                max_rel_dE=max(max(x["rel_de2"], x["rel_de3"]) for x in out),
                reference="tests/golden/%s_s*.json (FP64 oracle, %s)" % (
                    workload, golden(workload, probs[0].s).get("source", "oracle")))


def cpu_baseline(workload, probs):
    """The FP64 oracle as it stands, timed on this host's cores.

    tiny, small: one whole energy of the workload's middle problem (the dense engine for
    tiny, the block-sparse DF level for small).  medium, large: a bounded sample, the block
    level's first stage (cumulants, antisymmetrised integral blocks and first-order
    amplitudes) on the full problem, converted to a whole energy with the ratio of a whole
    small energy to its first stage, both timed in the same call (an upper bound on the
    oracle's rate)."""
    p = probs[len(probs) // 2]
    cores = blas_threads()
    if workload == "tiny":
        from oracle import dsrg
        t0 = time.perf_counter()
        dsrg.run(p)
        dt = time.perf_counter() - t0
        return dict(value=1.0 / dt, unit="energies/s", cores=cores, kind="oracle",
                    sample="one whole energy, oracle/dsrg.py, %.2f s" % dt)
    from oracle import dsrg_df
    if workload == "small":
        t0 = time.perf_counter()
        dsrg_df.run(p)
        dt = time.perf_counter() - t0
        return dict(value=1.0 / dt, unit="energies/s", cores=cores, kind="oracle",
                    sample="one whole energy (s = %g), oracle/dsrg_df.py, %.1f s" % (p.s, dt))
    # medium, large: a whole oracle energy takes hours here.  Sample: the block level's first
    # stage (densities, integral blocks, first-order amplitudes) on the full problem, scaled
    # by the ratio of a whole energy to that stage measured now on the small workload; the
    # ratio grows with the virtual space, so the value bounds the oracle's rate from above.
    t0 = time.perf_counter()
    dsrg_df.run(p, through="first_order")
    t_first = time.perf_counter() - t0
    from paper_1701_02011_amd.synth import make_config
    q = make_config("small")
    t0 = time.perf_counter()
    dsrg_df.run(q, through="first_order")
    t_small_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    dsrg_df.run(q)
    t_small = time.perf_counter() - t0
    ratio = t_small / t_small_first
    return dict(value=1.0 / (t_first * ratio), unit="energies/s", cores=cores, kind="oracle",
                bound="upper",
                sample="first stage of oracle/dsrg_df.py (cumulants, integral blocks, first-order "
                       "amplitudes) on the full %s problem: %.1f s; scaled by the whole-energy / "
                       "first-stage ratio measured on the small workload (%.1f s / %.2f s = %.0f), "
                       "so >= %.0f s per %s energy (the ratio grows with the virtual space)"
                       % (workload, t_first, t_small, t_small_first, ratio, t_first * ratio, workload))


def progress(msg):
    """A progress line on stderr (the JSON result is the only line on stdout)."""
    sys.stderr.write("bench: %s\n" % msg)
    sys.stderr.flush()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium", choices=["tiny", "small", "medium", "large", "curve"])
    ap.add_argument("--geometries", type=int, default=4, help="curve workload: number of geometries")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"],
                    help="precision of the timed headline loop (fp32: FP32 products, bf16x3: split "
                         "BF16 x3 products; FP64 sums)")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="timed steps of the FP32-product pass reported beside the headline")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.stderr.write("bench.py: this benchmark runs on exactly one GPU; --gpus %d is not "
                         "supported (the multi-GPU sharding is a design note only)\n" % args.gpus)
        sys.exit(2)

    import torch
    from paper_1701_02011_amd import _lib
    _lib.load()
    if args.workload == "curve":
        # tile choices per size class from the package's autotuner, when it has stored them
        rules = _lib.load_tile_rules()
        progress("tile rules: %s" % ("none stored" if rules is None else rules))
    probs = workload_problems(args.workload, args.geometries)
    progress("inputs drawn: %d problem(s)" % len(probs))
    dev = [_lib.to_device(p) for p in probs]
    torch.cuda.synchronize()

    def step(prec):
        if args.workload == "curve":
            # geometries of different shapes: the batch entry point (rounds of two, unplanned
            # shapes on worker threads)
            res, codes = _lib.dsrg_pt3_energy_batch(dev, precision=prec)
            assert all(c == 0 for c in codes), codes
            return res
        return [_lib.dsrg_pt3_energy(d, precision=prec) for d in dev]

    def timed(prec, warmup, steps):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        progress("warm-up done (%d step(s))" % warmup)
        t0 = time.perf_counter()
        for _ in range(steps):
            res = step(prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        progress("timed %d step(s): %.3f s" % (steps, dt))
        return res, dt

    prec = {"fp64": 0, "fp32": 1, "bf16x3": 2}[args.precision]
    res, dt = timed(prec, args.warmup, args.steps)
    energies = args.steps * len(dev)
    ms_per_step = dt * 1e3 / args.steps

    # roofline of the dominant kernel instance: HIP events bracket every contraction launch
    # (on the stream it runs on) in a profiled pass over the same problems; the timed loop
    # above replays the recorded graph instead
    prof = [_lib.dsrg_pt3_energy(d, profile=True, precision=prec) for d in dev]
    progress("profiled pass done")
    torch.cuda.synchronize()
    roofline, (ksec, kfl, kn) = dominant_kernel(prof, prec, dt / args.steps / len(dev))
    roofline["traffic"] = measured_traffic(roofline["kernel"], args.workload, args.precision)
    peak = roofline["peak"]
    # whole-energy algorithmic rate: every contraction's 2 M N K over the step time
    alg_flops = sum(r["alg_flops"] for r in res)
    whole = dict(alg_tflop_per_energy=alg_flops / len(dev) / 1e12,
                 alg_tflops=alg_flops * args.steps / dt / 1e12,
                 frac_of_peak=alg_flops * args.steps / dt / 1e12 * (3 if prec == 2 else 1) / peak)

    out = {
        "metric": METRIC, "value": energies / dt, "unit": "energies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ["f64", "f64 (FP32 products)", "f64 (split BF16 x3 products)"][prec],
        "data": "synthetic",
        "config": {"workload": args.workload,
                   "problems": [dict(n_core=p.n_core, n_active=p.n_active, n_virtual=p.n_virtual,
                                     n_aux=p.n_aux, s=p.s) for p in probs],
                   "energies_per_step": len(dev)},
        "roofline": roofline,
        "whole_energy": whole,
        "energies": [dict(s=p.s, e2=r["e2"], e3=r["e3"]) for p, r in zip(probs, res)],
        "parity": parity_of(probs, res, args.workload),
        "kernels": {kernel_name(k, prec): dict(seconds=ksec[k], launches=kn[k], tflop=kfl[k] / 1e12)
                    for k in range(8) if kn[k]},
        "plan": [r["plan"] for r in res],
    }
    if args.mixed_steps > 0 and not prec:
        # the FP32-product path beside the FP64 headline: rate, and its error against the
        # FP64 GPU energies and the stored oracle values
        mres, mdt = timed(1, 1, args.mixed_steps)
        mprof = [_lib.dsrg_pt3_energy(d, profile=True, precision=1) for d in dev]
        mixed = dict(value=args.mixed_steps * len(dev) / mdt, unit="energies/s",
                     roofline=dominant_kernel(mprof, 1, mdt / args.mixed_steps / len(dev))[0],
                     speedup_vs_fp64=(args.mixed_steps * len(dev) / mdt) / (energies / dt),
                     parity=parity_of(probs, mres, args.workload),
                     vs_fp64_gpu=[dict(s=p.s, d_e2=m["e2"] - r["e2"], d_e3=m["e3"] - r["e3"],
                                       rel_e2=abs(m["e2"] - r["e2"]) / abs(r["e2"]),
                                       rel_e3=abs(m["e3"] - r["e3"]) / abs(r["e3"]))
                                  for p, m, r in zip(probs, mres, res)])
        out["fp32_products"] = mixed
        # split BF16 x3 products beside them (measured error, not a parity claim: R19)
        bres, bdt = timed(2, 1, args.mixed_steps)
        bprof = [_lib.dsrg_pt3_energy(d, profile=True, precision=2) for d in dev]
        out["bf16x3_products"] = dict(
            value=args.mixed_steps * len(dev) / bdt, unit="energies/s",
            roofline=dominant_kernel(bprof, 2, bdt / args.mixed_steps / len(dev))[0],
            speedup_vs_fp64=(args.mixed_steps * len(dev) / bdt) / (energies / dt),
            parity=parity_of(probs, bres, args.workload),
            vs_fp64_gpu=[dict(s=p.s, d_e2=b["e2"] - r["e2"], d_e3=b["e3"] - r["e3"],
                              rel_e2=abs(b["e2"] - r["e2"]) / abs(r["e2"]),
                              rel_e3=abs(b["e3"] - r["e3"]) / abs(r["e3"]))
                         for p, b, r in zip(probs, bres, res)])
    if not args.no_cpu_baseline and args.workload != "curve":
        out["cpu_baseline"] = cpu_baseline(args.workload, probs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

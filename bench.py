#!/usr/bin/env python3
"""Throughput of the spin spherical-harmonic transform on one MI355X.

A step is one inverse + forward SHT pair (the paper's round-trip timing, Sec.
6.3.2) of one MW map at L = 2048, spin 0, FP64, on synthetic Gaussian
coefficients scaled by 1/(1+l) (seed 1), with inputs resident in HBM.  Prints
one JSON line with pairs/s, the dominant kernel's FP64 roofline fraction
(algorithmic flops / live HIP-event launch duration), the round-trip error,
and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector peak
HBM_PEAK_GBS = 8000.0


def _log(msg):
    """Progress line on stderr (the result is the one JSON line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_flops(L, spin, rings):
    """Per direction per map: 6 flop per (ring, l, m) triple at spin 0, 8 otherwise
    (4 contraction + 4 recursion per generated d; spin 0 generates d for m >= 0 only)."""
    T = rings * (L * L - spin * spin)
    return (6 if spin == 0 else 8) * T


def kernel_source_sha():
    """First 16 hex digits of the sha256 over the sources the sweep kernels are built
    from (the kernel file and the device headers it includes)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("s2mi_kernels.hip", "s2mi_recur.h", "s2mi_internal.h", "s2mi_fft.h"):
        h.update(open(os.path.join(ROOT, "paper_2311_14670_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, L, spin):
    """HBM bytes per launch of a sweep kernel from the committed counter summary
    (FETCH_SIZE / WRITE_SIZE scaled by a plain-copy calibration), only when the
    summary was taken on this workload and on the current kernel source; else None."""
    if (L, spin) != (2048, 0):
        return None
    summ = os.path.join(ROOT, "profiles", "dstage_counters_mw_L2048_spin0.md")
    try:
        text = open(summ).read()
        sha = kernel_source_sha()
    except OSError:
        return None
    if f"kernels source sha256 (first 16 hex): {sha}" not in text:
        return None
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic_bytes" and parts[1] == kernel:
            return float(parts[2])
    return None


def mixed_precision(L, batch, steps, dev, fp64_plan):
    """Batched MW spin-0 pairs with the contraction on the matrix cores (FP32 and
    split BF16): maps/s, the stage split, and the max relative coefficient error of
    maps 0 and batch-1 against the FP64 path (whose parity with the oracle the tests
    check) and of their round trips against the input."""
    import torch
    from paper_2311_14670_amd import binding
    from paper_2311_14670_amd.synth import flm_gaussian
    flm = flm_gaussian(L, 0, seed=2, batch=batch, scale="inv1pl")
    x = torch.from_numpy(flm).to(dev)
    f64_inv = fp64_plan.inverse(x[0]).cpu().numpy()
    f64_pair = fp64_plan.forward(fp64_plan.inverse(x[0])).cpu().numpy()
    res = {"workload": f"MW L={L} spin 0, batch {batch} maps, Gaussian coefficients x 1/(1+l), seed 2",
           "batch": batch}
    for prec in ("fp32", "split_bf16"):
        plan = binding.Plan(L, spin=0, max_batch=batch, precision=prec, device=dev)
        _ = plan.workspace
        y = plan.forward(plan.inverse(x))          # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            finv = plan.inverse(x)
            y = plan.forward(finv)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # stage split of one more pair (HIP events around every launch, on the launch stream)
        plan.set_timing(True)
        plan.read_timing()
        plan.forward(plan.inverse(x))
        stages = plan.read_timing()
        plan.set_timing(False)
        fi = finv[0].cpu().numpy()
        y0 = y[0].cpu().numpy()

        def err(a, b):
            return {"max_rel": float(np.max(np.abs(a - b)) / np.max(np.abs(b))),
                    "rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b))}
        res[prec] = {"ms_per_batch_pair": ms, "maps_per_s": batch * 1e3 / ms,
                     "stage_ms": {k: v[0] for k, v in stages.items()},
                     "stage_launches": {k: v[1] for k, v in stages.items()},
                     "inverse_vs_fp64": err(fi, f64_inv), "pair_vs_fp64": err(y0, f64_pair),
                     "pair_vs_input": err(y0, flm[0]),
                     "pair_vs_input_last_map": err(y[batch - 1].cpu().numpy(), flm[batch - 1]),
                     "contraction_tflops": _contraction_tflops(L, batch, prec, stages)}
        plan.close()
        del y, finv
        torch.cuda.empty_cache()
    return res


def _contraction_tflops(L, batch, prec, stages):
    """The matrix-core kernels' rate on the contraction's algorithmic work: 4 flop per
    (ring, l, m) triple and map per direction (8 T B for the pair), tripled for split
    BF16's three products, over the measured MFMA-stage time of one pair."""
    T = L * L * L
    flops = 8 * T * batch * (3 if prec == "split_bf16" else 1)
    ms = stages.get("mfma", (0.0, 0))[0]
    peak = 2500.0 if prec == "split_bf16" else 157.3
    if ms <= 0:
        return None
    tf = flops / (ms * 1e-3) / 1e12
    return {"achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak, "mfma_ms_per_pair": ms,
            "algorithmic_flops_per_pair": flops}


def largest_size(L, steps, dev):
    """The paper's largest MW size (one spin-0 map, FP64): ms per inverse+forward
    pair and the round-trip error, beside the headline figure."""
    import torch
    from paper_2311_14670_amd import binding
    from paper_2311_14670_amd.synth import flm_gaussian
    flm = flm_gaussian(L, 0, seed=1, scale="inv1pl")
    x = torch.from_numpy(flm).to(dev)
    plan = binding.Plan(L, device=dev)
    y = plan.forward(plan.inverse(x))
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        y = plan.forward(plan.inverse(x))
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    err = float(np.linalg.norm(y.cpu().numpy() - flm) / np.linalg.norm(flm))
    del plan, x, y
    torch.cuda.empty_cache()
    return {"workload": f"MW L={L} spin-0 inverse+forward pair, one map, complex128 Gaussian coefficients "
                        "x 1/(1+l), seed 1", "L": L, "steps": steps, "ms_per_pair": ms, "pairs_per_s": 1e3 / ms,
            "roundtrip_rel_l2": err}


def real_signal(L, steps, dev):
    """The real-signal path (s2_inverse_real / s2_forward_real, MW spin 0) at the
    headline size: ms per pair and the round-trip error against the Hermitian
    completion of the input (what the exact round trip of a real map returns)."""
    import torch
    from paper_2311_14670_amd import binding
    from paper_2311_14670_amd.synth import flm_gaussian
    flm = flm_gaussian(L, 0, seed=1, scale="inv1pl")
    x = torch.from_numpy(flm).to(dev)
    plan = binding.Plan(L, device=dev)
    y = plan.forward_real(plan.inverse_real(x))
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        y = plan.forward_real(plan.inverse_real(x))
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    full = flm.copy()                              # flm[l][-m] = (-1)^m conj(flm[l][m]), order 0 real
    for m in range(1, L):
        full[:, L - 1 - m] = (-1.0) ** m * np.conj(full[:, L - 1 + m])
    full[:, L - 1] = full[:, L - 1].real
    err = float(np.linalg.norm(y.cpu().numpy() - full) / np.linalg.norm(full))
    stages = _stage_split(plan, x, plan.forward_real, plan.inverse_real)
    del plan, x, y
    torch.cuda.empty_cache()
    return {"workload": f"MW L={L} spin-0 real-signal inverse+forward pair, one map (orders m >= 0 of the "
                        "headline coefficients)", "L": L, "steps": steps, "ms_per_pair": ms,
            "pairs_per_s": 1e3 / ms, "roundtrip_rel_l2": err, "stage_ms": stages}


def _stage_split(plan, x, forward=None, inverse=None):
    """Per-stage milliseconds of one more inverse+forward pair (HIP events around
    every launch, on the launch stream)."""
    inverse = inverse or plan.inverse
    forward = forward or plan.forward
    plan.set_timing(True)
    plan.read_timing()
    forward(inverse(x))
    t = plan.read_timing()
    plan.set_timing(False)
    return {k: v[0] for k, v in t.items()}


def mw_pairs(cases, steps, dev):
    """Further one-map MW FP64 pairs (L, spin): ms per pair and the round trip."""
    import torch
    from paper_2311_14670_amd import binding
    from paper_2311_14670_amd.synth import flm_gaussian
    res = []
    for L, spin in cases:
        flm = flm_gaussian(L, spin, seed=1, scale="inv1pl")
        x = torch.from_numpy(flm).to(dev)
        plan = binding.Plan(L, spin=spin, device=dev)
        y = plan.forward(plan.inverse(x))
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            y = plan.forward(plan.inverse(x))
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        err = float(np.linalg.norm(y.cpu().numpy() - flm) / np.linalg.norm(flm))
        stages = _stage_split(plan, x)
        flops = algorithmic_flops(L, spin, L)
        res.append({"L": L, "spin": spin, "ms_per_pair": ms, "pairs_per_s": 1e3 / ms, "roundtrip_rel_l2": err,
                    "pair_fp64_frac": 2 * flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, "stage_ms": stages})
        del plan, x, y
        torch.cuda.empty_cache()
    return res


def healpix_pair(L, nside, steps, dev):
    """HEALPix (RING, nside) spin-0 inverse+forward pair at the headline L, one map:
    ms per pair, whether the sweeps run over the northern rings (mirror symmetry),
    and the stage split (parity with the oracle is checked by the tests)."""
    import torch
    from paper_2311_14670_amd import binding
    from paper_2311_14670_amd.synth import flm_gaussian
    flm = flm_gaussian(L, 0, seed=1, scale="inv1pl")
    x = torch.from_numpy(flm).to(dev)
    plan = binding.Plan(L, sampling="healpix", nside=nside, device=dev)
    y = plan.forward(plan.inverse(x))
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        y = plan.forward(plan.inverse(x))
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    swept = plan.info["swept_rings"]
    stages = _stage_split(plan, x)
    del plan, x, y
    torch.cuda.empty_cache()
    return {"workload": f"HEALPix nside={nside} L={L} spin-0 inverse+forward pair, one map", "L": L, "nside": nside,
            "steps": steps, "ms_per_pair": ms, "pairs_per_s": 1e3 / ms, "swept_rings": swept,
            "rings": 4 * nside - 1, "stage_ms": stages,
            "algorithmic_flops_per_pair": 2 * algorithmic_flops(L, 0, 4 * nside - 1),
            "executed_flops_per_pair": 2 * algorithmic_flops(L, 0, swept)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(L, spin, flm, nring_sample, norder_sample, runs=3, one_core_rings=8, one_core_orders=8):
    """The oracle (direct sums, OpenMP over rings / orders) on the host cores: the
    inverse on a sample of rings and the forward on a sample of orders at the same
    L, extrapolated to one pair (every ring costs the same; the sampled orders span
    the whole range).  Median of `runs` runs on all the threads OpenMP is given,
    and of `runs` runs on one thread with a smaller sample."""
    import ctypes
    import oracle
    oracle._load()
    gomp = ctypes.CDLL("libgomp.so.1")          # the OpenMP runtime the oracle runs on
    g = np.random.default_rng(11).standard_normal((L, 2 * L - 1)) + 0j

    def one_run(nr, no):
        rings = np.unique(np.linspace(0, L - 1, nr).astype(int))
        ms = np.unique(np.linspace(-(L - 1), L - 1, no).astype(int))
        t0 = time.perf_counter()
        oracle.s2_inverse(flm, L, spin, rings=rings)
        t1 = time.perf_counter()
        oracle.s2_forward(g, L, spin, ms=ms)
        t2 = time.perf_counter()
        return (t1 - t0) * L / rings.size + (t2 - t1) * (2 * L - 1) / ms.size, t2 - t0, rings.size, ms.size

    threads = int(gomp.omp_get_max_threads())
    multi = [one_run(nring_sample, norder_sample) for _ in range(runs)]
    gomp.omp_set_num_threads(1)
    try:
        single = [one_run(one_core_rings, one_core_orders) for _ in range(runs)]
    finally:
        gomp.omp_set_num_threads(threads)
    med = float(np.median([r[0] for r in multi]))
    med1 = float(np.median([r[0] for r in single]))
    nr, no = multi[0][2], multi[0][3]
    return {"value": 1.0 / med, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"median of {runs} runs: inverse on {nr} of {L} rings + forward on {no} of {2 * L - 1} "
                      f"orders, L={L} MW spin {spin}, extrapolated to one pair "
                      f"({sum(r[1] for r in multi):.1f} s measured in all)",
            "cpu_model": _cpu_model(),
            "one_core": {"value": 1.0 / med1, "unit": "pairs/s", "cores": 1,
                         "sample": f"median of {runs} runs: inverse on {single[0][2]} rings + forward on "
                                   f"{single[0][3]} orders, extrapolated to one pair "
                                   f"({sum(r[1] for r in single):.1f} s measured in all)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=2048)
    ap.add_argument("--spin", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rings", type=int, default=160)
    ap.add_argument("--cpu-orders", type=int, default=160)
    ap.add_argument("--mixed-batch", type=int, default=64,
                    help="maps per call of the matrix-core (FP32 / split-BF16) comparison; 0 skips it")
    ap.add_argument("--mixed-steps", type=int, default=3)
    ap.add_argument("--large-L", type=int, default=4096, help="also time one MW spin-0 pair at this L (0: skip)")
    ap.add_argument("--serving-requests", type=int, default=80,
                    help="also serve a seeded mixed request stream (L log-uniform in [64, --serving-lmax], SO(3) "
                         "L <= --serving-so3-lmax) at FP64 and split BF16; 0: skip")
    ap.add_argument("--serving-lmax", type=int, default=4096)
    ap.add_argument("--serving-so3-lmax", type=int, default=512)
    ap.add_argument("--large-steps", type=int, default=3)
    ap.add_argument("--mw-steps", type=int, default=10,
                    help="also time MW pairs at L=1024 (spin 0, 2) and L=2048 spin 2; 0: skip")
    ap.add_argument("--healpix-steps", type=int, default=10,
                    help="also time a HEALPix nside=L/2 spin-0 pair at the headline L; 0: skip")
    ap.add_argument("--real-steps", type=int, default=10,
                    help="also time the real-signal path at the headline L (spin 0); 0: skip")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run plain device copies of MIB MiB (a reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the transform is not sharded "
              "across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_14670_amd import binding
    from paper_2311_14670_amd.synth import flm_gaussian

    L, spin = args.L, args.spin
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    flm = flm_gaussian(L, spin, seed=1, scale="inv1pl")
    x = torch.from_numpy(flm).to(dev)
    plan = binding.Plan(L, spin=spin, device=dev)
    _ = plan.workspace
    for _ in range(args.warmup):
        y = plan.forward(plan.inverse(x))
    torch.cuda.synchronize()

    plan.set_timing(True)
    plan.read_timing()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        y = plan.forward(plan.inverse(x))
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = plan.read_timing()
    plan.set_timing(False)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    wall_ms_step = (t1 - t0) * 1e3 / args.steps

    # accuracy of the benchmarked pair (round trip of band-limited input)
    yh = y.cpu().numpy()
    rt_err = float(np.linalg.norm(yh - flm) / np.linalg.norm(flm))

    # dominant kernel and its FP64 roofline (stages: totals over the timed steps); a
    # direction's algorithmic flops are split over its launches per step (spin s != 0:
    # the runs n = -s and n = +s, one side each)
    dom = max(stages, key=lambda s: stages[s][0])
    nlaunch = max(stages[dom][1], 1)
    dom_ms = stages[dom][0] / nlaunch
    per_step = max(1, round(nlaunch / args.steps))
    flops = algorithmic_flops(L, spin, L)
    if dom in ("dstage_inv", "dstage_fwd"):
        per_launch = flops / per_step
        achieved = per_launch / (dom_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": measured_traffic("k_" + dom, L, spin),
                "algorithmic_flops_per_launch": per_launch, "avg_launch_ms": dom_ms, "launches_per_step": per_step}
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "avg_launch_ms": dom_ms}
    # whole-pair FP64 fraction (both d-stage directions' algorithmic flops over the step time)
    pair_frac = 2 * flops / (ms_step * 1e-3) / 1e12 / FP64_PEAK_TFLOPS

    out = {
        "metric": "SHT pairs/s at L=2048 (err<=1e-11)",
        "value": 1e3 / ms_step,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "wall_ms_per_step": wall_ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"MW L={L} spin-{spin} inverse+forward SHT pair, one map, complex128 "
                               "Gaussian coefficients x 1/(1+l), seed 1",
                   "L": L, "spin": spin, "sampling": "mw", "batch": 1},
        "roundtrip_rel_l2": rt_err,
        "pair_fp64_frac": pair_frac,
        "stage_ms_per_step": {s: v[0] / args.steps for s, v in stages.items()},
        "roofline": roof,
    }
    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 17                      # float64 elements in MIB MiB
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = n * 8
    _log(f"headline: {out['value']:.1f} pairs/s")
    if args.mixed_batch > 0 and spin == 0:
        _log("matrix-core batch")
        out["mixed_precision"] = mixed_precision(L, args.mixed_batch, args.mixed_steps, dev, plan)
    if args.real_steps > 0 and spin == 0:
        _log("real-signal pair")
        out["real_signal"] = real_signal(L, args.real_steps, dev)
    if args.healpix_steps > 0:
        _log("HEALPix pair")
        out["healpix"] = healpix_pair(L, L // 2, args.healpix_steps, dev)
    if args.mw_steps > 0:
        _log("MW L=1024 and spin-2 pairs")
        out["mw_other"] = mw_pairs([(1024, 0), (1024, 2), (2048, 2)], args.mw_steps, dev)
    if args.large_L > 0 and args.large_steps > 0:
        _log(f"MW L={args.large_L} pair")
        out["large_L"] = largest_size(args.large_L, args.large_steps, dev)
    if args.serving_requests > 0:
        from paper_2311_14670_amd.serving import run_mix
        from paper_2311_14670_amd.serving import check_subset
        kw = dict(n_requests=args.serving_requests, lmax=args.serving_lmax, so3_lmax=args.serving_so3_lmax,
                  device=str(dev))
        _log("serving, FP64")
        out["serving"] = run_mix(**kw)
        out["serving"]["sampled_check"] = check_subset(**kw)
        _log("serving, split BF16")
        out["serving_split_bf16"] = run_mix(**kw, precision="split_bf16")
        out["serving_split_bf16"]["sampled_check"] = check_subset(**kw, precision="split_bf16")
    if not args.no_cpu_baseline:
        _log("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(L, spin, flm, args.cpu_rings, args.cpu_orders)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

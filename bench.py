"""Benchmark of the chain RK4 hot path on one MI355X.

Default workload: the quartic chain with N = 2^24 sites, periodic, q and p
uniform on [-1, 1) from SplitMix64 seed 0, dt = 0.01. One bench step is one
job of 1000 RK4 steps over the whole chain plus its energy read-back. The
state is resident in HBM before the timed region starts.

Prints one JSON line: site-updates per second (N * RK4 steps / s), the
roofline of the dominant kernel, p50/p99 job latency, and the CPU oracle's
rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts.
HBM_PEAK_GBPS = 8000.0
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
# FP64 vector lane-operations per second: every SIMD retires 16 FP64 lane-ops
# per clock (an FMA is one op), the rate behind the 78.6 TFLOP/s FP64 vector
# peak (which counts an FMA as two flops).
VALU_PEAK_TOPS = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_GHZ * 1e9 / 1e12  # 39.32
FP64_VECTOR_TFLOPS = 78.6
# FP32 vector lane-operations per second: the published 157.3 TFLOP/s FP32
# vector peak counts an FMA as two flops, so 78.6 T lane-ops/s, twice the
# FP64 rate. The FP32 kernels are built without packed FP32 instructions;
# their SQ counters show single FP32 VALU instructions retiring faster than
# one wave64 instruction per 4 cycles per SIMD (the FP64 rate), so this is
# the ceiling they are measured against.
FP32_VALU_PEAK_TOPS = 2 * VALU_PEAK_TOPS
# Algorithmic work of the compensated FP32 update: the 42 operations of RK4
# plus the compensation (t = y + v, c = (t - y) - v: 3 operations, and the
# carry subtracted from the increment: 1) for q and p.
OPS_PER_SU_FP32_KAHAN = 42 + 8

# Algorithmic work of one site-update (one RK4 step of one site), quartic:
# force 7 ops (bond diff, 2 mul for the cube, q^2, fma, 2 sub) x 4 stages,
# stage arguments 2 fma x 3 stages, accumulators 3 ops x 2 components,
# final update 1 fma x 2 components.
# Roessler (three coordinates): right-hand side 7 ops (bond diff, two subs,
# y + z, two fma, x - c) x 4 stages, stage arguments 3 fma x 3 stages,
# accumulators 3 ops x 3 stages, final update 3 fma.
# Second-neighbour bonds (quartic): the force is 12 ops per stage.
OPS_PER_SU = {"quartic": 42, "harmonic": 26, "roessler": 49, "quartic_nnn": 62,
              "harmonic_nnn": 38}
# What the kernels execute: for dq/dt = p the q stage arguments and the q
# update follow from p and the forces, without the p stage values, which
# saves 3 of the 14 operations around the forces (Roessler: unchanged); the
# quartic force subtracts U'(q) = q (1 + q^2) with one fused multiply-add,
# 6 operations per stage instead of 7.
EXECUTED_FORCE_OPS = {"quartic": 6, "harmonic": 3}
EXECUTED_OPS_PER_SU = {"quartic": 35, "harmonic": 23, "roessler": 49, "quartic_nnn": 55,
                       "harmonic_nnn": 35}
FLOPS_PER_SU = {"quartic": 58, "harmonic": 38, "roessler": 75, "quartic_nnn": 78,
                "harmonic_nnn": 50}
# Bytes per site-update of one pass: read q, p and write q, p once.
BYTES_PER_SITE_PASS = {"fp64": 32, "fp32_kahan": 32,      # FP32: q, p, cq, cp
                       "fp32_kahan64": 48,                # FP32 q, p; FP64 cq, cp
                       "fp32": 16}                        # FP32 q, p, no carries
BYTES_PER_SITE_PASS_ROESSLER = 48                       # x, y, z in FP64


# HBM bytes per fused pass from two rocprofv3 counter runs (FETCH_SIZE and
# WRITE_SIZE, each scaled by what it reads for a 512 MiB device copy), for
# the kernel sources with this sha256 and this cluster shape (sites per lane,
# wavefronts per cluster, halo) on N = 2^24.
MEASURED_TRAFFIC = {
    "sha256": "47167e8e53c2edc1514f913f6727e24722f2a91ebe1a2d26ae59c5e10f3c21aa",
    "shape": (8, 4, 64), "n": 1 << 24,
    "bytes_per_launch": 555367872, "fetch_factor": 0.5000, "write_factor": 1.0000,
}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1412_0544_amd", "csrc")
    for name in sorted(("fused.hip", "cluster.hpp", "rk4_device.hpp", "launch.hpp")):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def roofline(n, ksteps, t_launch, model="quartic", prec="fp64"):
    """Roofline of one fused pass of `ksteps` steps over n sites taking t_launch s."""
    bytes_alg = (BYTES_PER_SITE_PASS_ROESSLER if model == "roessler"
                 else BYTES_PER_SITE_PASS[prec]) * n
    fp64 = prec == "fp64"
    ops_su = OPS_PER_SU_FP32_KAHAN if prec == "fp32_kahan" and model == "quartic" else \
        OPS_PER_SU[model]
    peak = VALU_PEAK_TOPS if fp64 else FP32_VALU_PEAK_TOPS
    ops_alg = ops_su * n * ksteps
    t_hbm = bytes_alg / (HBM_PEAK_GBPS * 1e9)
    t_alu = ops_alg / (peak * 1e12)
    hbm = {"achieved": bytes_alg / t_launch / 1e9, "peak": HBM_PEAK_GBPS, "unit": "GB/s"}
    alu = {"achieved": ops_alg / t_launch / 1e12, "peak": peak, "unit": "Tops/s"}
    for d in (hbm, alu):
        d["frac"] = d["achieved"] / d["peak"]
    if t_alu >= t_hbm:
        r = {"bound": "alu", **alu,
             "op": ("FP64" if fp64 else "FP32") + " VALU lane-op (an fma is one op)",
             "hbm_view": hbm}
        if fp64:
            ex = EXECUTED_OPS_PER_SU[model] * n * ksteps / t_launch / 1e12
            r["flops_TFLOPs"] = FLOPS_PER_SU[model] * n * ksteps / t_launch / 1e12
            r["executed"] = {"ops_per_su": EXECUTED_OPS_PER_SU[model], "achieved": ex,
                             "frac": ex / VALU_PEAK_TOPS}
    else:
        r = {"bound": "hbm", **hbm, "alu_view": alu}
    r["algorithmic_per_launch"] = {"bytes": bytes_alg, "ops": ops_alg, "sites": n, "ksteps": ksteps}
    return r


def time_jobs(ch, steps_per_job, jobs, with_energy=True):
    """Run `jobs` jobs; return per-job (latency_s, step_gpu_s) and total wall."""
    import torch
    st = ch.stream
    lat, gpu = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(jobs):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        tj = time.perf_counter()
        a.record(st)
        ch.step(steps_per_job)
        b.record(st)
        if with_energy:
            ch.energy()  # synchronises the stream
        else:
            b.synchronize()
        lat.append(time.perf_counter() - tj)
        gpu.append(a.elapsed_time(b) / 1e3)
    torch.cuda.synchronize()
    return lat, gpu, time.perf_counter() - t0


def fused_launches(plan, steps):
    """Number of fused passes a step call of `steps` makes (see the host plan)."""
    if plan["resident"]:
        return 1
    k = plan["kdepth"]
    m = steps // k + (1 if steps % k else 0)
    if m % 2 == 1 and any(x >= 2 for x in [k] * (steps // k) + ([steps % k] if steps % k else [])):
        m += 1
    return m


# The paper's own CPU measurements (Sec. 3.2.1-3.2.2): one core each, the
# Roessler chain (three FP64 coordinates per site) at N = 2^20, T = 50 steps,
# the best of 10 runs. Site-updates/s are derived as Perf * 2^20. Context
# only: other hardware and another model than the quartic chain above.
PAPER_CPU = [
    {"hardware": "Intel Xeon E5 at 3.8 GHz (turbo), one core, ICC 15.0",
     "version": "standard RK4", "steps_per_s": "< 30", "site_updates_per_s": "< 3.1e7"},
    {"hardware": "Intel Xeon E5 at 3.8 GHz (turbo), one core, ICC 15.0",
     "version": "granular + SIMD (AVX)", "steps_per_s": "about 90",
     "site_updates_per_s": "about 9.4e7"},
    {"hardware": "AMD Opteron 6272 at 2.1 GHz, one core, clang 3.4",
     "version": "standard RK4", "steps_per_s": "about 10", "site_updates_per_s": "about 1.05e7"},
    {"hardware": "AMD Opteron 6272 at 2.1 GHz, one core, clang 3.4",
     "version": "granular + SIMD", "steps_per_s": "about 30", "site_updates_per_s": "about 3e7"},
]


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_oracle(n, dt, threads, target_s, chunk):
    """Advance the seed-0 chain in chunks of `chunk` steps until about
    `target_s` seconds; (site-updates/s, steps, seconds)."""
    import oracle
    import workloads
    q, p = workloads.chain_ics(n, 0)
    oracle.rk4(oracle.QUARTIC, q, p, dt, 1, threads=threads)      # first touch, thread start
    steps = 0
    t = time.perf_counter()
    while True:
        q, p = oracle.rk4(oracle.QUARTIC, q, p, dt, chunk, threads=threads)
        steps += chunk
        el = time.perf_counter() - t
        if el >= target_s:
            break
    return n * steps / el, steps, el


def cpu_baseline(n, dt, target_s=12.0, chunk=20, single_s=8.0, single_chunk=2):
    """The oracle (as it stands: plain C, FP64, whole-ring sweeps, -O3 for
    generic x86-64) on the host cores: the same chain and ICs, on every
    thread the run may use and on one thread, plus the paper's CPU numbers
    for context."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    v, steps, el = time_oracle(n, dt, threads, target_s, chunk)
    v1, steps1, el1 = time_oracle(n, dt, 1, single_s, single_chunk)
    return {"value": v, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"quartic chain N={n}, {steps} RK4 steps from the seed-0 initial state "
                      f"in chunks of {chunk}, {threads} OpenMP threads, {el:.1f} s",
            "single_thread": {"value": v1, "unit": "site-updates/s", "cores": 1,
                              "sample": f"the same chain, {steps1} RK4 steps in chunks of "
                                        f"{single_chunk}, one thread, {el1:.1f} s"},
            "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count(),
            "build": "gcc -O3 -std=c99 -fopenmp -ffp-contract=off (generic x86-64)",
            "paper_cpu_context": PAPER_CPU}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed jobs")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--job-steps", type=int, default=1000)
    ap.add_argument("--sites", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--kdepth", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="pick the cluster shape with the autotuner (default: the library plan)")
    ap.add_argument("--sweep", action="store_true", help="autotune over the full (S, W, k) grid")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with device copies of known size (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=500,
                    help="served jobs per load (0 = skip)")
    ap.add_argument("--size-sweep", action="store_true",
                    help="only sweep N = 2^10..2^26, fused vs per-stage, T = 50, best of 10")
    ap.add_argument("--plan-sweep", action="store_true",
                    help="only the cluster-shape study over N = 2^10..2^26 (S, W, k)")
    ap.add_argument("--nnn", action="store_true",
                    help="only the quartic chain with second-neighbour bonds on the bench chain")
    ap.add_argument("--tableaus", action="store_true",
                    help="only the explicit methods by Butcher tableau on the bench chain")
    ap.add_argument("--roessler", action="store_true",
                    help="only the Roessler chain with the paper's protocol (N = 2^20, T = 50 "
                         "steps, best of 10)")
    ap.add_argument("--serve", action="store_true",
                    help="only the served-job workload: --serve-jobs jobs at each load in "
                         "--serve-rho")
    ap.add_argument("--serve-rho", default="0.5,0.8",
                    help="offered loads of --serve, comma separated")
    ap.add_argument("--serve-sites", type=int, default=4,
                    help="sites per lane of the job server's rounds (--serve)")
    ap.add_argument("--serve-rate", type=float, default=6.5e11,
                    help="device capacity (site-updates/s) the loads of --serve refer to")
    ap.add_argument("--roessler-n", type=int, default=1 << 20,
                    help="chain length of --roessler (the paper's is 2^20)")
    ap.add_argument("--roessler-steps", type=int, default=50,
                    help="steps per timed call of --roessler (the paper's T is 50)")
    ap.add_argument("--prec", default="fp64",
                    choices=("fp64", "fp32_kahan", "fp32_kahan64", "fp32"),
                    help="precision of the timed chain (the headline line is FP64; the "
                         "others from the FP32-rounded initial state, for profiling)")
    ap.add_argument("--batch", action="store_true",
                    help="only the 4096-chain batch (one persistent launch per precision)")
    ap.add_argument("--batch-steps", type=int, default=2000,
                    help="steps of the timed launch of --batch")
    ap.add_argument("--batch-precs", default="fp64,fp32_kahan",
                    help="precisions of --batch, comma separated")
    ap.add_argument("--batch-shape", default="",
                    help="sites per lane and depth of --batch as S,K (default: the batch "
                         "autotuner's pick)")
    ap.add_argument("--batch-host-ics", action="store_true",
                    help="draw the --batch initial states on the host (the same values; far "
                         "fewer device launches, for profiled runs)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the chain path "
              "is built and measured on a single MI355X", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import workloads
    from paper_1412_0544_amd import Chain

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.size_sweep:
        print(json.dumps({"metric": "site-updates/sec vs chain length", "unit": "site-updates/s",
                          "n_gpus": 1, "data": "synthetic", "dtype": "f64",
                          "config": {"workload": "quartic chain, dt=0.01, T=50 steps, best of 10"},
                          "size_sweep": size_sweep(dev)}), flush=True)
        return 0
    if args.plan_sweep:
        print(json.dumps({"metric": "site-updates/sec by cluster shape and chain length",
                          "unit": "site-updates/s", "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": "quartic chain, dt=0.01, 64 steps, best of 3"},
                          "plan_sweep": plan_sweep(dev)}), flush=True)
        return 0
    if args.serve:
        loads = {}
        for rho in (float(x) for x in args.serve_rho.split(",")):
            log(f"[bench] serving {args.serve_jobs} jobs at load {rho}")
            loads[str(rho)] = variant_serving(0.01, dev, jobs=args.serve_jobs, rho=rho,
                                              rate_su=args.serve_rate,
                                              sites_per_lane=args.serve_sites)
        print(json.dumps({"metric": "served-job latency p50/p99 and throughput", "unit": "s",
                          "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": f"{args.serve_jobs} jobs, N log-uniform "
                                                 "[1e3, 4e6], steps U[1e3, 1e5], Poisson "
                                                 f"arrivals at rho x {args.serve_rate:.3g} "
                                                 "site-updates/s"},
                          "serving": loads}), flush=True)
        return 0
    if args.roessler:
        rn, rs = args.roessler_n, args.roessler_steps
        print(json.dumps({"metric": "RK4 steps/s of the Roessler chain (Perf = T / t_wall)",
                          "unit": "steps/s", "n_gpus": 1, "data": "synthetic", "dtype": "f64",
                          "config": {"workload": f"Roessler chain N={rn}, dt=0.01, T={rs} steps, "
                                                 "best of 10"},
                          "roessler": variant_roessler(dev, n=rn, steps=rs, sweep=args.sweep),
                          "copy_probe_bytes": copy_probe(dev) if args.copy_probe else None}),
              flush=True)
        return 0
    if args.batch:
        print(json.dumps({"metric": "site-updates/sec of one persistent launch over 4096 chains",
                          "unit": "site-updates/s", "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": "4096 quartic chains, N log-uniform [256, 65536], "
                                                 f"dt=0.01, {args.batch_steps} steps"},
                          "batch4096": variant_batch(
                              0.01, dev, steps=args.batch_steps, precs=args.batch_precs.split(","),
                              extras=False, host_ics=args.batch_host_ics,
                              shape=tuple(int(x) for x in args.batch_shape.split(","))
                              if args.batch_shape else None),
                          "copy_probe_bytes": copy_probe(dev) if args.copy_probe else None}),
              flush=True)
        return 0
    n, dt, js = args.n, 0.01, args.job_steps
    log(f"[bench] generating ICs n={n}")
    q0, p0 = workloads.chain_ics(n, 0)
    if args.prec != "fp64":
        q0, p0 = q0.astype(np.float32), p0.astype(np.float32)
    qd = torch.from_numpy(q0).to(dev)
    pd = torch.from_numpy(p0).to(dev)
    if args.nnn:
        print(json.dumps({"metric": "site-updates/sec, second-neighbour bonds",
                          "unit": "site-updates/s", "n_gpus": 1, "data": "synthetic",
                          "dtype": "f64", "config": {"workload": "quartic NNN chain N=2^24, dt=0.01"},
                          "quartic_nnn": variant_nnn(qd, pd, dt, n, dev, sweep=args.sweep)}), flush=True)
        return 0
    if args.tableaus:
        print(json.dumps({"metric": "site-updates/sec by explicit RK method",
                          "unit": "site-updates/s", "n_gpus": 1, "data": "synthetic",
                          "dtype": "f64", "config": {"workload": "quartic chain N=2^24, dt=0.01"},
                          "tableaus": variant_tableaus(qd, pd, dt, n, dev, sweep=args.sweep)}),
              flush=True)
        return 0

    from paper_1412_0544_amd import autotune
    sweep = {}
    if args.sites and args.waves and args.kdepth:
        S, W, K = args.sites, args.waves, args.kdepth
    elif args.autotune or args.sweep:
        cands = None
        if args.sweep:
            cands = [(s, w, k) for s in autotune.SITES for w in autotune.WAVES
                     for k in autotune.DEPTHS if 64 * s * w > 16 * k]
        log("[bench] autotuning the cluster shape")
        (S, W, K), table = autotune.tune(n, q=qd, p=pd, dt=dt, candidates=cands, device=dev,
                                        use_cache=False)
        sweep = {f"s{s}_w{w}_k{k}": v for (s, w, k), v in sorted(table.items())}
    else:
        probe = Chain(qd, pd, dt, prec=args.prec, resident=False, device=dev).plan()
        S, W, K = probe["sites_per_lane"], probe["waves_per_cluster"], probe["kdepth"]
    log(f"[bench] plan S={S} W={W} K={K}")

    ch = Chain(qd, pd, dt, prec=args.prec, sites_per_lane=S, waves_per_cluster=W, kdepth=K,
               resident=False, device=dev)
    plan = ch.plan()
    time_jobs(ch, js, args.warmup)
    log(f"[bench] timing {args.steps} jobs of {js} steps")
    lat, gpu, wall = time_jobs(ch, js, args.steps)
    e_final = ch.energy()
    ch.close()
    su = n * js * args.steps
    value = su / wall
    launches = fused_launches(plan, js)
    t_launch = statistics.mean(gpu) / launches
    rl = roofline(n, js / launches, t_launch, prec=args.prec)
    rl["launches_per_job"] = launches
    # the bandwidth a plain device copy reaches, to read the HBM view against
    # the achievable as well as the published peak
    copy = hbm_copy_gbps(dev)
    rl["hbm_view"]["copy_probe_GBps"] = copy
    rl["hbm_view"]["frac_of_copy_probe"] = rl["hbm_view"]["achieved"] / copy
    # the attainable rate of this plan: the lower of the HBM bound at its
    # depth and the VALU ceiling less the recomputed halo
    if args.prec in ("fp64", "fp32_kahan"):
        E = 64 * S * W
        alu_ceiling = (VALU_PEAK_TOPS if args.prec == "fp64" else FP32_VALU_PEAK_TOPS) * 1e12 / (
            OPS_PER_SU["quartic"] if args.prec == "fp64" else OPS_PER_SU_FP32_KAHAN)
        hbm_ceiling = HBM_PEAK_GBPS * 1e9 / BYTES_PER_SITE_PASS[args.prec] * (js / launches)
        bound = min(hbm_ceiling, alu_ceiling * plan["tile"] / E)
        rl["attainable"] = {"su_per_s": bound, "frac": value / bound,
                            "hbm_bound_su_per_s": hbm_ceiling,
                            "valu_bound_less_halo_su_per_s": alu_ceiling * plan["tile"] / E}
    rl["traffic"] = None
    mt = MEASURED_TRAFFIC
    if (args.prec == "fp64" and kernel_sources_sha256() == mt["sha256"]
            and (S, W, plan["halo"]) == mt["shape"]
            and n == mt["n"]):
        rl["traffic"] = mt["bytes_per_launch"]
        rl["traffic_vs_algorithmic"] = mt["bytes_per_launch"] / rl["algorithmic_per_launch"]["bytes"]

    out = {
        "metric": "site-updates/sec (RK4 steps x N / s) + % HBM roofline; p50/p99 job latency",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "quartic chain, N=2^24, periodic, q,p~U[-1,1) seed 0, dt=0.01, "
                               "1000 RK4 steps per job + energy",
                   "precision": args.prec,
                   "n": n, "job_steps": js, "sites_per_lane": S, "waves_per_cluster": W,
                   "kdepth": K, "tile": plan["tile"], "halo": plan["halo"],
                   "overlap_factor": plan["overlap_factor"]},
        "hbm_roofline_pct": 100.0 * value / (HBM_PEAK_GBPS * 1e9 / 32),
        "latency_ms": {"p50": 1e3 * pct(lat, 50), "p99": 1e3 * pct(lat, 99)},
        # the step call of each timed job alone (HIP events on its stream, no
        # energy): best and median over the jobs, the min-of-M protocol
        "per_job_device_su_per_s": {"best": n * js / min(gpu),
                                    "median": n * js / statistics.median(gpu),
                                    "jobs": len(gpu)},
        "roofline": rl,
        "energy_final": e_final,
    }
    if sweep:
        out["autotune_su_per_s"] = sweep

    if not args.no_variants:
        out["variants"] = variants(qd, pd, dt, n, dev, (S, W), serve_jobs=args.serve_jobs)

    if args.copy_probe:
        out["copy_probe_bytes"] = copy_probe(dev)

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        try:
            out["cpu_baseline"] = cpu_baseline(n, dt)
        except Exception as e:  # noqa: BLE001 -- reported in the JSON line
            log(f"[bench] CPU baseline failed: {e!r}")
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)
    return 0


def copy_probe(dev):
    """Three plain device copies of 512 MiB, for scaling the HBM byte
    counters of a profiled run; returns the bytes of one copy."""
    import torch
    src = torch.empty(1 << 26, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 8


def hbm_copy_gbps(dev, nbytes=1 << 30, trials=5):
    """Achievable HBM bandwidth: the best of `trials` device copies of
    `nbytes` (read and written, so 2*nbytes move), timed with HIP events."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream(dev)
    dst.copy_(src)
    t = min(ev_seconds(lambda: dst.copy_(src), st) for _ in range(trials))
    del src, dst
    return 2 * nbytes / t / 1e9


def ev_seconds(fn, stream):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / 1e3


def variant_precision(n, dt, dev, steps=10_000, every=100):
    """FP32 state with compensated update (FP32 or FP64 carries), and plain
    FP32 as the control, vs the FP64 GPU path on the same
    chain: relative energy drift sampled every `every` steps, and the 100-step
    state error against the FP64 oracle (sampled sites, from the FP32-rounded
    initial state)."""
    import numpy as np
    import torch
    import oracle
    import workloads
    from paper_1412_0544_amd import Chain
    q32, p32 = workloads.chain_ics_torch(n, 0, dev, torch.float32)
    out = {"n": n, "steps": steps, "dt": dt}
    for name, prec, q, p in (("fp64", "fp64", q32.double(), p32.double()),
                             ("fp32_kahan", "fp32_kahan", q32, p32),
                             ("fp32_kahan64", "fp32_kahan64", q32, p32),
                             ("fp32", "fp32", q32, p32)):
        ch = Chain(q, p, dt, prec=prec, device=dev)
        e0 = ch.energy()
        drift = []
        t = 0.0
        for _ in range(steps // every):
            t += ev_seconds(lambda: ch.step(every), ch.stream)
            drift.append((ch.energy() - e0) / e0)
        out[name] = {"su_per_s": n * steps / t, "rel_drift_final": drift[-1],
                     "rel_drift_max_abs": float(np.max(np.abs(drift))),
                     "rel_drift_samples": drift[:: max(1, len(drift) // 20)],
                     "plan": {k: v for k, v in ch.plan().items()
                              if k in ("sites_per_lane", "waves_per_cluster", "kdepth", "halo")}}
        if prec in ("fp32_kahan", "fp32", "fp64"):
            ops = {"fp64": OPS_PER_SU["quartic"], "fp32": OPS_PER_SU["quartic"],
                   "fp32_kahan": OPS_PER_SU_FP32_KAHAN}[prec]
            peak = VALU_PEAK_TOPS if prec == "fp64" else FP32_VALU_PEAK_TOPS
            a = ops * n * steps / t / 1e12
            out[name]["roofline"] = {
                "bound": "alu", "achieved": a, "peak": peak, "unit": "Tops/s", "frac": a / peak,
                "ops_per_su": ops, "op": ("FP64" if prec == "fp64" else "FP32") +
                " VALU lane-op (an fma is one op)", "timed": "device time of the step calls"}
        ch.close()
    # the drift again at a step exact in FP32 (2^-7): the FP32 stages then
    # advance by the same step as the final combination
    dt2 = 2.0 ** -7
    out["exact_dt"] = {"dt": dt2, "steps": steps}
    for name, prec, q, p in (("fp64", "fp64", q32.double(), p32.double()),
                             ("fp32_kahan", "fp32_kahan", q32, p32),
                             ("fp32_kahan64", "fp32_kahan64", q32, p32),
                             ("fp32", "fp32", q32, p32)):
        ch = Chain(q, p, dt2, prec=prec, device=dev)
        e0 = ch.energy()
        ch.step(steps)
        out["exact_dt"][name + "_rel_drift"] = (ch.energy() - e0) / e0
        ch.close()
    # 100-step error against the oracle (FP32-rounded ICs), sampled sites
    q0 = q32.double().cpu().numpy()
    p0 = p32.double().cpu().numpy()
    sites = np.unique(np.linspace(0, n - 1, 48).astype(np.int64))
    qs, ps = oracle.rk4_sites(oracle.QUARTIC, q0, p0, dt, 100, sites)
    for name, prec, q, p in (("fp64", "fp64", q32.double(), p32.double()),
                             ("fp32_kahan", "fp32_kahan", q32, p32),
                             ("fp32_kahan64", "fp32_kahan64", q32, p32),
                             ("fp32", "fp32", q32, p32)):
        ch = Chain(q, p, dt, prec=prec, device=dev)
        ch.step(100)
        cq, cp = ch.carry_tensors()
        qq = ch.q.double() - (cq.double() if cq is not None else 0)
        pp = ch.p.double() - (cp.double() if cp is not None else 0)
        err = max(float(np.abs(qq.cpu().numpy()[sites] - qs).max()),
                  float(np.abs(pp.cpu().numpy()[sites] - ps).max()))
        out[name]["err100_vs_oracle"] = err
        ch.close()
    return out


def variant_batch(dt, dev, steps=2000, count=4096, precs=("fp64", "fp32_kahan"), extras=True,
                  shape=None, host_ics=False):
    """4096 chains, lengths log-uniform in [256, 65536], one persistent
    launch of `steps` steps, FP64 and FP32 with compensated update, at the
    shape the batch autotuner picks, and the same launch with wide clusters
    only; with `extras`, also the resident-ring form and one step call per
    chain."""
    import torch
    import workloads
    from paper_1412_0544_amd import Batch, Chain, autotune
    from paper_1412_0544_amd import _lib as L
    lengths = workloads.batch_lengths(count)
    tot = int(lengths.sum())
    out = {"chains": count, "sites": tot, "steps": steps}
    for prec in precs:
        dtype = torch.float64 if prec == "fp64" else torch.float32
        if host_ics:
            import numpy as np
            npt = np.float64 if prec == "fp64" else np.float32
            chains = [Chain(*workloads.chain_ics(int(n_), 1000 + i, dtype=npt), dt, prec=prec,
                            device=dev) for i, n_ in enumerate(lengths)]
        else:
            chains = [Chain(*workloads.chain_ics_torch(int(n_), 1000 + i, dev, dtype), dt,
                            prec=prec, device=dev) for i, n_ in enumerate(lengths)]
        if shape:
            S, K = shape
        else:
            # the batch autotuner picks (sites per lane, depth) on these chains
            (S, K), table = autotune.tune_batch(chains, use_cache=False)
            out[f"{prec}_autotune_su_per_s"] = {f"s{s_}_k{k_}": v for (s_, k_), v in table.items()}
        b = Batch(chains, max_steps=steps, sites_per_lane=S, kdepth=K)
        b.step(24)
        b.check()
        t = ev_seconds(lambda: b.step(steps), chains[0].stream)
        b.check()
        plan = b.plan()
        ops = OPS_PER_SU["quartic"] if prec == "fp64" else OPS_PER_SU_FP32_KAHAN
        peak = VALU_PEAK_TOPS if prec == "fp64" else FP32_VALU_PEAK_TOPS
        a = ops * tot * steps / t / 1e12
        E = 64 * S * plan["waves_per_cluster"]
        nar = plan["narrow_clusters"]
        lane_sites = (plan["total_clusters"] - nar) * E + nar * 64 * S
        # the same launch with wide clusters only (no one-wavefront clusters)
        bw = Batch(chains, max_steps=steps, sites_per_lane=S, kdepth=K, flags=L.CHAIN_BATCH_WIDE_ONLY)
        bw.step(24)
        bw.check()
        tw = ev_seconds(lambda: bw.step(steps), chains[0].stream)
        bw.check()
        pw = bw.plan()
        bw.close()
        out[prec] = {"su_per_s": tot * steps / t, "ms": t * 1e3, "sites_per_lane": S,
                     "kdepth": K, "grid_blocks": plan["grid_blocks"],
                     "resident_chains": plan["resident_chains"],
                     "clusters": plan["total_clusters"], "narrow_clusters": nar,
                     "kept_lane_site_frac": tot / lane_sites,
                     "wide_only": {"su_per_s": tot * steps / tw, "clusters": pw["total_clusters"],
                                   "kept_lane_site_frac": tot / (pw["total_clusters"] * E)},
                     "roofline": {"bound": "alu", "achieved": a, "peak": peak, "unit": "Tops/s",
                                  "frac": a / peak, "ops_per_su": ops,
                                  "timed": "device time of one persistent launch"}}
        b.close()
        if not extras:
            for c in chains:
                c.close()
            continue
        # the same with the rings of <= 1024 sites kept on chip for all steps
        b = Batch(chains, max_steps=steps, sites_per_lane=S, kdepth=K,
                  flags=L.CHAIN_BATCH_RESIDENT_RINGS)
        b.step(24)
        b.check()
        t = ev_seconds(lambda: b.step(steps), chains[0].stream)
        b.check()
        out[f"{prec}_resident_rings_su_per_s"] = tot * steps / t
        b.close()
        if prec == "fp64":
            # the same chains, one step call per chain (100 steps each)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in chains:
                c.step(100)
            torch.cuda.synchronize()
            out["fp64_one_call_per_chain_su_per_s"] = tot * 100 / (time.perf_counter() - t0)
        for c in chains:
            c.close()
    return out


def variant_persistent_single(qd, pd, dt, dev, steps=1000):
    """The bench chain as a batch of one: one persistent launch for all the
    steps of a job (the batch's default shape), against the per-pass fused
    launches of the headline."""
    from paper_1412_0544_amd import Batch, Chain
    ch = Chain(qd, pd, dt, device=dev)
    b = Batch([ch], max_steps=steps)
    b.step(32)
    t = ev_seconds(lambda: b.step(steps), ch.stream)
    b.check()
    b.close()
    ch.close()
    return qd.numel() * steps / t


# Served jobs: HBM budget of the default run. The largest job (4e6 sites,
# 32 bytes per site with its workspace) takes 128 MB, so 256 MiB holds two of
# them; with 4 GiB the server never came near its budget (peak 0.33 GB over
# 500 jobs at load 0.8), so admission by footprint was never exercised.
SERVE_BUDGET = 256 << 20


def variant_serving(dt, dev, jobs=500, rho=0.8, rate_su=4e11, budget=SERVE_BUDGET, quantum=1000,
                    max_active=64, sites_per_lane=4):
    """Poisson arrivals at load rho of `rate_su`; N log-uniform in [1e3, 4e6],
    steps uniform in [1e3, 1e5], FP64/FP32 and quartic/harmonic each a coin;
    admission in arrival order while the HBM budget and a slot allow."""
    import workloads
    from paper_1412_0544_amd.serve import GpuExecutor, Server, percentiles
    mean_work = 4.82e5 * 5.05e4
    lam = rho * rate_su / mean_work
    js = workloads.served_jobs(jobs, lam, seed=5)
    ex = GpuExecutor(device=dev, dt=dt, quantum=quantum, max_active=max_active,
                     hbm_budget=budget, sites_per_lane=sites_per_lane)
    srv = Server(ex, hbm_budget=budget, max_active=max_active, quantum=quantum)
    t0 = time.perf_counter()
    res = srv.run(js)
    wall = time.perf_counter() - t0
    done = [r for r in res if r.status == "done"]
    su = sum(r.n * r.steps for r in done)
    lat = percentiles([r.latency for r in done])
    waited = [r for r in done if r.waited_for_memory]
    return {"jobs": jobs, "done": len(done), "arrival_rate_per_s": lam, "rho": rho,
            "hbm_budget_bytes": budget, "quantum": quantum, "max_active": max_active,
            "latency_s": lat, "queue_s": percentiles([r.queue_s for r in done]),
            "service_s": percentiles([r.service_s for r in done]),
            "rejected": sum(r.status == "rejected" for r in res),
            "failed": sum(r.status == "failed" for r in res),
            "waited_for_memory": len(waited),
            "queue_s_of_memory_waits": percentiles([r.queue_s for r in waited]),
            "jobs_per_s": len(done) / wall, "su_per_s": su / wall, "wall_s": wall,
            "rounds": srv.rounds, "peak_hbm_bytes": srv.peak_used,
            "peak_hbm_frac_of_budget": srv.peak_used / budget}


def size_sweep(dev, dt=0.01, steps=50, trials=10, exps=range(10, 27, 2)):
    """Fused (library plan) vs the per-stage baseline over chain length, with
    the paper's protocol: T steps from random initial conditions, the best
    of M trials, Perf = T / t_wall (Sec. 3.2, Eq. 8)."""
    import torch
    import workloads
    from paper_1412_0544_amd import Chain
    rows = []
    for e in exps:
        n = 1 << e
        q, p = workloads.chain_ics_torch(n, 0, dev)
        row = {"n": n, "state_bytes": 16 * n}
        for method in ("fused", "naive"):
            ch = Chain(q, p, dt, method=method, device=dev)
            ch.step(steps)
            best = min(ev_seconds(lambda: ch.step(steps), ch.stream) for _ in range(trials))
            row[method] = {"su_per_s": n * steps / best, "steps_per_s": steps / best,
                           "plan": {k: v for k, v in ch.plan().items()
                                    if k in ("resident", "sites_per_lane", "waves_per_cluster",
                                             "kdepth")}}
            ch.close()
        row["speedup"] = row["fused"]["su_per_s"] / row["naive"]["su_per_s"]
        log(f"[bench] N=2^{e}: fused {row['fused']['su_per_s']:.3e}, naive "
            f"{row['naive']['su_per_s']:.3e}, x{row['speedup']:.1f}")
        rows.append(row)
        del q, p
        torch.cuda.empty_cache()
    return rows


def roessler_shapes():
    return [(s, w, k) for s in (4, 6, 8) for w in (1, 2, 4, 8) for k in (8, 13, 16, 21, 25, 32)
            if 64 * s * w > 16 * k and (s != 6 or w == 4)]


def variant_roessler(dev, dt=0.01, n=1 << 20, steps=50, trials=10, shapes=None, sweep=True):
    """The paper's performance protocol on its own workload (Sec. 3.2): a
    Roessler chain of N = 2^20 from random initial conditions, T = 50 steps
    of dt = 0.01, the best of M = 10 trials, Perf = T / t_wall (Eq. 8). The
    wall time brackets the step call and a stream synchronisation. Beside it
    the device time per call (HIP events, best of M) around a run of
    RUN_CALLS back-to-back calls, which the roofline uses, and around a lone
    call (which also holds the launch latency). Fused at the library plan
    (eager and replayed from a graph), the exchange form, every cluster
    shape in `shapes`, and the one-kernel-per-stage method."""
    import torch
    import workloads
    from paper_1412_0544_amd import RoesslerChain
    x0, y0, z0 = (torch.from_numpy(v).to(dev) for v in workloads.roessler_ics(n, 0))

    def measure(**kw):
        ch = RoesslerChain(x0, y0, z0, dt, device=dev, **kw)
        ch.step(steps)
        torch.cuda.synchronize()
        walls, gpus, runs = [], [], []
        for _ in range(trials):
            t = time.perf_counter()
            gpus.append(ev_seconds(lambda: ch.step(steps), ch.stream))
            walls.append(time.perf_counter() - t)
        # device time per call in a run of back-to-back calls (events around
        # the run): a lone call's events also hold the launch latency
        for _ in range(trials):
            runs.append(ev_seconds(lambda: [ch.step(steps) for _ in range(RUN_CALLS)],
                                   ch.stream) / RUN_CALLS)
        plan = ch.plan()
        ch.close()
        w, g, r = min(walls), min(gpus), min(runs)
        return {"steps_per_s": steps / w, "su_per_s": n * steps / w,
                "device_single_call_su_per_s": n * steps / g,
                "device_steps_per_s": steps / r, "device_su_per_s": n * steps / r,
                "plan": {k: plan[k] for k in ("sites_per_lane", "waves_per_cluster", "kdepth",
                                              "tile", "halo", "waves", "exchange")}}

    RUN_CALLS = 20
    out = {"n": n, "steps": steps, "trials": trials, "dt": dt, "run_calls": RUN_CALLS}
    # bring the device to its working clock first: the first timed calls of
    # a cold device ran up to 13% slower than the same calls later in the run
    ch = RoesslerChain(x0, y0, z0, dt, device=dev)
    t_end = time.perf_counter() + 0.5
    while time.perf_counter() < t_end:
        ch.step(steps * 20)
        torch.cuda.synchronize()
    ch.close()
    log("[bench] Roessler: library plan")
    out["fused"] = measure()
    out["fused_graph"] = measure(graph=True)
    # the whole chain held in registers for each call, clusters swapping only
    # edge sites between passes (one launch per call); where the chain fits
    from paper_1412_0544_amd import ChainError
    try:
        out["exchange"] = measure(exchange=True)
        x = out["exchange"]
        out["exchange"]["roofline"] = roofline(n, steps, n * steps / x["device_su_per_s"],
                                               model="roessler")
        if sweep:
            xt = {}
            for s_, w in ((4, 4), (4, 8), (6, 4), (6, 2), (8, 2)):
                for k in (6, 8, 10, 13, 17, 21, 25, 32):
                    try:
                        xt[f"s{s_}_w{w}_k{k}"] = measure(sites_per_lane=s_, waves_per_cluster=w,
                                                         kdepth=k,
                                                         exchange=True)["device_su_per_s"]
                    except ChainError:
                        pass
            out["exchange_shapes_device_su_per_s"] = xt
    except ChainError as e:
        out["exchange"] = {"not_held": str(e)}
    log("[bench] Roessler: per-stage baseline")
    out["naive"] = measure(method="naive")
    table = {}
    for s, w, k in (shapes or roessler_shapes()) if sweep else ():
        table[f"s{s}_w{w}_k{k}"] = measure(sites_per_lane=s, waves_per_cluster=w, kdepth=k,
                                          graph=True)["device_su_per_s"]
    if table:
        out["shapes_device_su_per_s"] = table
        out["best_shape"] = max(table, key=table.get)
    out["speedup_fused_vs_naive"] = out["fused"]["steps_per_s"] / out["naive"]["steps_per_s"]
    # roofline of the library plan's passes (device time over the launches)
    f = out["fused"]
    k = f["plan"]["kdepth"]
    plan = {"resident": 0, "kdepth": k}
    launches = fused_launches(plan, steps)
    out["roofline"] = roofline(n, steps / launches, n * steps / f["device_su_per_s"] / launches,
                               model="roessler")
    log(f"[bench] Roessler: fused {f['steps_per_s']:.0f} steps/s (device "
        f"{f['device_steps_per_s']:.0f}), naive {out['naive']['steps_per_s']:.0f}" +
        (f", best shape {out['best_shape']} {table[out['best_shape']]:.3e} SU/s" if table else ""))
    return out


def variant_short_rings(dt, dev, steps=1000, jobs=5):
    """Short rings, 1000-step jobs: the ring kept resident in one workgroup
    (all steps in one launch) against the tiled plan (one launch per pass),
    eager and replayed from a graph; p50 wall time of a job (step call plus
    stream synchronisation)."""
    import torch
    import workloads
    from paper_1412_0544_amd import Chain
    out = {}
    for n in (256, 1024, 4096):
        q0, p0 = workloads.chain_ics(n, 0)
        row = {}
        for name, kw in (("resident", {"resident": True}), ("tiled", {}),
                         ("tiled_graph", {"graph": True})):
            ch = Chain(q0, p0, dt, device=dev, **kw)
            ch.step(steps)
            torch.cuda.synchronize()
            lat = []
            for _ in range(jobs):
                t = time.perf_counter()
                ch.step(steps)
                ch.stream.synchronize()
                lat.append(time.perf_counter() - t)
            plan = ch.plan()
            ch.close()
            row[name] = {"p50_ms": 1e3 * pct(lat, 50),
                         "plan": {x: plan[x] for x in ("resident", "sites_per_lane",
                                                       "waves_per_cluster", "kdepth")}}
        out[str(n)] = row
    return out


def variant_nnn(qd, pd, dt, n, dev, steps=480, sweep=False):
    """The quartic chain with second-neighbour bonds on the bench chain: the
    library plan (halo 4 per step) and the per-stage baseline, device time of
    `steps` steps (best of 3); with `sweep`, every cluster shape at depths 8,
    12 and 16 (device time of 96 steps)."""
    from paper_1412_0544_amd import Chain
    out = {}
    if sweep:
        table = {}
        for s_ in (2, 4, 8):
            for w in (1, 2, 4, 8):
                for k in (8, 12, 16):
                    if 64 * s_ * w <= 16 * k:
                        continue
                    ch = Chain(qd, pd, dt, model="quartic_nnn", sites_per_lane=s_,
                               waves_per_cluster=w, kdepth=k, device=dev)
                    ch.step(k)
                    best = min(ev_seconds(lambda: ch.step(96), ch.stream) for _ in range(3))
                    ch.close()
                    table[f"s{s_}_w{w}_k{k}"] = n * 96 / best
        out["shapes_su_per_s"] = table
        out["best_shape"] = max(table, key=table.get)
        log(f"[bench] NNN shapes: best {out['best_shape']} {table[out['best_shape']]:.3e} SU/s")
    for method in ("fused", "naive"):
        ch = Chain(qd, pd, dt, model="quartic_nnn", method=method, device=dev)
        ch.step(32)
        k = steps if method == "fused" else 20
        best = min(ev_seconds(lambda: ch.step(k), ch.stream) for _ in range(3))
        plan = ch.plan()
        ch.close()
        out[method] = {"su_per_s": n * k / best,
                       "plan": {x: plan[x] for x in ("sites_per_lane", "waves_per_cluster",
                                                     "kdepth", "halo", "tile")}}
    f = out["fused"]
    launches = fused_launches({"resident": 0, "kdepth": f["plan"]["kdepth"]}, steps)
    out["roofline"] = roofline(n, steps / launches, n * steps / f["su_per_s"] / launches,
                               model="quartic_nnn")
    out["speedup_fused_vs_naive"] = f["su_per_s"] / out["naive"]["su_per_s"]
    return out


def tableau_ops_per_su(a, b, force_ops=OPS_PER_SU["quartic"] - 14):
    """VALU ops of one site-update of the tableau kernel: per stage the
    force (`force_ops` / 4 for the quartic chain) plus, from stage 2 on, two
    fma per earlier stage and two to form the argument; the final
    combination is two fma per stage plus two."""
    s = len(b)
    f = force_ops // 4
    return s * f + sum(2 * j + 2 for j in range(1, s)) + 2 * s + 2


def tableau_executed_ops_per_su(a, b, force_ops=4 * EXECUTED_FORCE_OPS["quartic"]):
    """VALU ops the tableau kernel executes per site-update: the force as the
    kernels form it (`force_ops` / 4), and for dq/dt = p stage j's argument as
    q + hc_j p + sum_{l<j-1} g_jl F_l (j ops) and the update in two sums (one
    fma each per stage), then 3 ops."""
    s = len(b)
    f = force_ops // 4
    return s * f + s * (s - 1) // 2 + 2 * s + 3


def variant_tableaus(qd, pd, dt, n, dev, steps=192, sweep=False):
    """Explicit methods by Butcher tableau on the bench chain (library plan,
    device time of `steps` steps, best of 3): site-updates/s and the VALU
    roofline of each; with `sweep`, also every cluster shape and depth the
    tableau kernel is built for."""
    from paper_1412_0544_amd import Chain, tableaus

    def timed(a, b, k=steps, **kw):
        ch = Chain(qd, pd, dt, tableau=(a, b), device=dev, **kw)
        ch.step(4)
        best = min(ev_seconds(lambda: ch.step(k), ch.stream) for _ in range(3))
        plan = ch.plan()
        ch.close()
        return n * k / best, plan

    out = {}
    for name, (a, b) in tableaus.ALL.items():
        su, plan = timed(a, b)
        naive, _ = timed(a, b, k=8, method="naive")
        ops = tableau_ops_per_su(a, b)
        ex = tableau_executed_ops_per_su(a, b)
        out[name] = {"stages": len(b), "su_per_s": su, "ops_per_su": ops,
                     "valu_frac": su * ops / (VALU_PEAK_TOPS * 1e12),
                     "executed_ops_per_su": ex,
                     "executed_valu_frac": su * ex / (VALU_PEAK_TOPS * 1e12),
                     "naive_su_per_s": naive, "speedup_fused_vs_naive": su / naive,
                     "plan": {x: plan[x] for x in ("sites_per_lane", "waves_per_cluster", "kdepth",
                                                   "halo", "tile")}}
        log(f"[bench] tableau {name}: {su:.3e} SU/s, {out[name]['executed_valu_frac']:.2f} of VALU "
            f"peak ({ex} executed ops/SU); "
            f"per-stage {naive:.3e} SU/s")
        if sweep:
            table = {}
            for s_ in ((4, 8) if len(b) <= 4 else (4,)):
                for w in (1, 4):
                    for k in (8, 16, 32):
                        table[f"s{s_}_w{w}_k{k}"] = timed(a, b, sites_per_lane=s_,
                                                          waves_per_cluster=w, kdepth=k)[0]
            out[name]["shapes_su_per_s"] = table
    return out


def plan_sweep(dev, dt=0.01, steps=64, exps=range(10, 27, 2), precs=("fp64", "fp32_kahan")):
    """Cluster shape by chain length (the granularity study of Sec. 2.3 and
    Sec. 3.2.1, over S, W, k and N): device time of `steps` steps, best of 3,
    replayed from a captured graph so that launch overhead counts as little
    as it can; the resident ring where it applies."""
    import torch
    import workloads
    from paper_1412_0544_amd import Chain
    out = {}
    for prec in precs:
        dtype = torch.float64 if prec == "fp64" else torch.float32
        rows = []
        for e in exps:
            n = 1 << e
            q, p = workloads.chain_ics_torch(n, 0, dev, dtype)
            table = {}

            def timed(**kw):
                ch = Chain(q, p, dt, prec=prec, device=dev, graph=True, **kw)
                ch.step(steps)
                best = min(ev_seconds(lambda: ch.step(steps), ch.stream) for _ in range(3))
                ch.close()
                return n * steps / best

            if n <= 4096:
                table["resident"] = timed(resident=True)
            for s_ in ((2, 4, 6, 8, 16) if prec == "fp64" else (2, 4, 8, 16)):
                for w in (1, 2, 4, 8):
                    for k in (4, 8, 16, 24, 32):
                        if 64 * s_ * w > 4 * k + 16:
                            table[f"s{s_}_w{w}_k{k}"] = timed(sites_per_lane=s_, waves_per_cluster=w,
                                                              kdepth=k, resident=False)
            best = max(table, key=table.get)
            rows.append({"n": n, "best": best, "best_su_per_s": table[best], "table": table})
            log(f"[bench] plan sweep {prec} N=2^{e}: best {best} {table[best]:.3e} SU/s")
            del q, p
            torch.cuda.empty_cache()
        out[prec] = rows
    return out


def variant_naive(qd, pd, dt, n, dev):
    from paper_1412_0544_amd import Chain
    ch = Chain(qd, pd, dt, method="naive", device=dev)
    ch.step(2)
    _, g, _ = time_jobs(ch, 20, 2, with_energy=False)
    ch.close()
    return n * 20 / min(g)


def variant_ring1024(dt, dev):
    import workloads
    from paper_1412_0544_amd import Chain
    q0, p0 = workloads.chain_ics(1024, 0)
    ch = Chain(q0, p0, dt, device=dev)
    time_jobs(ch, 1000, 1)
    lat, g, _ = time_jobs(ch, 1000, 5)
    ch.close()
    return {"p50": 1e3 * pct(lat, 50), "gpu_min": 1e3 * min(g)}


def variants(qd, pd, dt, n, dev, sw, serve_jobs=500):
    """Other rows of the hot path, each measured at its own configuration. A
    variant that fails records its error; the others and the headline line
    still come out."""
    from paper_1412_0544_amd import autotune
    res = {}

    def run(key, title, fn):
        log(f"[bench] variant: {title}")
        try:
            res[key] = fn()
        except Exception as e:  # noqa: BLE001 -- reported in the JSON line
            log(f"[bench] variant {key} failed: {e!r}")
            res[key] = {"error": repr(e)}

    run("fused_k_su_per_s", "temporal depth sweep", lambda: {
        str(k): autotune.time_shape(qd, pd, dt, (sw[0], sw[1], k), steps=48, device=dev)
        for k in (1, 2, 4, 8)})
    run("naive_su_per_s", "naive per-stage", lambda: variant_naive(qd, pd, dt, n, dev))
    run("persistent_single_su_per_s", "persistent single chain",
        lambda: variant_persistent_single(qd, pd, dt, dev))
    run("ring1024_1000steps_ms", "1024-site ring", lambda: variant_ring1024(dt, dev))
    run("short_rings_1000steps_ms", "short rings, resident vs tiled",
        lambda: variant_short_rings(dt, dev))
    run("precision", "FP32 with compensated update, 1e4 steps",
        lambda: variant_precision(n, dt, dev))
    run("batch4096", "4096-chain batch", lambda: variant_batch(dt, dev))
    run("tableaus", "explicit methods by Butcher tableau",
        lambda: variant_tableaus(qd, pd, dt, n, dev))
    run("quartic_nnn", "next-nearest-neighbour coupling", lambda: variant_nnn(qd, pd, dt, n, dev))
    run("roessler", "Roessler chain, the paper's protocol", lambda: variant_roessler(dev, dt))
    run("size_sweep", "chain length sweep N = 2^10..2^26 (every 4th power), fused vs per-stage",
        lambda: size_sweep(dev, trials=3, exps=range(10, 27, 4)))
    if serve_jobs:
        rate = res.get("batch4096", {}).get("fp64", {}).get("su_per_s", 4e11)
        run("serving", f"serving {serve_jobs} jobs at loads 0.5 and 0.8",
            lambda: {str(rho): variant_serving(dt, dev, jobs=serve_jobs, rho=rho, rate_su=rate)
                     for rho in (0.5, 0.8)})
    return res

if __name__ == "__main__":
    sys.exit(main())

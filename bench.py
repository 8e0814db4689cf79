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

# Algorithmic work of one site-update (one RK4 step of one site), quartic:
# force 7 ops (bond diff, 2 mul for the cube, q^2, fma, 2 sub) x 4 stages,
# stage arguments 2 fma x 3 stages, accumulators 3 ops x 2 components,
# final update 1 fma x 2 components.
OPS_PER_SU = {"quartic": 42, "harmonic": 30}
FLOPS_PER_SU = {"quartic": 58, "harmonic": 42}
# Bytes per site-update of one pass: read q, p and write q, p once.
BYTES_PER_SITE_PASS = {"fp64": 32, "fp32_kahan": 32}   # FP32: q, p, cq, cp


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
    bytes_alg = BYTES_PER_SITE_PASS[prec] * n
    ops_alg = OPS_PER_SU[model] * n * ksteps
    t_hbm = bytes_alg / (HBM_PEAK_GBPS * 1e9)
    t_alu = ops_alg / (VALU_PEAK_TOPS * 1e12)
    hbm = {"achieved": bytes_alg / t_launch / 1e9, "peak": HBM_PEAK_GBPS, "unit": "GB/s"}
    alu = {"achieved": ops_alg / t_launch / 1e12, "peak": VALU_PEAK_TOPS, "unit": "Tops/s"}
    for d in (hbm, alu):
        d["frac"] = d["achieved"] / d["peak"]
    if t_alu >= t_hbm:
        r = {"bound": "alu", **alu, "op": "FP64 VALU lane-op (an fma is one op)",
             "flops_TFLOPs": FLOPS_PER_SU[model] * n * ksteps / t_launch / 1e12,
             "hbm_view": hbm}
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


def cpu_baseline(n, dt, target_s=10.0):
    import numpy as np
    import oracle
    import workloads
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    q0, p0 = workloads.chain_ics(n, 0)
    t = time.perf_counter()
    oracle.rk4(oracle.QUARTIC, q0, p0, dt, 1, threads=threads)
    one = time.perf_counter() - t
    steps = max(1, min(200, int(target_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.rk4(oracle.QUARTIC, q0, p0, dt, steps, threads=threads)
    el = time.perf_counter() - t
    return {"value": n * steps / el, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"quartic chain N={n}, {steps} RK4 steps from seed-0 ICs, "
                      f"{threads} OpenMP threads, {el:.1f} s"}


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
    ap.add_argument("--sweep", action="store_true", help="time the full (S, W, k) grid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
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
    n, dt, js = args.n, 0.01, args.job_steps
    log(f"[bench] generating ICs n={n}")
    q0, p0 = workloads.chain_ics(n, 0)
    qd = torch.from_numpy(q0).to(dev)
    pd = torch.from_numpy(p0).to(dev)

    from paper_1412_0544_amd import autotune
    sweep = {}
    if args.sites and args.waves and args.kdepth:
        S, W, K = args.sites, args.waves, args.kdepth
    else:
        cands = None
        if args.sweep:
            cands = [(s, w, k) for s in autotune.SITES for w in autotune.WAVES
                     for k in autotune.DEPTHS if 64 * s * w > 16 * k]
        log("[bench] autotuning the cluster shape")
        (S, W, K), table = autotune.tune(n, q=qd, p=pd, dt=dt, candidates=cands, device=dev,
                                        use_cache=False)
        sweep = {f"s{s}_w{w}_k{k}": v for (s, w, k), v in sorted(table.items())}
    log(f"[bench] plan S={S} W={W} K={K}")

    ch = Chain(qd, pd, dt, sites_per_lane=S, waves_per_cluster=W, kdepth=K, resident=False,
               device=dev)
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
    rl = roofline(n, js / launches, t_launch)
    rl["launches_per_job"] = launches
    rl["traffic"] = None

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "quartic chain, N=2^24, periodic, q,p~U[-1,1) seed 0, dt=0.01, "
                               "1000 RK4 steps per job + energy",
                   "n": n, "job_steps": js, "sites_per_lane": S, "waves_per_cluster": W,
                   "kdepth": K, "tile": plan["tile"], "halo": plan["halo"],
                   "overlap_factor": plan["overlap_factor"]},
        "hbm_roofline_pct": 100.0 * value / (HBM_PEAK_GBPS * 1e9 / 32),
        "latency_ms": {"p50": 1e3 * pct(lat, 50), "p99": 1e3 * pct(lat, 99)},
        "roofline": rl,
        "energy_final": e_final,
    }
    if sweep:
        out["autotune_su_per_s"] = sweep

    if not args.no_variants:
        out["variants"] = variants(qd, pd, dt, n, dev, (S, W))

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(n, dt)
    print(json.dumps(out), flush=True)
    return 0


def variants(qd, pd, dt, n, dev, sw):
    """Other rows of the hot path, measured briefly at the same N."""
    from paper_1412_0544_amd import Chain, autotune
    import workloads
    res = {}
    # temporal depth k = 1, 2, 4, 8 at the tuned cluster shape
    res["fused_k_su_per_s"] = {
        str(k): autotune.time_shape(qd, pd, dt, (sw[0], sw[1], k), steps=48, device=dev)
        for k in (1, 2, 4, 8)}
    # the standard implementation: one kernel per stage
    ch = Chain(qd, pd, dt, method="naive", device=dev)
    ch.step(2)
    _, g, _ = time_jobs(ch, 20, 2, with_energy=False)
    res["naive_su_per_s"] = n * 20 / min(g)
    ch.close()
    # FP32 state with compensated update
    res["fp32_kahan_su_per_s"] = autotune.time_shape(
        qd.float(), pd.float(), dt, (16, 4, 12), prec="fp32_kahan", steps=96, device=dev)
    # the 1024-site ring resident on chip, 1000 steps per job
    q0, p0 = workloads.chain_ics(1024, 0)
    ch = Chain(q0, p0, dt, device=dev)
    time_jobs(ch, 1000, 1)
    lat, g, _ = time_jobs(ch, 1000, 5)
    res["ring1024_1000steps_ms"] = {"p50": 1e3 * pct(lat, 50), "gpu_min": 1e3 * min(g)}
    ch.close()
    return res


if __name__ == "__main__":
    sys.exit(main())

"""Benchmark: Monte Carlo throughput of the forest-subtracted AMM integrands.

Workload (the configuration the metric is quoted on that fits one GPU): all
10 three-loop self-energy graphs without lepton loops (50 vertex graphs, 8
Feynman parameters), plain combinatorial density (Calc 2 constants), FP64,
Philox seed 0; one step evaluates `--batch` consecutive sample counters of
every graph (the full configuration is 1e9 counters per graph = 1e9/batch
steps).  Inputs are generated on the device from the counters, so nothing is
copied from the host inside the timed region.

Prints one JSON line (see the repository's bench contract).
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12     # MI355X: 256 CUs x 128 FP64 flop/clk x 2.4 GHz (FMA = 2)


def cpu_baseline(seconds_target=15.0):
    """Time the oracle (as it stands) on the host: 3-loop graph 0."""
    import numpy as np
    from oracle import estimate as E
    from oracle import integrand as I
    cache = os.path.join(ROOT, 'tests', 'golden', 'oracle_level_polys.json.gz')
    if os.path.exists(cache):
        I.load_poly_cache(cache)
    E.run(3, 0, 0, 0, 200)            # warm (derives tables if no cache)
    n = 2000
    t0 = time.perf_counter()
    E.run(3, 0, 0, 0, n, chunk=n)
    dt = time.perf_counter() - t0
    reps = max(1, int(seconds_target / max(dt, 1e-3)))
    reps = min(reps, 2000)
    t0 = time.perf_counter()
    E.run(3, 0, 0, 0, n * reps, chunk=n)
    dt = time.perf_counter() - t0
    cpu = platform.processor() or platform.machine()
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                cpu = line.split(':', 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n * reps / dt, "unit": "integrand evals/s (3-loop SE-graph samples, 5 insertions each)",
            "cores": 1, "kind": "oracle",
            "sample": f"3-loop SE graph 0, counters [0, {n * reps}) of seed 0, numpy FP64 oracle in one process "
                      f"({cpu}); the oracle's one-time numerator derivation is excluded",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=5)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--batch', type=int, default=3_276_800,
                    help='sample counters per graph per step (10 x 3276800 = one group of 32000 chunks)')
    ap.add_argument('--pilot', type=int, default=100_000, help='double-double pilot samples per graph')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) != 1:
        print('bench.py: this build runs on one GPU only; multi-GPU runs are not part of it '
              '(samples shard by Philox counter range across GPUs)', file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1909_08015_amd import Context

    ctx = Context(0)
    ctx.enumerate(3)
    ctx.build_tables()
    G = ctx.n_se
    flops = [ctx.plan_stats(g)['flops_per_sample'] for g in range(G)]
    stream = torch.cuda.current_stream()
    B = args.batch
    # pilot (every point in double-double, seed 1) -> round-off acceptance
    # thresholds of eq. (interval_accept) for the full 1e9-sample run
    ctx.integrate(seed=1, n_per_graph=args.pilot, force_flag=1)
    tau = ctx.accept_thresholds(1_000_000_000)
    counter = 0
    first = True
    for _ in range(args.warmup):
        ctx.integrate(seed=0, n_per_graph=B, counter0=counter, accumulate=0 if first else 1, accept_tau=tau)
        first = False
        counter += B
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.integrate(seed=0, n_per_graph=B, counter0=counter, accumulate=0 if first else 1, accept_tau=tau,
                      stream=stream)
        first = False
        counter += B
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile(False)
    samples = args.steps * B * G
    value = samples / dt
    total_flops = sum(flops) * args.steps * B
    achieved = total_flops / (prof['ms_fp64'] * 1e-3) if prof['ms_fp64'] > 0 else 0.0
    est = ctx.read(-1, -1, None)
    out = {
        "metric": "integrand evals/s + FP64 % of peak; sigma^2*time learned vs plain sampler, 5-loop",
        "value": value,
        "unit": "integrand evals/s (3-loop SE-graph samples, 5 vertex-graph insertions each)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3-loop set: all 10 three-loop no-lepton-loop SE graphs, 8 Feynman "
                               "parameters, plain combinatorial density (Calc 2), FP64, Philox seed 0; "
                               f"one step = {B} sample counters per graph",
                   "graphs": G, "loops": 3, "batch_per_graph": B, "counters_done": counter},
        "vertex_graph_evals_per_s": value * 5,
        "fp64_frac_of_peak": achieved / PEAK_FP64_VALU,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": None,
                     "kernel": "k_integrate<3>", "kernel_ms": prof['ms_fp64'],
                     "kernel_launches": prof['launches'],
                     "flops_per_sample": {str(g): flops[g] for g in range(G)}},
        "phase_ms": {"fp64": prof['ms_fp64'], "dd": prof['ms_dd'], "reduce": prof['ms_reduce']},
        "estimate_3loop_so_far": {"mean": est['mean'], "sigma": est['sigma'], "n": est['n'],
                                  "n_flag": est['n_flag'], "n_dd_fail": est['n_dd_fail'], "n_ood": est['n_ood']},
        "flag_rate": est['n_flag'] / max(est['n'], 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()

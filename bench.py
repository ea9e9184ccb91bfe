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


def counters_record():
    """HBM bytes and executed FP64 flops per sample of the 3-loop FP64 pass,
    from the committed rocprofv3 counter runs, if they were taken on this very
    library build (same sha256); else None."""
    import hashlib
    rec_path = os.path.join(ROOT, 'profiles', 'k_integrate_3loop_counters.json')
    lib_path = os.path.join(ROOT, 'paper_1909_08015_amd', 'libamm.so')
    try:
        rec = json.load(open(rec_path))
        sha = hashlib.sha256(open(lib_path, 'rb').read()).hexdigest()
    except (OSError, ValueError):
        return None
    return rec if rec.get('libamm_sha256') == sha else None


def _progress(msg):
    """One line per finished phase on stderr (stdout carries the JSON line)."""
    print(f'bench: {msg}', file=sys.stderr, flush=True)


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def learned_vs_plain(ctx, tau, n):
    """sigma^2 * time of the learned mixture against the plain density on the
    3-loop set: pilot (seed 1, 1e6 samples per graph) -> MLP training on the
    GPU -> n samples per graph of each sampler on seed 0; sigma^2 summed over
    graphs (per graph the sum of its class variances)."""
    import torch
    G = ctx.n_se
    t_pilot = _timed(torch, lambda: ctx.pilot(1, 1_000_000))
    t_train = _timed(torch, lambda: ctx.mlp_train(300, lr=1e-2, init_seed=0))
    res = {}
    for name, smp in (('plain', 0), ('learned', 1)):
        ctx.integrate(seed=0, n_per_graph=n, sampler=smp, accept_tau=tau)          # warm
        dt = _timed(torch, lambda: ctx.integrate(seed=0, n_per_graph=n, sampler=smp, accept_tau=tau))
        var = sum(ctx.read(g, -1)['sigma'] ** 2 for g in range(G))
        res[name] = (var, dt)
    (vp, tp), (vl, tl) = res['plain'], res['learned']
    return {"sigma2_time_ratio_learned_over_plain": (vl * tl) / (vp * tp), "var_plain": vp, "var_learned": vl,
            "s_plain": tp, "s_learned": tl, "samples_per_graph": n, "pilot_samples_per_graph": 1_000_000,
            "pilot_s": t_pilot, "train_epochs": 300, "train_s": t_train, "loops": 3}


def measured_costs(ctx, tau, n):
    """t_j of Sec. IV.C as measured: seconds per sample of each graph run
    alone (n samples, FP64 pass, recompute and reduction), after a warm-up."""
    import torch
    t = []
    for g in range(ctx.n_se):
        tg = [tau[g]] if tau is not None else None
        ctx.integrate(seed=5, n_per_graph=max(n // 4, 1024), graph_begin=g, graph_end=g + 1, accept_tau=tg)
        dt = _timed(torch, lambda: ctx.integrate(seed=5, n_per_graph=n, graph_begin=g, graph_end=g + 1,
                                                 accept_tau=tg))
        t.append(dt / n)
    return t


def adaptive_vs_equal(ctx, tau, n, seed=0, rounds=2, floor_frac=0.25, cost=None):
    """sigma^2 * time of the adaptive split of samples over graphs (Sec. IV.C;
    pilot n/10 per graph, then rounds split by C_j / sqrt(t_j)) against an
    equal split of n samples per graph at the same plan cost.  sigma^2 of the
    total over graphs (eq. sigma_sum), as measured, and as implied by the
    equal run's per-graph deviations C_j for the adaptive sample counts
    (sum_j C_j^2 / n_j: heavy tails make one run's sigma^2 fluctuate)."""
    import torch
    res = {}
    for name in ('equal', 'adaptive', 'equal', 'adaptive'):                      # second pass warm
        if name == 'equal':
            dt = _timed(torch, lambda: ctx.integrate(seed=seed, n_per_graph=n, accept_tau=tau))
            done = [n] * ctx.n_se
            c2 = [ctx.read(g)['sigma'] ** 2 * n for g in range(ctx.n_se)]
        else:
            box = []
            dt = _timed(torch, lambda: box.append(ctx.integrate_adaptive(
                seed=seed, n_pilot=max(n // 10, 1024), budget_per_graph=n, n_rounds=rounds, floor_frac=floor_frac,
                cost=cost, accept_tau=tau)))
            done = box[0]
        tot = ctx.read(-1, -1, None)
        res[name] = (tot['sigma'] ** 2, dt, tot['mean'], done)
    (ve, te, me, _), (va, ta, ma, done) = res['equal'], res['adaptive']
    implied = sum(c / k for c, k in zip(c2, done)) / sum(c / n for c in c2)
    return {"sigma2_time_ratio_adaptive_over_equal": (va * ta) / (ve * te),
            "implied_sigma2_time_ratio": implied * ta / te, "implied_var_ratio": implied,
            "var_equal": ve, "var_adaptive": va, "s_equal": te, "s_adaptive": ta, "mean_equal": me,
            "mean_adaptive": ma, "samples_per_graph_equal": n, "samples_per_graph_adaptive_min": min(done),
            "samples_per_graph_adaptive_max": max(done), "rounds": rounds, "floor_frac": floor_frac, "seed": seed,
            "cost": "plan flops per sample" if cost is None else "measured seconds per sample"}


def second_calculation(ctx, n):
    """Calc 1 (Sec. V: MRG32k3a, C2..C4 = .03/.035/.035) next to Calc 2
    (Philox4x32-10, .03/.01/.06) on the 3-loop set, n samples per graph each:
    samples/s of each run and the graph-by-graph combination (eq. sigma_sum
    after combining)."""
    import torch
    from paper_1909_08015_amd import CALC1, CALC2
    from paper_1909_08015_amd.amm import OPT_GENERATOR, combine
    res = {}
    try:
        for name, gen, params in (('calc2', 0, CALC2), ('calc1', 1, CALC1)):
            ctx.set_option(OPT_GENERATOR, gen)
            ctx.build_tables(params=params)
            ctx.integrate(seed=1, n_per_graph=100_000, force_flag=1)
            tau = ctx.accept_thresholds(n)
            ctx.integrate(seed=7, n_per_graph=n // 4, accept_tau=tau)                       # warm
            dt = _timed(torch, lambda: ctx.integrate(seed=7, n_per_graph=n, accept_tau=tau))
            per = [ctx.read(g) for g in range(ctx.n_se)]
            tot = ctx.read(-1, -1, None)
            res[name] = {"samples_per_s": ctx.n_se * n / dt, "mean": tot['mean'], "sigma": tot['sigma'],
                         "means": [p['mean'] for p in per], "sigmas": [p['sigma'] for p in per]}
    finally:
        ctx.set_option(OPT_GENERATOR, 0)
        ctx.build_tables(params=CALC2)
    _, _, tm, ts = combine(res['calc1']['means'], res['calc1']['sigmas'], res['calc2']['means'],
                           res['calc2']['sigmas'])
    short = lambda r: {k: r[k] for k in ('samples_per_s', 'mean', 'sigma')}
    return {"calc1_mrg32k3a": short(res['calc1']), "calc2_philox": short(res['calc2']),
            "combined_mean": tm, "combined_sigma": ts, "samples_per_graph": n, "loops": 3}


def other_loop_orders(ctx, args):
    """Samples/s and FP64 fraction of peak at 1, 2 (generated code) and 4
    loops (74 graphs, table interpreter, one persistent launch per group,
    autotuned launch configuration)."""
    import torch
    out = {}
    for n, per_graph in ((1, 1 << 24), (2, 1 << 23), (4, 1 << 16)):
        ctx.enumerate(n)
        t_build = _timed(torch, lambda: ctx.build_tables())
        G = ctx.n_se
        flops = sum(ctx.plan_stats(g)['flops_per_sample'] for g in range(G))
        tau = None
        if n > 1:
            ctx.integrate(seed=1, n_per_graph=10_000 if n == 4 else 100_000, force_flag=1)
            tau = ctx.accept_thresholds(10 ** 10 // G if n == 4 else 10 ** 7)
        tune = None
        if n == 4:
            tune = ctx.autotune(seed=0, n_per_graph=8192, accept_tau=tau)
        ctx.integrate(seed=0, n_per_graph=per_graph // 4, accept_tau=tau)               # warm
        ctx.profile(True)
        dt = _timed(torch, lambda: ctx.integrate(seed=0, n_per_graph=per_graph, accept_tau=tau))
        prof = ctx.profile(False)
        est = ctx.read(-1, -1, None)
        achieved = flops * per_graph / (prof['ms_fp64'] * 1e-3)
        learned = None
        if n == 4:
            # learned sampler on the 4-loop set: pilot (seed 1) -> GPU training ->
            # sigma^2 * time of the learned mixture against the plain density
            t_pilot = _timed(torch, lambda: ctx.pilot(1, 50_000))
            t_train = _timed(torch, lambda: ctx.mlp_train(200, lr=1e-2, init_seed=0))
            res = {}
            for name, smp in (('plain', 0), ('learned', 1)):
                t = _timed(torch, lambda: ctx.integrate(seed=2, n_per_graph=per_graph, sampler=smp, accept_tau=tau))
                res[name] = (sum(ctx.read(g, -1)['sigma'] ** 2 for g in range(G)), t, ctx.read(-1, -1, None))
            (vp, tp, ep), (vl, tl, el) = res['plain'], res['learned']
            learned = {"sigma2_time_ratio_learned_over_plain": (vl * tl) / (vp * tp), "var_plain": vp,
                       "var_learned": vl, "s_plain": tp, "s_learned": tl, "mean_plain": ep['mean'],
                       "sigma_plain": ep['sigma'], "mean_learned": el['mean'], "sigma_learned": el['sigma'],
                       "pilot_samples_per_graph": 50_000, "pilot_s": t_pilot, "train_epochs": 200, "train_s": t_train,
                       "samples_per_graph": per_graph, "seed": 2}
        adaptive = adaptive_vs_equal(ctx, tau, per_graph, seed=3) if n == 4 else None
        _progress(f'{n}-loop set done')
        out[str(n)] = {"graphs": G, "samples_per_graph": per_graph, "samples_per_s": G * per_graph / dt,
                       "fp64_pass_ms": prof['ms_fp64'], "dd_ms": prof['ms_dd'],
                       "fp64_tflops": achieved / 1e12, "fp64_frac_of_peak": achieved / PEAK_FP64_VALU,
                       "flag_rate": est['n_flag'] / max(est['n'], 1), "n_dd_fail": est['n_dd_fail'],
                       "tables_build_s": t_build, "autotune": tune, "learned_vs_plain": learned,
                       "adaptive_vs_equal": adaptive,
                       "evaluator": "generated" if n < 4 else "interpreter, fused persistent launch"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=5)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--batch', type=int, default=3_276_800,
                    help='sample counters per graph per step (10 x 3276800 = one group of 32000 chunks)')
    ap.add_argument('--pilot', type=int, default=100_000, help='double-double pilot samples per graph')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-learned', action='store_true', help='skip the learned-sampler sigma^2*time measurement')
    ap.add_argument('--no-other-orders', action='store_true', help='skip the 1-, 2- and 4-loop measurements')
    ap.add_argument('--no-adaptive', action='store_true', help='skip the adaptive-split sigma^2*time measurement')
    ap.add_argument('--no-second-calc', action='store_true', help='skip the MRG32k3a (Calc 1) measurement')
    ap.add_argument('--copy-probe', type=int, default=0, metavar='BYTES',
                    help='only copy BYTES between two device buffers (calibrates HBM byte counters) and exit')
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) != 1:
        print('bench.py: this build runs on one GPU only; multi-GPU runs are not part of it '
              '(samples shard by Philox counter range across GPUs)', file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        x = torch.empty(args.copy_probe // 8, dtype=torch.float64, device='cuda').fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
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
    rec = counters_record()
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
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                     "traffic": (None if rec is None else
                                 (rec['fetch_bytes_per_sample'] + rec['write_bytes_per_sample']) * B),
                     "kernel": "k_integrate<3>", "kernel_ms": prof['ms_fp64'],
                     "kernel_launches": prof['launches'],
                     # a step's 10 launches overlap on 4 streams: the duration of one
                     # launch is the FP64 phase's span (HIP events) over its launches
                     "launch_ms_effective": prof['ms_fp64'] / max(prof['launches'], 1),
                     "flops_per_sample": {str(g): flops[g] for g in range(G)}},
        "traffic_unit": "HBM bytes per FP64-pass launch (one graph, batch_per_graph samples), calibrated "
                        "FETCH_SIZE + WRITE_SIZE scaled from the committed counter runs of this library build",
        "executed_fp64_tflops": (None if rec is None else
                                 rec['executed_fp64_flops_per_sample'] * samples / (prof['ms_fp64'] * 1e-3) / 1e12),
        "phase_ms": {"fp64": prof['ms_fp64'], "dd": prof['ms_dd'], "reduce": prof['ms_reduce']},
        "estimate_3loop_so_far": {"mean": est['mean'], "sigma": est['sigma'], "n": est['n'],
                                  "n_flag": est['n_flag'], "n_dd_fail": est['n_dd_fail'], "n_ood": est['n_ood']},
        "flag_rate": est['n_flag'] / max(est['n'], 1),
    }
    # the same steps as captured HIP-graph replays (one capture, `steps` replays)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.integrate_batches(seed=0, n_per_graph=B, n_batches=args.steps, counter0=counter, accumulate=1,
                          accept_tau=tau)
    torch.cuda.synchronize()
    out["graph_replay_samples_per_s"] = args.steps * B * G / (time.perf_counter() - t0)
    _progress('timed steps and graph replays done')
    if not args.no_learned:
        out["learned_vs_plain"] = learned_vs_plain(ctx, tau, B)
        _progress('learned sampler done')
    if not args.no_adaptive:
        out["adaptive_vs_equal"] = adaptive_vs_equal(ctx, tau, B)
        out["adaptive_vs_equal_measured_cost"] = adaptive_vs_equal(ctx, tau, B, cost=measured_costs(ctx, tau, B // 4))
        _progress('adaptive split done')
    if not args.no_second_calc:
        out["second_calculation"] = second_calculation(ctx, B)
        _progress('second calculation done')
    if not args.no_other_orders:
        out["other_loop_orders"] = other_loop_orders(ctx, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()

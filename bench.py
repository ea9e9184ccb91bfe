"""Benchmark: Monte Carlo throughput of the forest-subtracted AMM integrands.

Headline workload: the largest configuration this library runs end to end on
one GPU, all 74 four-loop self-energy graphs without lepton loops (518
vertex graphs, 11 Feynman parameters), plain combinatorial density (Calc 2
constants), FP64 with the round-off check of eq. (interval_accept) and
double-double recompute of flagged points, one persistent fused launch per
group with the autotuned launch configuration, Philox seed 0.  One step
evaluates `--batch` consecutive sample counters of every graph (the full
configuration is 1e10 samples in all).  At 5 loops (706 graphs) the density
tables and sampling of every graph run on the GPU, but the integrand tables
take minutes per graph to build, so the bench measures graph 0 alone there.  Inputs are generated on the device from the counters, so
nothing is copied from the host inside the timed region.

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


def _oracle_chunk(job):
    """One worker of the CPU baseline: the oracle's FP64 estimate over a
    counter range of one graph (the oracle as it stands)."""
    loops, gi, start, count, cache = job
    import time as _t
    from oracle import estimate as E
    from oracle import integrand as I
    if cache:
        I.load_poly_cache(cache)
    t0 = _t.perf_counter()
    E.run(loops, gi, 0, start, count, chunk=count)
    return _t.perf_counter() - t0


def cpu_baseline(seconds_target=15.0):
    """Time the oracle (numpy FP64, as it stands) on the host's cores: 4-loop
    SE graph 0 (the headline workload's first graph), with its numerator
    polynomials loaded from the oracle's own committed cache, one process per
    core over disjoint counter ranges of seed 0."""
    import multiprocessing as mp
    cache = os.path.join(ROOT, 'tests', 'golden', 'oracle_level_polys_4loop_g0.json.gz')
    if not os.path.exists(cache):
        return None
    cores = max(1, min(16, os.cpu_count() or 1))
    probe = 64
    with mp.get_context('spawn').Pool(cores) as pool:
        pool.map(_oracle_chunk, [(4, 0, 10 ** 6 + 1000 * k, 8, cache) for k in range(cores)])   # load caches
        dt1 = max(pool.map(_oracle_chunk, [(4, 0, 1000 * k, probe, cache) for k in range(cores)]))
        n = max(probe, int(probe * seconds_target / max(dt1, 1e-3)))
        for _ in range(3):
            # the probe's time per point is inflated by per-call costs that
            # larger chunks amortise: resize from the timed run while it comes
            # out far too short
            t0 = time.perf_counter()
            pool.map(_oracle_chunk, [(4, 0, 2 * 10 ** 6 + n * k, n, cache) for k in range(cores)])
            dt = time.perf_counter() - t0
            if dt >= 0.5 * seconds_target:
                break
            n = int(n * seconds_target / max(dt, 1e-3))
    cpu = platform.processor() or platform.machine()
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                cpu = line.split(':', 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n * cores / dt, "unit": "integrand evals/s (4-loop SE-graph samples, 7 insertions each)",
            "cores": cores, "kind": "oracle",
            "sample": f"4-loop SE graph 0, {cores} processes x {n} consecutive counters of seed 0 (disjoint ranges), "
                      f"numpy FP64 oracle ({cpu}); numerator polynomials from the oracle's committed cache, "
                      f"their derivation (hours) excluded",
            "seconds": dt}


def counters_record(name='k_integrate_3loop_counters.json'):
    """HBM bytes and executed FP64 flops per sample of an FP64 pass, from the
    committed rocprofv3 counter runs, if they were taken on this very library
    build (same sha256); else None."""
    import hashlib
    rec_path = os.path.join(ROOT, 'profiles', name)
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


def three_loop_set(ctx, args):
    """The 3-loop set (10 graphs, generated straight-line integrand code, one
    launch per graph on four side streams): samples/s, FP64 fraction of peak
    and the learned-sampler, adaptive-split and second-calculation
    measurements on it."""
    import torch
    ctx.enumerate(3)
    ctx.build_tables()
    G = ctx.n_se
    flops = [ctx.plan_stats(g)['flops_per_sample'] for g in range(G)]
    B = 3_276_800
    ctx.integrate(seed=1, n_per_graph=100_000, force_flag=1)
    tau = ctx.accept_thresholds(1_000_000_000)
    ctx.integrate(seed=0, n_per_graph=B, accept_tau=tau)                      # warm
    ctx.profile(True)
    dt = _timed(torch, lambda: [ctx.integrate(seed=0, n_per_graph=B, counter0=(k + 1) * B, accumulate=k > 0,
                                              accept_tau=tau) for k in range(3)])
    prof = ctx.profile(False)
    achieved = sum(flops) * 3 * B / (prof['ms_fp64'] * 1e-3)
    est = ctx.read(-1, -1, None)
    rec = counters_record()
    out = {"graphs": G, "samples_per_graph_per_step": B, "samples_per_s": 3 * B * G / dt,
           "ms_per_step": dt / 3 * 1e3, "fp64_pass_ms_per_step": prof['ms_fp64'] / 3,
           "dd_ms_per_step": prof['ms_dd'] / 3,
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "kernel": "k_integrate<3> (generated)",
                        "launch_ms_effective": prof['ms_fp64'] / max(prof['launches'], 1),
                        "traffic": (None if rec is None else
                                    (rec['fetch_bytes_per_sample'] + rec['write_bytes_per_sample']) * B)},
           "executed_fp64_tflops": (None if rec is None else
                                    rec['executed_fp64_flops_per_sample'] * 3 * B * G / (prof['ms_fp64'] * 1e-3) / 1e12),
           "flag_rate": est['n_flag'] / max(est['n'], 1), "estimate": {"mean": est['mean'], "sigma": est['sigma']},
           "evaluator": "generated"}
    _progress('3-loop set done')
    if not args.no_learned:
        out["learned_vs_plain"] = learned_vs_plain(ctx, tau, B)
        _progress('learned sampler (3 loops) done')
    if not args.no_adaptive:
        out["adaptive_vs_equal"] = adaptive_vs_equal(ctx, tau, B)
        out["adaptive_vs_equal_measured_cost"] = adaptive_vs_equal(ctx, tau, B, cost=measured_costs(ctx, tau, B // 4))
        _progress('adaptive split done')
    if not args.no_second_calc:
        out["second_calculation"] = second_calculation(ctx, B)
        _progress('second calculation done')
    return out


def low_loop_orders(ctx):
    """Samples/s and FP64 fraction of peak at 1 and 2 loops (generated code)."""
    import torch
    out = {}
    for n, per_graph in ((1, 1 << 24), (2, 1 << 23)):
        ctx.enumerate(n)
        ctx.build_tables()
        G = ctx.n_se
        flops = sum(ctx.plan_stats(g)['flops_per_sample'] for g in range(G))
        tau = None
        if n > 1:
            ctx.integrate(seed=1, n_per_graph=100_000, force_flag=1)
            tau = ctx.accept_thresholds(10 ** 7)
        ctx.integrate(seed=0, n_per_graph=per_graph // 4, accept_tau=tau)               # warm
        ctx.profile(True)
        dt = _timed(torch, lambda: ctx.integrate(seed=0, n_per_graph=per_graph, accept_tau=tau))
        prof = ctx.profile(False)
        achieved = flops * per_graph / (prof['ms_fp64'] * 1e-3)
        out[str(n)] = {"graphs": G, "samples_per_graph": per_graph, "samples_per_s": G * per_graph / dt,
                       "fp64_frac_of_peak": achieved / PEAK_FP64_VALU, "evaluator": "generated"}
    _progress('1- and 2-loop sets done')
    return out


def five_loop(ctx):
    """The 5-loop set (706 graphs, M = 14): density tables and sampling of
    every graph; then the integrand tables of graph 0 (2.8 million monomials,
    built on the host's threads) and its FP64 pass with the round-off check,
    double-double recompute and per-class accumulation."""
    import torch
    from paper_1909_08015_amd.amm import OPT_PLANS
    ctx.enumerate(5)
    ctx.set_option(OPT_PLANS, 0)
    try:
        t_build = _timed(torch, lambda: ctx.build_tables())
        n = 1 << 16
        ctx.sample(0, 0, 0, n)
        dt = _timed(torch, lambda: [ctx.sample(g, 0, 0, n) for g in range(ctx.n_se)])
    finally:
        ctx.set_option(OPT_PLANS, 1)
    out = {"graphs": ctx.n_se, "samples_per_graph": n, "sampling_samples_per_s": ctx.n_se * n / dt,
           "density_tables_build_s": t_build}
    _progress('5-loop sampling done')
    t_plan = _timed(torch, lambda: ctx.build_tables(0, 1))
    st = ctx.plan_stats(0)
    ctx.integrate(seed=1, n_per_graph=4096, graph_begin=0, graph_end=1, force_flag=1)
    tau = ctx.accept_thresholds(10 ** 11 // ctx.n_se, 0, 1)
    N = 1 << 20                                # 1024 chunks: four 64-thread blocks per compute unit
    ctx.integrate(seed=0, n_per_graph=N // 16, graph_begin=0, graph_end=1, accept_tau=tau)       # warm
    ctx.profile(True)
    dt = _timed(torch, lambda: ctx.integrate(seed=0, n_per_graph=N, graph_begin=0, graph_end=1, accept_tau=tau))
    prof = ctx.profile(False)
    est = ctx.read(0, -1)
    _, cls = ctx.graph_desc(0)
    achieved = st['flops_per_sample'] * N / (prof['ms_fp64'] * 1e-3)
    out["graph0"] = {"monomials_per_sample": st['n_monomials'], "flops_per_sample": st['flops_per_sample'],
                     "tables_build_s": t_plan, "samples": N, "samples_per_s": N / dt,
                     "fp64_pass_ms": prof['ms_fp64'], "dd_ms": prof['ms_dd'],
                     "fp64_tflops": achieved / 1e12, "fp64_frac_of_peak": achieved / PEAK_FP64_VALU,
                     "mean": est['mean'], "sigma": est['sigma'], "flag_rate": est['n_flag'] / max(est['n'], 1),
                     "classes": sorted(set(cls)), "evaluator": "interpreter, fused persistent launch"}
    _progress('5-loop graph 0 integrands done')
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=5)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--batch', type=int, default=65_536,
                    help='sample counters per graph per step (74 x 65536 samples, one group of 4736 chunks)')
    ap.add_argument('--pilot', type=int, default=20_000, help='double-double pilot samples per graph')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-learned', action='store_true', help='skip the learned-sampler sigma^2*time measurements')
    ap.add_argument('--no-other-orders', action='store_true', help='skip the 1-, 2-, 3- and 5-loop measurements')
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
    ctx.enumerate(4)
    t_build = _timed(torch, lambda: ctx.build_tables())
    G = ctx.n_se
    flops = [ctx.plan_stats(g)['flops_per_sample'] for g in range(G)]
    stream = torch.cuda.current_stream()
    B = args.batch
    # pilot (every point in double-double, seed 1) -> round-off acceptance
    # thresholds of eq. (interval_accept) for the full 1e10-sample run
    ctx.integrate(seed=1, n_per_graph=args.pilot, force_flag=1)
    tau = ctx.accept_thresholds(10 ** 10 // G)
    tune = ctx.autotune(seed=9, n_per_graph=max(B // 2, 1024), accept_tau=tau)
    _progress(f'4-loop tables ({t_build:.1f} s), pilot and autotune done')
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
    rec = counters_record('k_integrate_fused_4loop_counters.json')
    out = {
        "metric": "integrand evals/s + FP64 % of peak; sigma^2*time learned vs plain sampler, 5-loop",
        "value": value,
        "unit": "integrand evals/s (4-loop SE-graph samples, 7 vertex-graph insertions each)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4-loop set: all 74 four-loop no-lepton-loop SE graphs (518 vertex graphs), 11 "
                               "Feynman parameters, plain combinatorial density (Calc 2), FP64 with round-off check "
                               "and double-double recompute, fused persistent launch, autotuned launch "
                               f"configuration, Philox seed 0; one step = {B} sample counters per graph",
                   "graphs": G, "loops": 4, "batch_per_graph": B, "counters_done": counter},
        "vertex_graph_evals_per_s": value * 7,
        "fp64_frac_of_peak": achieved / PEAK_FP64_VALU,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                     "traffic": (None if rec is None else
                                 (rec['fetch_bytes_per_sample'] + rec['write_bytes_per_sample']) * B * G),
                     "kernel": "k_integrate_fused<4>", "kernel_ms": prof['ms_fp64'],
                     "kernel_launches": prof['launches'],
                     "launch_ms": prof['ms_fp64'] / args.steps,
                     "flops_per_sample": {str(g): flops[g] for g in range(G)}},
        "traffic_unit": "HBM bytes per fused launch (74 graphs x batch_per_graph samples), calibrated "
                        "FETCH_SIZE + WRITE_SIZE scaled from the committed counter runs of this library build",
        "executed_fp64_tflops": (None if rec is None else
                                 rec['executed_fp64_flops_per_sample'] * samples / (prof['ms_fp64'] * 1e-3) / 1e12),
        "phase_ms": {"fp64": prof['ms_fp64'], "dd": prof['ms_dd'], "reduce": prof['ms_reduce']},
        "estimate_4loop_so_far": {"mean": est['mean'], "sigma": est['sigma'], "n": est['n'],
                                  "n_flag": est['n_flag'], "n_dd_fail": est['n_dd_fail'], "n_ood": est['n_ood']},
        "flag_rate": est['n_flag'] / max(est['n'], 1),
        "autotune": tune, "tables_build_s": t_build,
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
        # learned sampler on the 4-loop set: pilot (seed 1) -> GPU training ->
        # sigma^2 * time of the learned mixture against the plain density
        t_pilot = _timed(torch, lambda: ctx.pilot(1, 50_000))
        t_train = _timed(torch, lambda: ctx.mlp_train(200, lr=1e-2, init_seed=0))
        res = {}
        n4 = 1 << 17
        for name, smp in (('plain', 0), ('learned', 1)):
            t = _timed(torch, lambda: ctx.integrate(seed=2, n_per_graph=n4, sampler=smp, accept_tau=tau))
            res[name] = (sum(ctx.read(g, -1)['sigma'] ** 2 for g in range(G)), t, ctx.read(-1, -1, None))
        (vp, tp, ep), (vl, tl, el) = res['plain'], res['learned']
        out["learned_vs_plain_4loop"] = {
            "sigma2_time_ratio_learned_over_plain": (vl * tl) / (vp * tp), "var_plain": vp, "var_learned": vl,
            "s_plain": tp, "s_learned": tl, "mean_plain": ep['mean'], "sigma_plain": ep['sigma'],
            "mean_learned": el['mean'], "sigma_learned": el['sigma'], "pilot_samples_per_graph": 50_000,
            "pilot_s": t_pilot, "train_epochs": 200, "train_s": t_train, "samples_per_graph": n4, "seed": 2,
            "note": "heavy-tailed 4-loop integrands: one run's sigma^2 moves by large factors"}
        _progress('learned sampler (4 loops) done')
    if not args.no_other_orders:
        out["three_loop_set"] = three_loop_set(ctx, args)
        out["other_loop_orders"] = low_loop_orders(ctx)
        out["five_loop"] = five_loop(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()

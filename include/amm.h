/*
 * amm.h -- C ABI of the MI355X (gfx950) Monte Carlo library for the
 * forest-subtracted anomalous-magnetic-moment (AMM) integrands of QED graphs
 * without lepton loops (S. Volkov, arXiv:1909.08015).
 *
 * Conventions shared by every entry point
 *   - Return value: 0 on success, a negative AMM_E_* code on failure; the
 *     message of the last failure on the calling thread is amm_last_error().
 *     No C++ exception crosses this boundary.
 *   - Pointers documented as "device" must point to device memory of the
 *     context's device (e.g. a torch tensor's data_ptr()); "host" pointers are
 *     ordinary host memory.  The caller owns every pointer it passes; the
 *     context owns what it allocates and frees it in amm_destroy.
 *   - A stream argument is a hipStream_t passed as void* (NULL = default
 *     stream).  Calls that take a stream enqueue work and return; the results
 *     are valid after the stream is synchronised (amm_read synchronises).
 *   - Parameter numbering of an n-loop SE graph (M = 3n-1 parameters):
 *     electron segments 0..2n-2 along the line, then the n photons in the
 *     order of the graph's sorted chord list.  The insertion e of the external
 *     photon into segment e merges the two lines next to it into parameter e
 *     (Sec. III.A, footnote on the 3n -> 3n-1 reduction).
 *   - Graph ids: SE graphs of one loop order in lexicographic order of their
 *     sorted chord lists.
 */
#ifndef AMM_H
#define AMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMM_OK            0
#define AMM_E_ARG        -1   /* bad argument or call order                 */
#define AMM_E_NOTBUILT   -2   /* tables not built yet                       */
#define AMM_E_HIP        -3   /* a HIP runtime call failed                  */
#define AMM_E_NOMEM      -4   /* allocation failed                          */
#define AMM_E_NUMERIC    -5   /* a numeric invariant failed on the host     */
#define AMM_E_TOOBIG     -6   /* size beyond the library's stated maximum   */

typedef struct amm_ctx amm_ctx;

/* Density constants.  Sec. III.A eq. (mc_settings): the six Deg(s)
 * constants; Sec. V: mixture weights c[0..3] = C1..C4 and D (Calc 2:
 * C2 = 0.03, C3 = 0.01, C4 = 0.06; Calc 1, run with AMM_OPT_GENERATOR = 1:
 * C2 = 0.03, C3 = 0.035, C4 = 0.035; both D = 0.75, C1 = 1 - C2 - C3 - C4).
 * degmax caps the sector exponents of the first component:
 *   Deg1(s) = max(cbigz, min(cbigf w(s), degmax))   (degmax <= 0: no cap),
 * w(s) = n_photons(s) + n_electrons(s)/2 - 2 loops(s).  Near the face where
 * the lines of s vanish the density scales like rho^(Deg(s) - |s|) and the
 * subtracted integrand like rho^(w_f(s) - |s|) with w_f(s) >= 1, so f/g has
 * finite variance only if Deg(s) < 2 w_f(s); the default 1.0 keeps f/g
 * bounded at every face. */
typedef struct {
    double cbigz, cbigf, cadd, csubi, csubse, csubo;
    double c[4];
    double d;
    double degmax;
} amm_density_params;

/* One Monte Carlo run over a range of graphs (Sec. III.B, eq.
 * integral_approx).  Samples counter0 .. counter0+n_per_graph-1 of every graph
 * in [graph_begin, graph_end) are evaluated.
 *   sampler:     0 plain density g; 1 learned mixture q = (q_theta + g)/2
 *                (falls back to plain if no trained table exists).
 *   accept_tau:  per-graph round-off acceptance threshold of eq.
 *                (interval_accept) as a host array of length graph_end -
 *                graph_begin, or NULL for no flagging.
 *   force_flag:  1 = recompute every point in double-double.
 *   blocks_per_cu: resident blocks per compute unit of the FP64 pass (grid =
 *                blocks_per_cu x CUs); 0 = the context's value (amm_autotune,
 *                default 8).  Results do not depend on it.
 *   accumulate:  0 = reset the accumulators of these graphs first. */
typedef struct {
    uint64_t seed;
    uint64_t counter0;
    uint64_t n_per_graph;
    int graph_begin, graph_end;
    int sampler;
    int force_flag;
    int blocks_per_cu;
    int accumulate;
    const double *accept_tau;
} amm_run_params;

/* Accumulators of one insertion (vertex graph) or one class. */
typedef struct {
    double mean, sigma;                 /* eq. (integral_approx), eq. (sigma_down) */
    double sum_y, sum_y2, sum_abs;
    uint64_t n, n_flag, n_dd_fail, n_ood;
} amm_estimate;

/* Static cost of evaluating one sample of an SE graph. */
typedef struct {
    int n_insertions;
    int n_terms;            /* forest terms (L-U merged) over all insertions */
    int n_terms_expanded;   /* with (L-U) split in two, Sec. II counting     */
    int n_level_evals;      /* level evaluations per sample                  */
    int64_t n_monomials;    /* numerator monomials evaluated per sample      */
    double flops_per_sample;/* algorithmic FP64 flops per sample (values only: a monomial of nv variables counts nv + 1; FMA = 2), excluding the sampler and the error bound */
} amm_plan_info;

/* Create a context on HIP device `device`. */
int amm_create(amm_ctx **out, int device);
/* Free everything the context allocated. */
void amm_destroy(amm_ctx *ctx);
/* Message of the last error on this thread ("" if none). */
const char *amm_last_error(void);

/* Enumerate the n-loop SE graphs without lepton loops (1 <= loops <= 5):
 * counts per Sec. I (3213 vertex graphs at 5 loops modulo reversal). Outputs
 * may be NULL. n_vertex counts oriented vertex graphs (SE graph x insertion). */
int amm_enumerate(amm_ctx *ctx, int loops, int *n_se, int *n_vertex, int *M);

/* Chords (2*loops ints, pairs of vertex positions 0..2n-1) and the class
 * (k, m, m') of each insertion ((2n-1)*3 ints; Sec. V definition before
 * Table I) of SE graph g.  Host pointers; either may be NULL. */
int amm_graph_desc(const amm_ctx *ctx, int g, int *chords, int *classes);

/* Build the per-graph density tables (Sec. III.A) and subtraction tables
 * (Sec. II forest formula) for graphs [graph_begin, graph_end) of the
 * enumerated loop order and upload them once.  params NULL = Calc 2.
 * At 5 loops the integrand tables hold about 3 million monomials per graph
 * (70 MB each for the double-double table and the FP64 group stream) and take
 * minutes per graph to build (a thread pool); AMM_OPT_PLANS = 0: density only. */
int amm_build_tables(amm_ctx *ctx, const amm_density_params *params,
                     int graph_begin, int graph_end);

/* Static plan statistics of graph g (after amm_build_tables). */
int amm_plan_stats(const amm_ctx *ctx, int g, amm_plan_info *out);

/* Sample n points of graph g: sample indices counter0..counter0+n-1; learned
 * = 1 draws from the learned mixture (needs a sector table; component 4 =
 * q_theta).
 * Device outputs (any may be NULL): z [n x M] doubles, gx [n] mantissa and
 * gj [n] int32 exponent of g = gx 2^gj (Sec. IV.A), path [n x M] int32 line
 * order z_{path0} >= z_{path1} >= ..., comp [n] int32 mixture component. */
int amm_sample(amm_ctx *ctx, int g, uint64_t seed, uint64_t counter0, uint64_t n,
               int learned, double *z, double *gx, int32_t *gj, int32_t *path, int32_t *comp,
               void *stream);

/* Evaluate the integrands of all 2n-1 insertions of graph g at n device
 * points z [n x M]: I [n x (2n-1)], the sum of |term| per insertion
 * absI [n x (2n-1)] and a bound [n x (2n-1)] (any output may be NULL).
 * precision: 0 = FP64, bound = the running round-off bound of I (Sec. IV.A,
 * eq. interval_accept); 1 = double-double (value rounded to double);
 * 2 = FP64 interval arithmetic with outward rounding (the first interval rung
 * of Sec. IV.A; table interpreter): I and absI are interval midpoints and
 * bound the radius, |exact I - I| <= bound, barring overflow and underflow.
 * Errors: AMM_E_ARG (bad graph or precision, z NULL), AMM_E_NOTBUILT. */
int amm_eval(amm_ctx *ctx, int g, const double *z, uint64_t n,
             double *I, double *absI, double *bound, int precision, void *stream);

/* Run the Monte Carlo (sample, evaluate, round-off check, double-double
 * recompute of flagged points, accumulate) asynchronously on `stream`
 * (Sec. III.B, eq. integral_approx; Sec. IV.A).  The per-graph launches of a
 * group run on the context's internal streams, forked from `stream` and
 * joined back to it with events, so all work of the call is ordered before
 * later work on `stream`.  A context is not to be used by several host
 * threads at once.  Errors: AMM_E_ARG (bad range or parameters, sample
 * indices out of range), AMM_E_NOTBUILT, AMM_E_HIP. */
int amm_integrate(amm_ctx *ctx, const amm_run_params *run, void *stream);

/* The same run repeated n_batches times as consecutive counter ranges:
 * batch b evaluates counters counter0 + b*n_per_graph .. + n_per_graph - 1 of
 * every graph (b = 0 .. n_batches-1), accumulating (accumulate = 0 resets the
 * accumulators once, before batch 0).  The kernels of one batch (FP64 pass,
 * double-double recompute, reductions, advance of a device-resident counter
 * base) are captured once into a HIP graph and replayed; results equal those
 * of n_batches amm_integrate calls over the same counters.  Synchronises
 * `stream` (the graph runs on an internal stream ordered after it).
 * Errors: AMM_E_ARG, AMM_E_NOTBUILT, AMM_E_HIP. */
int amm_integrate_batches(amm_ctx *ctx, const amm_run_params *run, uint64_t n_batches, void *stream);

/* Caller-owned device workspace for the Monte Carlo runs (amm_integrate,
 * amm_integrate_batches, amm_integrate_adaptive, amm_autotune), so that a
 * framework's allocator (e.g. PyTorch) can supply the device memory: the
 * per-group chunk partial sums, flag words and double-double results.
 * dev_ptr: device memory of the context's device, 256-byte aligned, of
 * `bytes` bytes, owned by the caller, never freed by the context, and not to
 * be used by the caller while runs of the context are pending.  The group size
 * becomes the largest chunk count c (1024 samples each, c <= 32768) with
 * amm_workspace_bytes(c) <= bytes; results do not depend on it beyond the
 * order in which segment sums are added.  The context frees its own group
 * buffers; dev_ptr NULL returns to them (allocated again on the next run).
 * Waits for the context's last run.  Errors: AMM_E_ARG (misaligned, or
 * smaller than amm_workspace_bytes(1)), AMM_E_HIP. */
int amm_set_workspace(amm_ctx *ctx, void *dev_ptr, size_t bytes);
/* Bytes of a workspace for groups of chunks_per_group chunks (1 .. 32768;
 * any loop order), 0 for a count out of range. */
size_t amm_workspace_bytes(int chunks_per_group);

/* Options (value semantics per option):
 * AMM_OPT_GENERATED (default 1): evaluate integrands with the straight-line
 *   code generated at build time for the graph when it exists (1-3 loops),
 *   else (0, or no generated code) with the table interpreter.  Both compute
 *   the same levels and polynomials; results agree to rounding.
 * AMM_OPT_FUSED (default 1): a group whose graphs all use the interpreter
 *   runs its FP64 pass as one persistent launch (blocks take chunks from a
 *   work counter) instead of one launch per graph.
 * AMM_OPT_ORDER_BY_COST (default 1): order the graphs of a group by plan cost,
 *   heaviest first (0: graph order).
 * AMM_OPT_BLOCKS_PER_CU (default 0 = 8): blocks per compute unit of the FP64
 *   pass when a run does not set its own.
 * None of them changes results: sums are keyed by 1024-sample chunk.
 * AMM_OPT_GENERATOR (default 0): pseudorandom generator of amm_sample and of
 *   the amm_integrate* runs, 0 = Philox4x32-10 (the paper's Calc 2), 1 =
 *   MRG32k3a (Calc 1, Sec. V).  MRG32k3a streams: graph uid starts uid 2^100
 *   steps after a start state taken from the seed's 32-bit halves (lo, hi) as
 *   ((1 + lo mod (m1 - 1), 12345, 12345), (1 + hi mod (m2 - 1), 12345, 12345));
 *   sample i starts i 2^7 steps after its graph's start, and its uniform k is
 *   ((za >> 1) 2^21 + (zb >> 11) + 1/2) 2^-52 from outputs 2k+1, 2k+2.
 *   Sample indices must stay below 2^44 (AMM_E_ARG otherwise).  This option
 *   changes the samples, hence the results; the pilot of the learned sampler
 *   (amm_pilot) always uses Philox4x32-10.
 * AMM_OPT_PLANS (default 1): amm_build_tables builds the integrand tables as
 *   well as the density tables; 0 builds the density tables only (sampling
 *   with amm_sample, e.g. for all 706 graphs at 5 loops); amm_eval,
 *   amm_integrate* and amm_pilot then return AMM_E_NOTBUILT. */
#define AMM_OPT_GENERATED 1
#define AMM_OPT_FUSED 2
#define AMM_OPT_ORDER_BY_COST 3
#define AMM_OPT_BLOCKS_PER_CU 4
#define AMM_OPT_GENERATOR 5
#define AMM_OPT_PLANS 6
int amm_set_option(amm_ctx *ctx, int option, int value);

/* Launch-configuration autotuner: times the run `run` (its n_per_graph is the
 * probe size; a warm-up and a timed call per candidate) for blocks per CU in
 * {1, 2, 4, 8, 16} and both graph orders, keeps the fastest in the context
 * (AMM_OPT_BLOCKS_PER_CU, AMM_OPT_ORDER_BY_COST) and reports it (host
 * outputs, may be NULL; ms_best = milliseconds of the best probe).  The
 * accumulators are restored afterwards.  Synchronises `stream`. */
int amm_autotune(amm_ctx *ctx, const amm_run_params *run, int *blocks_per_cu, int *order_by_cost,
                 double *ms_best, void *stream);

/* Sample split of one adaptive round over n graphs, Sec. IV.C (eq. for p_j):
 * graph j receives samples in proportion to C_j / sqrt(t_j), C_j = sigma_j
 * sqrt(N_j) being its per-sample standard deviation and t_j its cost per
 * sample; this minimises sum_j C_j^2 / n_j (eq. sigma_sum) at the cost
 * sum_j n_j t_j = budget.  A share floor_frac of the budget is split equally
 * (stabilisation for graphs whose C_j is underestimated):
 *   w_j = C_j / sqrt(t_j),
 *   n_j = floor(floor_frac budget / sum_l t_l
 *               + (1 - floor_frac) budget w_j / sum_l w_l t_l),
 * evaluated in that order in FP64; if every C_j is 0 the split is equal.
 * Inputs are host arrays of n doubles (C_j >= 0, t_j > 0, finite), budget
 * >= 0 in the units of t, floor_frac in [0, 1]; n_out is a host array of n.
 * Host code only: needs no device.  Errors: AMM_E_ARG. */
int amm_adaptive_split(int n, const double *C, const double *t, double budget, double floor_frac,
                       uint64_t *n_out);

/* Adaptive distribution of samples over the graphs [graph_begin, graph_end)
 * of `run`, Sec. IV.C.  Round 0 draws run->n_per_graph samples of every graph
 * (counters from run->counter0; run->accumulate as in amm_integrate); each of
 * the n_rounds - 1 later rounds takes an equal part of the budget left and
 * splits it with amm_adaptive_split, C_j read from the accumulators so far.
 * Graph j's samples are the consecutive counters counter0 .. counter0 +
 * n_done[j] - 1 of its stream, so the result is that of amm_integrate calls
 * over those ranges, and the run is deterministic.  The budget is the cost of
 * budget_per_graph samples of every graph: sum_j n_done[j] t_j <=
 * budget_per_graph sum_j t_j.  cost: host array of t_j (NULL = the plan's
 * flops per sample, amm_plan_stats).  accept_tau applies unchanged in every
 * round.  n_done: host output (may be NULL), samples per graph.  Reads the
 * accumulators between rounds (synchronises `stream`); the last round is
 * left enqueued.  Errors: AMM_E_ARG (budget_per_graph < n_per_graph,
 * n_rounds < 1, floor_frac outside [0, 1], cost <= 0), AMM_E_NOTBUILT,
 * AMM_E_HIP. */
int amm_integrate_adaptive(amm_ctx *ctx, const amm_run_params *run, uint64_t budget_per_graph, int n_rounds,
                           double floor_frac, const double *cost, uint64_t *n_done, void *stream);

/* Graph-by-graph combination of two independent calculations (Sec. V: the
 * MRG32k3a and the Philox4x32-10 runs), then the sum over graphs with eq.
 * sigma_sum.  Per graph j the inverse-variance weighted mean
 *   w_k = 1 / sigma_k^2,  mean = (mean1 w1 + mean2 w2) / (w1 + w2),
 *   sigma = sqrt(1 / (w1 + w2)),
 * evaluated in that order in FP64; a calculation with sigma 0 takes all the
 * weight (both 0: the plain average, sigma 0).  Totals: sum of the means,
 * sqrt of the sum of sigma^2, in graph order.  Inputs: host arrays of n
 * doubles (sigmas >= 0).  Outputs: host arrays of n (mean, sigma) and host
 * scalars, each may be NULL.  Host code only.  Errors: AMM_E_ARG. */
int amm_combine(int n, const double *mean1, const double *sigma1, const double *mean2, const double *sigma2,
                double *mean, double *sigma, double *total_mean, double *total_sigma);

/* Round-off acceptance thresholds of eq. (interval_accept), Sec. IV.A (a
 * point of graph j is accepted when the round-off bounds of its 2n-1
 * insertion values, divided by g and added, do not exceed tau_j):
 * tau_j = (1/4) sigma_j sqrt(sum_l sigma_l^2) / sum_l sigma_l over the graphs
 * [graph_begin, graph_end), where sigma_j is the current accumulators'
 * sigma of graph j (all insertions summed; a pilot run) scaled to a run of
 * n_run samples: sigma_j sqrt(N_pilot / n_run).  Writes graph_end -
 * graph_begin doubles to the host array tau (to pass as accept_tau). */
int amm_accept_thresholds(amm_ctx *ctx, int graph_begin, int graph_end, uint64_t n_run, double *tau);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the run of
 * amm_integrate with every buffer it needs beyond the context's tables and
 * accumulators taken from a static device array of the library (20.4 MB
 * per device, held from the first amm_create on that device until the process
 * ends).  Calls no hipMalloc, hipFree or other allocating routine.  Groups
 * hold 256 chunks (262144 samples); a run may have at most 1024 segments,
 * i.e. sum over its graphs of ceil(n_per_graph / 262144) <= 1024, else
 * AMM_E_TOOBIG.  Results equal amm_integrate's up to the order in which
 * segment sums are added (counters exactly).  Every call on a device shares
 * that device's array: calls that overlap on one device (other contexts, or
 * other streams without ordering) race.  Errors: as amm_integrate, and
 * AMM_E_TOOBIG. */
int amm_integrate_static(amm_ctx *ctx, const amm_run_params *run, void *stream);

/* Read accumulators (synchronises the last stream used).  g >= 0 selects a
 * graph; e >= 0 an insertion of it, e = -1 the sum over its insertions.
 * cls_k >= 0 with g = -1 selects a class (k, m, m') summed over all built
 * graphs (class sigma^2 adds over graphs, eq. sigma_sum); cls_k = -1 with
 * g = -1 gives the total over all built graphs.  The insertions of one graph
 * are evaluated at the same points, so the sigma of a sum over insertions
 * (e = -1, or a class) is that of the per-point sums (eq. sigma_down applied
 * to them), which keeps the insertions' covariance. */
int amm_read(amm_ctx *ctx, int g, int e, int cls_k, int cls_m, int cls_mp,
             amm_estimate *out);

/* Per-phase device timing of amm_integrate with HIP events recorded on the
 * launch stream.  enable = 1 starts recording (and resets the totals),
 * 0 stops.  Outputs (host, may be NULL) are totals since enabling:
 * milliseconds in the FP64 sample+integrand kernel, in the double-double
 * recompute kernel, in the reduction kernel, and the number of FP64 kernel
 * launches and of samples they processed.  Reading synchronises. */
int amm_profile(amm_ctx *ctx, int enable, double *ms_fp64, double *ms_dd, double *ms_reduce,
                int64_t *n_launches, int64_t *n_samples);

/* ----- learned sector sampler (an extension, not in the paper) -----
 * A 3-layer FP32 MLP maps features of (graph, s, j) to a logit correction of
 * the plain sector probabilities; q = (q_theta + g)/2 stays exactly
 * computable so f/q remains unbiased. */

/* Record pilot statistics for graphs [graph_begin, graph_end): samples
 * [0, n_per_graph) of `seed` drawn from the plain density.  Per sample
 * w = sqrt(sum_e y_e^2), y_e = I_e / g (FP64, or double-double where the FP64
 * round-off bound exceeds 1% of w; out-of-double or non-finite points give 0).
 * With wref = mean of w over the first min(n_per_graph, 2^23) samples, the
 * integer q = floor(min(w / wref, 256) * 2^24) is added to W(s, j) for every
 * step (set s, chosen line j) of the sample's sector path; integer sums make
 * W independent of the order of the additions.  Synchronises the stream.
 * Errors: AMM_E_ARG (range, n = 0), AMM_E_NOTBUILT, AMM_E_HIP. */
int amm_pilot(amm_ctx *ctx, uint64_t seed, uint64_t n_per_graph,
              int graph_begin, int graph_end, void *stream);
/* Copy graph g's pilot table W [2^M x M] (row s = bitmask of the remaining
 * lines, column j = chosen line; exact integers as doubles) to host memory of
 * at least cap doubles.  Errors: AMM_E_ARG, AMM_E_NOTBUILT (no pilot yet). */
int amm_pilot_table(const amm_ctx *ctx, int g, double *host, size_t cap);
/* Train the MLP on the pilot table for `epochs` full-batch Adam steps with
 * learning rate lr, then tabulate P_theta(j | s) for every built graph. */
int amm_mlp_train(amm_ctx *ctx, int epochs, float lr, uint64_t init_seed, void *stream);
/* Number of MLP parameters; copy them (FP32) to host buffer (NULL = count only). */
int amm_mlp_params(const amm_ctx *ctx, float *host, size_t cap, size_t *count);
/* The same copy under the boundary's name: n floats of room in host_buf. */
int amm_mlp_get_params(const amm_ctx *ctx, float *host_buf, size_t n);
/* One Adam step of the training (beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
 * bias-corrected with step number t >= 1, FP32) on the context's parameters
 * with a device gradient grad [count floats]; reset_moments = 1 zeroes the
 * first and second moments first.  Enqueued on `stream`.  For checking the
 * update against a reference.  Errors: AMM_E_ARG, AMM_E_NOTBUILT (no
 * parameters yet). */
int amm_mlp_adam(amm_ctx *ctx, const float *grad, int t, float lr, int reset_moments, void *stream);
/* Set MLP parameters from a host buffer of `count` floats. */
int amm_mlp_set_params(amm_ctx *ctx, const float *host, size_t count);
/* Feature rows of graph g: rows [n_rows x 16] (s, j) features, host output;
 * row r corresponds to (s = mask_of_row[r], j = line_of_row[r]). */
int amm_mlp_features(const amm_ctx *ctx, int g, float *rows, int32_t *mask_of_row,
                     int32_t *line_of_row, size_t cap, size_t *n_rows);
/* Loss and gradient of the MLP objective on device rows (for gradient
 * checks): rows [n_rows x 16] features (feature 0 = log of the plain sector
 * probability), w [n_rows] row weights, goff [n_groups+1] offsets of the
 * softmax groups (rows of one set s are contiguous).  Outputs: loss (device,
 * 1 float) and grad (device, count floats).  Uses the current parameters
 * (amm_mlp_set_params).  Synchronises `stream`. */
int amm_mlp_loss_grad(amm_ctx *ctx, const float *rows, const float *w, const int32_t *goff,
                      int n_rows, int n_groups, float *loss, float *grad, void *stream);
/* Install a sector table P(j | s) for graph g from host memory
 * ([2^M x M] floats; row s holds the weights of the lines j in s; they are
 * normalised over j in s when used).  NULL removes the table.  Sampling with
 * the learned mixture (sampler = 1) then uses this table. */
int amm_set_sector_table(amm_ctx *ctx, int g, const float *host_table);

#ifdef __cplusplus
}
#endif
#endif /* AMM_H */

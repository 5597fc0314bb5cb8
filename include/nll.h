/*
 * nll.h -- C ABI of libnllmi: batched unbinned negative log-likelihoods of
 * composed probability densities on AMD Instinct MI355X (gfx950).
 *
 * What is computed (Hageboeck, "A Faster, More Intuitive RooFit",
 * arXiv:2003.12875):
 *   - a computation graph connecting observables, parameters and densities
 *     into a likelihood model fitted to data (Sec. 1);
 *   - the unbinned likelihood, one expression evaluated per dataset entry
 *     (Sec. 5.1), here reduced to NLL(theta) = -sum_i ln p(x_i; theta) over
 *     all events, in one fused streaming pass over structure-of-arrays
 *     event columns (the batched data flow of Sec. 5.2/5.3);
 *   - normalisation of every density over its observable range by closed
 *     forms or numerical quadrature (Sec. 3, "Analytic Integrals"), computed
 *     once per parameter point (Sec. 5.1, node-local caching);
 *   - parameter range checks and the rejection of non-positive or
 *     non-finite probabilities (Sec. 3, "Checking parameters");
 *   - the analytic gradient dNLL/dtheta from the same pass, many datasets
 *     per launch (toy studies, Sec. 1) and on-device gradient-descent fits
 *     in the role of fitTo (Sec. 5.3).
 *
 * Conventions
 *   - All event columns, parameter vectors and outputs are DEVICE pointers
 *     (memory of the model's device).  The caller owns them.  Entry points
 *     marked "enqueue" only enqueue work on the model's stream; results are
 *     valid when that stream reaches them (they never synchronise, so they
 *     can be captured into a HIP graph), and device-detected errors are
 *     reported later by nll_sync() or the per-set status arrays.
 *   - theta always holds all n_param values in declaration order, fixed
 *     ones included; gradients have n_param entries and those of fixed
 *     parameters are written as 0.  Batched theta and gradient arrays are
 *     row-major [set][param].
 *   - A model is used by one host thread at a time; calls on one model are
 *     not reentrant.  Different models are independent.
 *   - Errors: every entry point returns an nll_status; arguments are checked
 *     before anything is enqueued, and on a synchronous error nothing is
 *     enqueued.
 */
#ifndef NLLMI_NLL_H
#define NLLMI_NLL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NLL_MAX_OBS 4
#define NLL_MAX_PARAMS 32
#define NLL_MAX_NODES 16
#define NLL_NODE_MAX_PARAMS 12
#define NLL_NODE_MAX_CHILDREN 8

typedef enum nll_status {
  NLL_OK = 0,
  NLL_ERR_ARG = -1,          /* malformed argument or descriptor            */
  NLL_ERR_UNSUPPORTED = -2,  /* valid graph with no compiled kernel shape    */
  NLL_ERR_PARAM_RANGE = -3,  /* parameter outside its allowed range          */
  NLL_ERR_DOMAIN = -4,       /* event outside the closed observable range    */
  NLL_ERR_INVALID_PDF = -5,  /* some p(x_i) <= 0 or non-finite               */
  NLL_ERR_DEVICE = -6,       /* HIP runtime error                           */
  NLL_ERR_OOM = -7,          /* device allocation failed                    */
  NLL_ERR_STATE = -8,        /* call out of order (e.g. no data attached)    */
  NLL_ERR_SCRATCH = -9       /* request larger than the fixed scratch array  */
} nll_status;

/* Node kinds.  Leaf parameters, in this order:
 *   NLL_GAUSS  (mu, sigma)            g = exp(-((x-mu)/sigma)^2 / 2), sigma > 0
 *   NLL_EXP    (c)                    g = exp(c x)
 *   NLL_CHEB   (a_1 .. a_K), K <= 8   g = 1 + sum_k a_k T_k(x'), x' = (2x-lo-hi)/(hi-lo)
 *   NLL_CB     (m0, sigma, alpha, n)  Crystal Ball, Gaussian core for
 *              t = (x-m0)/sigma > -alpha, power-law tail A (B - t)^-n below,
 *              A = (n/alpha)^n exp(-alpha^2/2), B = n/alpha - alpha;
 *              sigma > 0, alpha > 0, n > 1
 *   NLL_ARGUS  (m0, c)                g = x sqrt(u) exp(c u), u = 1 - (x/m0)^2 for
 *              x < m0, 0 above; m0 > observable lo >= 0
 *   NLL_JOHNSON (mu, lambda, gamma, delta)  Johnson's S_U family (one of the
 *              built-in densities of Sec. 3): g = exp(-u^2/2) / sqrt(1 + z^2),
 *              z = (x-mu)/lambda, u = gamma + delta asinh(z); lambda > 0,
 *              delta > 0; closed-form normalisation through the substitution
 *              u(x), under which the density is a Gaussian in u
 *   NLL_CHI2   (nu)                   chi-square (the "ChiSquarePdf" model of
 *              Sec. 5.2): g = x^(nu/2-1) exp(-x/2), nu > 0; the observable
 *              range must lie in [0, 1000] (else NLL_ERR_UNSUPPORTED);
 *              closed-form normalisation by the lower incomplete gamma
 *              function, Gauss-Legendre after x = s^2 when lo = 0
 *   NLL_HYPATIA (mu, sigma, lambda, zeta, beta, a_l, n_l, a_r, n_r)
 *              Hypatia2 (Sec. 3): with d = x-mu, nu = lambda-1/2,
 *              delta^2 = sigma^2 zeta K_lambda(zeta)/K_{lambda+1}(zeta),
 *              alpha = zeta/delta, r^2 = d^2+delta^2, the core
 *              g = r^nu e^(beta d) K_nu(alpha r) on -a_l sigma <= d <= a_r sigma,
 *              continued below and above by power laws
 *              G (1 + k w)^-n (w: distance from the junction; n = n_l, n_r)
 *              with the core's value and slope; sigma, zeta, a_l, a_r > 0,
 *              n_l, n_r > 1, and both tails falling away from the core
 *              (else NLL_ERR_PARAM).  Normalised numerically whatever
 *              `norm` says (Gauss-Legendre in asinh(d/delta) on the core,
 *              in log(1 + k w) on each tail).  At most one per model, FP64
 *              only (else NLL_ERR_UNSUPPORTED); K_nu is tabulated per
 *              parameter point on the core's range, which takes
 *              |lambda| <= 6 and 1e-3 <= alpha r <= 700 over it
 *   NLL_JIT    (p[0] .. p[n-1]), 1 <= n <= 8: a density given as a formula
 *              string (Sec. 4: PDFs written as expressions and compiled at
 *              run time), `density` below, a C expression in x and p[k]
 *              (double arithmetic; + - * /, exp log sqrt pow sin cos tan
 *              atan tanh sinh cosh asinh erf fabs), p[k] the node's k-th
 *              parameter, k a literal index < n.  Normalised numerically
 *              whatever `norm` says: composite 256-point Gauss-Legendre on
 *              1, 2, 4, ... 256 equal panels of the range until two levels
 *              agree (to 1e-13 of the integral of |g|, 1e-11 of those of
 *              |dg/dp_k|); no agreement, or Z <= 0 or not finite, is an
 *              invalid density (NLL_ERR_INVALID_PDF through nll_sync), as
 *              is an event where g < 0 or is not finite (g = 0 is a term
 *              that contributes nothing).  Gradient by forward-mode dual
 *              numbers in the same pass.  Any graph position, any number
 *              of such leaves; FP64 only (else NLL_ERR_UNSUPPORTED).  A
 *              model with one is compiled at creation (run-time
 *              compilation, as any shape outside the compiled set); the
 *              expression is compiled as given: it must come from a
 *              trusted source, as any code the process runs
 * Composite nodes:
 *   NLL_SUM    over k >= 2 children on the same observables, either
 *              fractions (f_1 .. f_{k-1}): p = sum_{j<k} f_j p_j +
 *              (1 - sum f) p_k, f_j in [0, 1], sum f <= 1; or yields
 *              (nu_1 .. nu_k), as RooAddPdf takes k coefficients for k
 *              densities: p = sum_j nu_j p_j / sum_j nu_j, nu_j >= 0 with a
 *              positive total (an extended model's expected count, below)
 *   NLL_PROD   no params; children on disjoint observables: p = prod p_d   */
enum nll_node_kind {
  NLL_GAUSS = 1, NLL_EXP = 2, NLL_CHEB = 3, NLL_CB = 4, NLL_ARGUS = 5, NLL_SUM = 6, NLL_PROD = 7, NLL_JOHNSON = 8,
  NLL_CHI2 = 9, NLL_HYPATIA = 10, NLL_JIT = 11
};

/* Normalisation of a leaf over its observable range [lo, hi]:
 *   NLL_NORM_ANALYTIC      closed form (Sec. 3 "Analytic Integrals")
 *   NLL_NORM_GL256         256-point Gauss-Legendre per analytic panel: the
 *                          Crystal Ball is split at its core/tail junction,
 *                          the ARGUS endpoint is removed by x = m0 - s^2
 *   NLL_NORM_GL256_SINGLE  256-point Gauss-Legendre on [lo, hi] as one panel */
enum nll_norm_method { NLL_NORM_ANALYTIC = 0, NLL_NORM_GL256 = 1, NLL_NORM_GL256_SINGLE = 2 };

/* Arithmetic of the per-event pass.  NLL_FP64: FP64 everywhere, as the
 * paper's batched computations (Sec. 5.2 and 5.3 keep double precision and
 * quote their agreement with the scalar path).  NLL_FP32C, an option beyond
 * the paper: per-event density
 * arithmetic in FP32 (observables location-subtracted in FP64 first; steps
 * that add per-point constants in FP64), two-sum-compensated FP32 per-thread
 * sums widened to FP64, FP64 normalisation, cross-thread reduction and
 * minimiser.  FP32C results differ from FP64 by unbiased FP32 roundings:
 * about 1e-6/sqrt(N) relative for N events, and within 1e-9 (NLL) and 1e-8
 * (gradient, relative to the sum of |d log p_i / d theta|) at N = 1e8.
 * Parameter points at which a per-event FP32 intermediate overflows (e.g.
 * (x - mu)/sigma beyond ~1e19) give +inf where FP64 would not. */
enum nll_precision { NLL_FP64 = 0, NLL_FP32C = 1 };

typedef struct nll_node_desc {
  int32_t kind;                         /* nll_node_kind                     */
  int32_t obs;                          /* observable index (leaves), else -1 */
  int32_t n_param;
  int32_t param[NLL_NODE_MAX_PARAMS];   /* indices into theta                */
  int32_t n_child;
  int32_t child[NLL_NODE_MAX_CHILDREN]; /* indices of EARLIER nodes          */
  int32_t norm;                         /* nll_norm_method (leaves)          */
  const char* density;                  /* NLL_JIT: the formula (host string,
                                           <= 4096 characters, read during
                                           nll_create_model only); else NULL */
} nll_node_desc;

typedef struct nll_model_desc {
  int32_t n_obs;                  /* 1 .. NLL_MAX_OBS                         */
  const double* obs_lo;           /* host arrays [n_obs]: closed ranges       */
  const double* obs_hi;
  int32_t n_param;                /* 1 .. NLL_MAX_PARAMS                      */
  const double* param_lo;         /* host arrays [n_param]: allowed ranges    */
  const double* param_hi;
  const uint8_t* param_free;      /* host [n_param], 0 = fixed (NULL: all free) */
  int32_t n_node;                 /* 1 .. NLL_MAX_NODES, topological order     */
  const nll_node_desc* nodes;     /* host [n_node]                            */
  int32_t root;                   /* index of the top density                 */
  int32_t precision;              /* nll_precision                            */
  int32_t extended;               /* 1: add nu - N ln nu (Poisson yield term) */
  int32_t yield_param;            /* index of nu when extended, or -1: nu is
                                     the total of the root's sum of yields (the
                                     root itself, or the one sum of yields
                                     among a root product's children), whose
                                     yields then each get 1 - N / nu       */
  int32_t device;                 /* HIP device ordinal                       */
  void* stream;                   /* hipStream_t for all enqueued work (NULL: default) */
} nll_model_desc;

typedef struct nll_model nll_model; /* opaque, owned by the library */

/* Validate the descriptor, lower the graph onto a kernel shape and allocate
 * the model's device scratch.  Descriptor arrays are copied; the caller may
 * free them afterwards.
 * Lowering: the graph becomes a sum of K terms, each a product of leaf
 * densities with one coefficient (the product of the SUM fractions on its
 * path); leaves in every term are factors outside the per-event
 * log-sum-exp.  Any graph within these limits is supported: at most 8
 * leaves, 8 terms, 4 SUM nodes, 4 SUM nodes on the path to a term and 48
 * per-event sums (1 + (K if K > 1) + the leaves' parameters, + K - 1 in
 * NLL_FP32C).  Shapes compiled ahead of time (one leaf; two-term sums of
 * Gauss+Exp, Gauss+Gauss, CB+ARGUS, Johnson+Exp; (CB+ARGUS) x Chebyshev-4;
 * Gauss x Gauss) are ready at once; any other shape is compiled for the
 * model's device at creation from the same kernel templates (hipRTC, the
 * counterpart of the paper's just-in-time compilation, Sec. 4; about
 * 5-15 s, once per shape and device in a process, code objects cached on
 * disk under $NLLMI_RTC_CACHE, default ~/.cache/nllmi, "off" to disable).
 * Errors: NLL_ERR_ARG (malformed graph, bad indices, non-topological
 * order, SUM over different observables, PROD over shared observables,
 * unused observable), NLL_ERR_UNSUPPORTED (beyond the limits above),
 * NLL_ERR_DEVICE (also a failed run-time compilation: the compiler's log
 * goes to stderr), NLL_ERR_OOM. */
nll_status nll_create_model(const nll_model_desc* desc, nll_model** out);

/* Release the model and its device scratch (waits for its stream). */
void nll_destroy_model(nll_model* model);

/* Change the stream used by subsequent enqueue calls. */
nll_status nll_set_stream(nll_model* model, void* stream);

/* Attach n_events events: cols[o] is a device array of n_events doubles for
 * observable o (structure of arrays).  The library borrows the columns until
 * the next nll_set_data or nll_destroy_model.  Makes one validation pass and
 * SYNCHRONISES the stream: NLL_ERR_DOMAIN if any value lies outside its
 * closed observable range or is NaN (the data are then not attached). */
nll_status nll_set_data(nll_model* model, const double* const* cols, int64_t n_events);

/* Attach per-event weights to the attached data (weights: device array of
 * n_events doubles, borrowed until the next nll_set_weights, nll_set_data
 * or nll_destroy_model; NULL detaches them).  A binned dataset is its bin
 * centres weighted by the counts (Sec. 5.1 sets such binned fits against
 * unbinned ones); sWeights may be of either sign; weights are not
 * checked.  With weights attached:
 *   NLL = -sum_i w_i log p(x_i), gradient likewise; an extended model adds
 *   nu - W ln nu with W = sum_i w_i; nll_fit scales its steps by 1/W.
 *   nll_eval, nll_eval_grad, nll_fit and their step timing take them; the
 *   other entry points (batched, points, BHHH, autotuner) return
 *   NLL_ERR_UNSUPPORTED while they are attached.
 * Compiled for FP64 shapes over at most 3 observables.  One logarithm more
 * per event than the unweighted pass.  Errors: NLL_ERR_STATE (no data),
 * NLL_ERR_ARG (misaligned), NLL_ERR_UNSUPPORTED (FP32C or no weighted
 * kernel for the shape). */
nll_status nll_set_weights(nll_model* model, const double* weights);

/* Enqueue: NLL at theta (device [n_param]) into *nll_out (device [1]).
 * A parameter outside its range or an invalid density yields +inf and a
 * status bit read by nll_sync. */
nll_status nll_eval(nll_model* model, const double* theta, double* nll_out);

/* Enqueue: NLL and gradient (device [n_param]) from one fused pass. */
nll_status nll_eval_grad(nll_model* model, const double* theta, double* nll_out, double* grad_out);

/* Enqueue: many datasets in one launch.  Set s holds the attached events
 * [offsets[s], offsets[s+1]) (device int64 [n_sets+1]) and is evaluated at
 * theta[s * n_param ...] (device).  nll_out[s] (device), grad_out (device
 * [n_sets * n_param], NULL for NLL only) and status_out[s] (device, NULL
 * allowed: an nll_status per set).  The offsets must be non-decreasing
 * within [0, n_events]; otherwise every set reports NLL_ERR_ARG and +inf. */
nll_status nll_eval_batched(nll_model* model, int32_t n_sets, const int64_t* offsets, const double* theta,
                            double* nll_out, double* grad_out, int32_t* status_out);

/* Bytes of the fixed device array that nll_eval_batched_noalloc works in
 * (one copy per GPU, held until the process ends). */
#define NLL_NOALLOC_SCRATCH_BYTES (32u << 20)

/* Enqueue: nll_eval_batched without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * must not call hipMalloc).  Arguments, results and errors as
 * nll_eval_batched, and the same kernels and launch schedule, so the
 * results are the same bits.  The pass's scratch (tile schedule, per-set
 * constants, the work items and their partial sums) lives in one fixed
 * array of NLL_NOALLOC_SCRATCH_BYTES per GPU instead of the model's own
 * buffers; the array is looked up (hipGetSymbolAddress) on the first call
 * on each device.  It needs
 *   align256(8 (n_sets + 1)) + align256(4 n_sets) + align256(24 I)
 *   + align256(8 (H + 1)) + align256(C n_sets) + align256(T n_sets)
 *   + I * 16 (A + 1)  bytes,
 * with H = G ceil(n_events / (G tile_events)) chunks of the batched pass
 * (G = n_cu * sets_blocks_per_cu), I = n_sets + H + 1 work items (a set's
 * parts in the chunks), C the per-set
 * constant block and T the per-set tables of a Hypatia2 leaf (0 without
 * one; C + T is nll_info's per_set_bytes), and A the model's
 * accumulators (n_accumulators); a larger request returns NLL_ERR_SCRATCH
 * before anything is enqueued (4096 sets over 4.1e8 events of a one-leaf
 * model need about 22 MB).  Every word the pass reads is written earlier
 * in the same call, so nothing has to start at zero.  All calls on one GPU
 * share the array: calls that overlap on that GPU (other models, other
 * streams, other host threads) race and must be serialised by the caller;
 * the array keeps the last call's contents. */
nll_status nll_eval_batched_noalloc(nll_model* model, int32_t n_sets, const int64_t* offsets,
                                    const double* theta, double* nll_out, double* grad_out,
                                    int32_t* status_out);

/* Enqueue: the attached dataset at many parameter points in one pass (the
 * minimiser's repeated evaluations of the likelihood at different
 * parameter values, Sec. 1; a likelihood scan).  Point p is
 * theta[p * n_param ...] (device); nll_out[p] (device), grad_out (device
 * [n_points * n_param], NULL for NLL only) and status_out[p] (device, NULL
 * allowed) as in nll_eval_batched, each point normalised and checked on
 * its own.  The events are read once per point (work items of up to
 * tile_events events over all points share a persistent grid of at most
 * 4 blocks per CU; the tile is halved, down to 4096 events, while there
 * are fewer than two items per block). */
nll_status nll_eval_points(nll_model* model, int32_t n_points, const double* theta, double* nll_out,
                           double* grad_out, int32_t* status_out);

/* Enqueue: independent gradient-descent fits, one per set, all on the
 * device.  Each of the n_steps steps evaluates NLL and gradient at the
 * current proposal of every set in one launch; a proposal is accepted when
 * its NLL is finite and exceeds the last accepted one by at most 4 ulps
 * (rounding noise), otherwise that set's step size is halved; the next proposal is
 * theta_acc - eta * grad_acc / N_s over the free parameters.  theta (device
 * [n_sets * n_param]) holds the start points on entry and the last accepted
 * points on completion; nll_out / grad_out / status_out as above (at the
 * accepted points).  The whole fit is recorded once into a HIP graph and
 * replayed on later calls with the same arguments. */
nll_status nll_fit_batched(nll_model* model, int32_t n_sets, const int64_t* offsets, double* theta,
                           int32_t n_steps, double eta, double* nll_out, double* grad_out, int32_t* status_out);

/* Enqueue: the same fit on all attached events as one dataset.  One launch
 * per step: each launch first takes the previous step's update (in every
 * block, from that step's block records) and then evaluates the new
 * proposal; one finishing kernel takes the last step's update.  Library
 * scratch holds the fit state in two buffers by step parity. */
nll_status nll_fit(nll_model* model, double* theta, int32_t n_steps, double eta, double* nll_out,
                   double* grad_out, int32_t* status_out);

/* Enqueue: NLL, gradient and the BHHH matrix B = sum_i s_i s_i^T of the
 * events' scores s_i = d log p(x_i) / d theta (device [n_param * n_param],
 * row-major, symmetric; plus N / nu^2 at every pair (nu_i, nu_j) of the
 * parameters that make the expected count of an extended model;
 * rows and columns of fixed parameters 0) from one pass.  B approximates
 * the NLL's Hessian near the optimum (Berndt, Hall, Hall and Hausman 1974):
 * the outer-product information for the second-order minimiser that the
 * paper's fitTo leaves to MINUIT (Sec. 5.3), and a covariance estimate.
 * Compiled for FP64 shapes with at most 6 score features (responsibilities
 * of a mixture's terms plus the leaves' parameter features); other shapes
 * return NLL_ERR_UNSUPPORTED. */
nll_status nll_eval_bhhh(nll_model* model, const double* theta, double* nll_out, double* grad_out,
                         double* bhhh_out);

/* Enqueue: a damped BHHH fit (Levenberg-Marquardt on B) on all attached
 * events.  The proposal is theta_acc + d with (B_acc + lambda D) d =
 * -grad_acc over the free parameters, D the diagonal of B_acc floored at
 * 1e-12 of its largest entry, solved by Cholesky; acceptance as in nll_fit,
 * then lambda = max(lambda / 10, 1e-12), otherwise lambda *= 10; a damped
 * matrix that is not positive definite is retried with ten times the
 * damping at most 8 times, else the proposal is theta_acc.  lambda (> 0) is
 * the starting damping; the rest as nll_fit (recorded into a HIP graph).
 * NLL_ERR_UNSUPPORTED where nll_eval_bhhh is. */
nll_status nll_fit_bhhh(nll_model* model, double* theta, int32_t n_steps, double lambda, double* nll_out,
                        double* grad_out, int32_t* status_out);

/* Synchronise the model's stream and report (and clear) the errors found on
 * the device since the last call: NLL_ERR_PARAM_RANGE or NLL_ERR_INVALID_PDF
 * (also in *status_out if non-NULL), NLL_ERR_DEVICE on a runtime error. */
nll_status nll_sync(nll_model* model, int32_t* status_out);

/* Launch schedule of the streaming kernels.  A new model starts with
 * {4, 2, 16384, 16, 2}, or {2, 2, 16384, 16, 2} for shapes with more than 8
 * gradient accumulators (n_accumulators in nll_model_info); persistent
 * grids reserve LDS so that at most the given number of blocks share a CU. */
typedef struct nll_schedule {
  int32_t unroll;             /* events per thread per tile: 2, 4 or 8 (8
                                 falls back to 4 for shapes with more than 8
                                 accumulators)                              */
  int32_t blocks_per_cu;      /* persistent grid = CUs * blocks_per_cu     */
  int32_t tile_events;        /* batched: events per chunk; the attached
                                 events are cut into rounds of G chunks,
                                 block b streams the b-th chunk of every
                                 round (the last round's G chunks split
                                 what remains equally); nll_eval_points:
                                 at most this many events per (point,
                                 tile) work item                            */
  int32_t sets_blocks_per_cu; /* batched: grid G = CUs * sets_blocks_per_cu */
  int32_t sets_unroll;        /* batched: events per thread per tile, as
                                 unroll                                     */
} nll_schedule;

nll_status nll_get_schedule(const nll_model* model, nll_schedule* out);
/* Values outside unroll and sets_unroll in {2,4,8}, blocks_per_cu in [1,32],
 * tile_events in [1024, 1<<22] (multiple of 512), sets_blocks_per_cu in
 * [1,32] give NLL_ERR_ARG. */
nll_status nll_set_schedule(nll_model* model, const nll_schedule* sched);

/* Time the candidate schedules on the attached data (synchronises; several
 * evaluations per candidate), check each candidate's NLL against the
 * current schedule's (1e-12 relative in FP64; max(1e-9, 1e-6/sqrt(N)), or
 * 1e-6 for sets, in NLL_FP32C, whose single-precision per-thread sums
 * regroup with the schedule), keep the fastest.  which: 1 = single dataset,
 * 2 = batched with the given sets (n_sets/offsets/theta as in
 * nll_eval_batched).  Results are cached per model shape, precision and
 * event-count bucket in the file named by $NLLMI_TUNE_CACHE, if set. */
nll_status nll_autotune(nll_model* model, int32_t which, int32_t n_sets, const int64_t* offsets,
                        const double* theta);

/* Options (nll_set_option):
 *   NLL_OPT_GRAPH        1 (default): fits are recorded once into a HIP graph
 *                        and replayed; 0: fits are enqueued eagerly
 *   NLL_OPT_STEP_TIMING  1: fits are enqueued eagerly with a HIP event before
 *                        the first and after every step; 2: eagerly, with
 *                        the event-streaming kernel of every step launched
 *                        with a start and a stop event attached
 *                        (hipExtLaunchKernel), so that they record that
 *                        dispatch's own start and end (its duration alone,
 *                        without queue gaps; in a gradient-descent fit the
 *                        launch includes the previous step's update); read
 *                        by nll_step_times; 0 (default): no events.
 *                        Other values: NLL_ERR_ARG.                        */
enum nll_option { NLL_OPT_GRAPH = 1, NLL_OPT_STEP_TIMING = 2 };
nll_status nll_set_option(nll_model* model, int32_t option, int32_t value);

/* Synchronise and copy the duration in milliseconds of each step (or of each
 * step's streaming kernel, NLL_OPT_STEP_TIMING = 2) of the most recent fit run
 * with NLL_OPT_STEP_TIMING on (at most cap values; the count is written to
 * *n).  NLL_ERR_STATE if no timed fit has run. */
nll_status nll_step_times(nll_model* model, float* ms, int32_t cap, int32_t* n);

typedef struct nll_info {
  char variant[64];   /* compiled shape the model was lowered onto */
  int32_t n_leaf, n_term, n_accumulators, precision;
  int32_t n_cu;
  int64_t n_events;
  int32_t per_set_bytes;  /* device bytes of one set's per-point constants */
} nll_info;
nll_status nll_get_info(const nll_model* model, nll_info* out);

const char* nll_status_string(nll_status status);

/* Measurement utility: enqueue one read of n doubles at x (device, 16-byte
 * aligned) on `stream` (hipStream_t, NULL: default) by a streaming kernel of
 * n_blocks blocks of 256 threads (the likelihood kernels' pattern: tiles
 * of 8 x 256 consecutive doubles round robin over the blocks, two tiles of
 * non-temporal loads in flight ahead); block b writes the sum of the values
 * it read to block_sums[b]
 * (device [n_blocks]).  Timed by the caller, it gives the HBM read rate a
 * streaming pass reaches on the device, next to the data sheet's peak
 * (the likelihood kernels read their event columns the same way, Sec. 5.2).
 * Errors: NLL_ERR_ARG (null or misaligned pointers, n < 0, n_blocks outside
 * 1 .. 2^20), NLL_ERR_DEVICE. */
nll_status nll_read_probe(const double* x, int64_t n, double* block_sums, int32_t n_blocks, void* stream);

/* ------------------------------------------------------------------------
 * Binned template likelihood of HistFactory type (the binned models the
 * paper names as the next target of its work, Summary; HistFactory builds
 * models from histograms, Sec. 1).  The paper defines no formulas; the
 * reading follows the HistFactory definitions:
 *   bins b (channels concatenated), observed counts n_b >= 0, samples s with
 *   nominal expected counts T_sb, and modifiers, each acting on one sample
 *   through one parameter (a parameter may drive several):
 *     NLL_HF_NORMFACTOR  the sample times theta_p
 *     NLL_HF_NORMSYS     the sample times hi^a (a >= 0) or lo^-a (a < 0),
 *                        a = theta_p; hi, lo > 0
 *     NLL_HF_HISTOSYS    the sample's bins plus a (up_b - T_sb) (a >= 0) or
 *                        a (T_sb - down_b) (a < 0)
 *   nu_b = sum_s (product of the sample's factors) (T_sb + histosys terms)
 *   NLL  = sum_b (nu_b - n_b ln nu_b)
 *          + 1/2 sum_{constrained p} ((theta_p - m_p) / s_p)^2
 *   (a bin with n_b = 0 contributes nu_b; no ln n_b! terms; Gaussian
 *   constraints of mean m_p and width s_p, 0 and 1 by default, without
 *   their normalisation; a luminosity parameter is a normfactor on the
 *   samples it scales, constrained with mean 1 and width its relative
 *   uncertainty).  The derivative at a = 0 is the a >= 0 side's.  With
 *   interp = 1 a modifier uses the smooth codes instead (HistFactory's
 *   "code 4"): for |a| < 1 a normsys factor is 1 + sum_{i=1..6} c_i a^i,
 *   the polynomial meeting hi^a and lo^-a at a = +1, -1 with equal value,
 *   slope and curvature, and a histosys delta is
 *   a (S + a A (15 + a^2 (3 a^2 - 10))), S = (du + dd)/2, A = (du - dd)/16,
 *   du = up - T, dd = T - down (linear beyond +-1).  A parameter outside
 *   [lo, hi] gives +inf and NLL_ERR_PARAM_RANGE, nu_b < 0 or nu_b = 0 with
 *   n_b > 0 gives +inf and NLL_ERR_INVALID_PDF, both through nll_hf_sync.
 * Limits: 1..8 samples, <= 24 histosys (<= 12 when any uses interp = 1),
 * <= 16 normsys, <= 8 normfactor modifiers, 1..32 parameters.
 * ---------------------------------------------------------------------- */
enum nll_hf_modifier_type { NLL_HF_NORMFACTOR = 1, NLL_HF_NORMSYS = 2, NLL_HF_HISTOSYS = 3 };

typedef struct nll_hf_modifier {
  int32_t type;    /* nll_hf_modifier_type */
  int32_t sample;  /* 0 .. n_samples-1 */
  int32_t param;   /* 0 .. n_param-1 */
  int32_t interp;  /* normsys, histosys: 0 exponential / linear, 1 smooth */
  double hi, lo;   /* NLL_HF_NORMSYS only */
} nll_hf_modifier;

typedef struct nll_hf_desc {
  int64_t n_bins;
  int32_t n_samples;
  int32_t n_param;
  const double* param_lo;            /* n_param (host) */
  const double* param_hi;
  const uint8_t* param_free;         /* n_param, 0: fixed (gradient entry 0) */
  const uint8_t* param_constrained;  /* n_param, 1: + ((theta - mean) / sigma)^2 / 2 */
  const double* param_mean;          /* n_param or NULL (0): constraint means */
  const double* param_sigma;         /* n_param or NULL (1): constraint widths, > 0 */
  int32_t n_modifiers;
  const nll_hf_modifier* modifiers;  /* n_modifiers (host) */
  int32_t device;
  void* stream;                      /* hipStream_t, 0 = default stream */
} nll_hf_desc;

typedef struct nll_hf_model nll_hf_model; /* opaque, owned by the library */

/* Validate the descriptor and allocate the model's device scratch.
 * Descriptor arrays are copied.  Errors: NLL_ERR_ARG (bad counts or
 * indices, hi or lo <= 0, interp not 0 or 1, a constraint width not
 * positive and finite), NLL_ERR_UNSUPPORTED (beyond the limits),
 * NLL_ERR_DEVICE, NLL_ERR_OOM. */
nll_status nll_hf_create(const nll_hf_desc* desc, nll_hf_model** out);

/* Release the model (waits for its stream). */
void nll_hf_destroy(nll_hf_model* model);

/* Attach the data (device arrays of n_bins doubles): counts, nominal[s] for
 * every sample, and up[h], down[h] for the h-th histosys modifier in
 * modifier order (may be NULL without histosys).  counts and nominal are
 * borrowed until the next nll_hf_set_data or nll_hf_destroy; the histosys
 * templates are read once into the library's delta templates up - T and
 * T - down (2 n_bins doubles per histosys).  Validates the counts
 * (finite, >= 0) and SYNCHRONISES the stream: NLL_ERR_DOMAIN otherwise. */
nll_status nll_hf_set_data(nll_hf_model* model, const double* counts, const double* const* nominal,
                           const double* const* up, const double* const* down);

/* Enqueue: NLL at theta (device [n_param]) into *nll_out (device [1]) and,
 * if grad_out is not NULL, its gradient (device [n_param]).  One streaming
 * pass over the bins (8 (1 + samples + histosys) bytes per bin) and one
 * finishing block. */
nll_status nll_hf_eval(nll_hf_model* model, const double* theta, double* nll_out, double* grad_out);

/* Per-bin statistical parameters (HistFactory's staterror: the templates'
 * own statistical error, Barlow-Beeston lite).  The samples flagged in
 * sample_mask (bit s: sample s; nonzero, below 2^n_samples) share one
 * factor gamma_b per bin, with a Gaussian constraint of width sigma_b:
 *   nu_b = gamma_b (flagged samples' terms of bin b, histosys deltas
 *          included) + (the other samples' terms),
 *   NLL += 1/2 sum_b (gamma_b - 1)^2 / sigma_b^2.
 * sigma (device [n_bins]; the flagged templates' relative statistical
 * error per bin) is read once, now, into the library's 1/sigma_b^2; a bin
 * with sigma_b <= 0 or not finite has no parameter (gamma_b taken as 1,
 * derivative 0).  Enqueued on the model's stream; may be called again to
 * replace mask and widths.  Errors: NLL_ERR_ARG (mask, unaligned sigma),
 * NLL_ERR_DEVICE, NLL_ERR_OOM. */
nll_status nll_hf_set_staterror(nll_hf_model* model, uint32_t sample_mask, const double* sigma);

/* As nll_hf_set_staterror with a Poisson constraint instead (HistFactory's
 * shapesys: the templates' statistical error as an auxiliary count
 * tau_b = 1/sigma_b^2 observed for the mean gamma_b tau_b):
 *   NLL += sum_b tau_b (gamma_b - ln gamma_b)
 * (the Poisson term without its constant ln Gamma(tau + 1) - tau ln tau),
 * d NLL / d gamma_b = w_b (flagged part of nu_b) + tau_b (1 - 1/gamma_b);
 * gamma_b <= 0 in a bin with a parameter is an invalid density.  The model
 * keeps the last of nll_hf_set_staterror / nll_hf_set_shapesys. */
nll_status nll_hf_set_shapesys(nll_hf_model* model, uint32_t sample_mask, const double* sigma);

/* Enqueue: as nll_hf_eval with the per-bin statistical parameters at gamma
 * (device [n_bins], caller's): NLL into *nll_out, the parameters' gradient
 * into grad_out (device [n_param] or NULL) and d NLL / d gamma_b =
 * w_b (flagged part of nu_b) + (gamma_b - 1) / sigma_b^2, w_b = 1 - n_b/nu_b
 * (1 where n_b = 0), into grad_gamma (device [n_bins] or NULL; 0 for bins
 * without a parameter).  24 more bytes per bin than nll_hf_eval (gamma,
 * 1/sigma^2, the derivative).  Status as nll_hf_eval (a non-finite or
 * negative gamma_b that makes nu_b invalid: NLL_ERR_INVALID_PDF through
 * nll_hf_sync).  NLL_ERR_STATE before nll_hf_set_data and
 * nll_hf_set_staterror. */
nll_status nll_hf_eval_stat(nll_hf_model* model, const double* theta, const double* gamma, double* nll_out,
                            double* grad_out, double* grad_gamma);

/* Synchronise and return (and clear) the device status (as nll_sync). */
nll_status nll_hf_sync(nll_hf_model* model, int32_t* status_out);

/* ------------------------------------------------------------------------
 * Just-in-time densities (Sec. 4: PDFs given as formula strings, compiled
 * at run time).  One observable x on [obs_lo, obs_hi] and a density
 * expression g(x; p[0] .. p[n_param-1]) in C syntax (double arithmetic;
 * + - * /, exp log sqrt pow sin cos tan atan tanh sinh cosh asinh erf fabs),
 * normalised over the range by composite 256-point Gauss-Legendre on 1, 2,
 * 4, ... 256 equal panels until two levels agree (no agreement is an
 * invalid density); the same expressions serve as NLL_JIT leaves of
 * composite models (nll_node_desc):
 *   NLL = -sum_i log g(x_i) + N log Z,   Z = int g dx,
 * with the gradient from forward-mode dual numbers in the same pass.  An
 * event with g <= 0 or non-finite, or Z <= 0, gives +inf and
 * NLL_ERR_INVALID_PDF; a parameter outside its range NLL_ERR_PARAM_RANGE
 * (both through nll_jit_sync).  The expression is compiled into device code
 * as given: it must come from a trusted source, as any code the process
 * runs.  1 <= n_param <= 8.
 * ---------------------------------------------------------------------- */
typedef struct nll_jit_desc {
  const char* density;        /* C expression in x and p[k], <= 4096 characters */
  double obs_lo, obs_hi;
  int32_t n_param;
  const double* param_lo;     /* n_param (host) */
  const double* param_hi;
  const uint8_t* param_free;  /* n_param or NULL (all free) */
  int32_t device;
  void* stream;               /* hipStream_t, 0 = default stream */
} nll_jit_desc;

typedef struct nll_jit_model nll_jit_model; /* opaque, owned by the library */

/* Compile the density for the device (hipRTC; ~0.5-2 s) and allocate the
 * model's scratch.  log (may be NULL): the compiler's messages, truncated
 * to log_cap bytes.  Errors: NLL_ERR_ARG (bad descriptor, or the expression
 * does not compile: see log), NLL_ERR_UNSUPPORTED (more than 8 parameters or
 * a longer expression), NLL_ERR_DEVICE, NLL_ERR_OOM. */
nll_status nll_jit_create(const nll_jit_desc* desc, nll_jit_model** out, char* log, int32_t log_cap);

/* Release the model and its code object (waits for its stream). */
void nll_jit_destroy(nll_jit_model* model);

/* Attach n events (device array, borrowed until the next call or destroy);
 * validates the range and SYNCHRONISES the stream (NLL_ERR_DOMAIN). */
nll_status nll_jit_set_data(nll_jit_model* model, const double* x, int64_t n);

/* Enqueue: NLL at theta (device [n_param]) into *nll_out (device [1]) and,
 * if grad_out is not NULL, its gradient (device [n_param]). */
nll_status nll_jit_eval(nll_jit_model* model, const double* theta, double* nll_out, double* grad_out);

/* Synchronise and return (and clear) the device status (as nll_sync). */
nll_status nll_jit_sync(nll_jit_model* model, int32_t* status_out);

#ifdef __cplusplus
}
#endif

#endif /* NLLMI_NLL_H */

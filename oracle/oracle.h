/*
 * oracle.h -- scalar FP64 reference evaluator for unbinned negative
 * log-likelihoods of composed probability densities.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include,
 * link or call this code; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.  It shares no source with
 * the GPU library (its own types, its own quadrature rule, its own
 * special-function series).
 *
 * What it computes (paper, Sec. 5.1): for every entry of the dataset the
 * observable values are written into the leaves of the computation graph
 * and the probability of the top node is obtained by evaluating the
 * daughters and their normalisation; constant (parameter-only) branches,
 * i.e. the normalisation integrals, are computed once per parameter point.
 * The result is NLL(theta) = -sum_i log p(x_i; theta) (natural log),
 * accumulated with Neumaier-compensated FP64 sums, together with the
 * analytic gradient dNLL/dtheta obtained by forward-mode differentiation of
 * the same recursion (normalisation derivatives included).
 *
 * Normalisation (paper, Sec. 3, "Analytic Integrals"): closed forms when
 * requested, otherwise 256-point Gauss-Legendre quadrature, either on one
 * panel over the whole range or split into panels on which the integrand
 * is analytic (Crystal Ball junction, ARGUS square-root endpoint).
 *
 * Parameter and observable range checks follow Sec. 3 ("Checking
 * parameters"): a parameter outside its allowed range returns
 * ORC_E_PARAM with NLL = +inf, an event outside the closed observable
 * range returns ORC_E_DOMAIN, a non-positive or non-finite probability
 * returns ORC_E_PDF with NLL = +inf.
 */
#ifndef NLL_ORACLE_H
#define NLL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum orc_kind {
  ORC_GAUSS = 1, /* params (mu, sigma)                         */
  ORC_EXP = 2,   /* params (c)            g = exp(c x)           */
  ORC_CHEB = 3,  /* params (a_1..a_K)     g = 1 + sum a_k T_k(x') */
  ORC_CB = 4,    /* params (m0, sigma, alpha, n), low-side tail   */
  ORC_ARGUS = 5, /* params (m0, c), power 1/2                    */
  ORC_SUM = 6,   /* params (f_1..f_{k-1}) over k children: fractions,
                    or (nu_1..nu_k): yields, p = sum nu_j p_j / sum nu */
  ORC_PROD = 7,  /* no params; children on disjoint observables   */
  ORC_JOHNSON = 8, /* params (mu, lambda, gamma, delta), S_U family */
  ORC_CHI2 = 9,    /* params (nu): g = x^(nu/2-1) e^(-x/2), 0 <= lo  */
  ORC_HYPATIA = 10 /* params (mu, sigma, lambda, zeta, beta, a_l, n_l, a_r,
                      n_r): generalised hyperbolic core, power-law tails */
};

enum orc_norm {
  ORC_NORM_CLOSED = 0,    /* closed-form integral and derivatives        */
  ORC_NORM_GL_SPLIT = 1,  /* 256-point Gauss-Legendre per analytic panel */
  ORC_NORM_GL_SINGLE = 2  /* 256-point Gauss-Legendre on one panel       */
};

enum orc_status {
  ORC_OK = 0,
  ORC_E_ARG = -1,
  ORC_E_UNSUPPORTED = -2,
  ORC_E_PARAM = -3,
  ORC_E_DOMAIN = -4,
  ORC_E_PDF = -5
};

#define ORC_MAX_OBS 4
#define ORC_MAX_PAR 32
#define ORC_MAX_NODE 16
#define ORC_NODE_PAR 12
#define ORC_NODE_CHILD 8

typedef struct orc_node {
  int32_t kind;
  int32_t obs; /* observable index for leaves, -1 otherwise */
  int32_t n_param;
  int32_t param[ORC_NODE_PAR];
  int32_t n_child;
  int32_t child[ORC_NODE_CHILD];
  int32_t norm; /* orc_norm, leaves only */
} orc_node;

typedef struct orc_model {
  int32_t n_obs;
  double lo[ORC_MAX_OBS], hi[ORC_MAX_OBS];
  int32_t n_param;
  double par_lo[ORC_MAX_PAR], par_hi[ORC_MAX_PAR];
  uint8_t par_free[ORC_MAX_PAR];
  int32_t n_node;
  orc_node node[ORC_MAX_NODE];
  int32_t root;
  int32_t extended;    /* 1: add nu - N ln nu (Poisson yield term) */
  int32_t yield_param; /* index of nu when extended, or -1: nu is the sum
                          of the yields of the root's yield SUM (the root
                          itself, or the one such SUM among the children of
                          a root PROD)                                    */
} orc_model;

/* Structural validation (topological order, arities, disjoint products). */
int orc_check_model(const orc_model* m);

/* Normalisation integral Z of leaf `node` over its observable range and
 * dZ/dtheta for every model parameter (dZ has n_param entries).        */
int orc_leaf_norm(const orc_model* m, int32_t node, const double* theta,
                  double* Z, double* dZ);

/* log p and d log p / d theta (n_param entries, may be NULL) for ONE event
 * x[0..n_obs-1].                                                        */
int orc_log_density(const orc_model* m, const double* x, const double* theta,
                    double* logp, double* dlogp);

/* NLL and gradient (grad may be NULL) over n events held as columns
 * cols[obs][i].  threads <= 1 runs serially; otherwise contiguous chunks
 * are combined in fixed order.  stats (may be NULL) receives
 * [sum |l_i|, then sum_i |d l_i / d theta_k| for every k].              */
int orc_nll(const orc_model* m, const double* const* cols, int64_t n,
            const double* theta, int32_t threads, double* nll, double* grad,
            double* stats);

/* Weighted events (a binned dataset is its bin centres weighted by the
 * counts, Sec. 5.1 contrasts such fits with unbinned ones; sWeighted fits
 * have weights of either sign): NLL = -sum_i w_i log p(x_i), its gradient
 * likewise, and in an extended model nu - W ln nu with W = sum_i w_i.
 * stats as orc_nll over the weighted terms; wsum (may be NULL) gets W.   */
int orc_nll_weighted(const orc_model* m, const double* const* cols, const double* w,
                     int64_t n, const double* theta, int32_t threads, double* nll,
                     double* grad, double* stats, double* wsum);

/* Many datasets: set s holds events [offsets[s], offsets[s+1]) and its own
 * parameter row theta[s*n_param ...].  Per-set status in status[s].      */
int orc_nll_batched(const orc_model* m, const double* const* cols,
                    const int64_t* offsets, int32_t n_sets, const double* theta,
                    int32_t threads, double* nll, double* grad, int32_t* status);

/* Gradient descent on the mean NLL: proposal theta' = theta_acc -
 * eta * g_acc / N over free parameters; a proposal is accepted when its NLL
 * is finite and exceeds the last accepted one by at most 4 ulps (an
 * increase within rounding noise is not an increase), otherwise eta is
 * halved.  Exactly n_steps evaluations; the first evaluates the start
 * point.  On return theta/nll/grad hold the last accepted point and
 * eta_out the final step size.  trace (may be NULL) receives per step
 * [nll_prop, theta_prop...].                                            */
int orc_gd_fit(const orc_model* m, const double* const* cols, int64_t n,
               double* theta, int32_t n_steps, double eta, int32_t threads,
               double* nll, double* grad, double* eta_out, double* trace);

/* orc_gd_fit with the acceptance slack given: a proposal is accepted when
 * its NLL is finite and at most accept_ulps * DBL_EPSILON * |NLL_acc| above
 * the last accepted one (0: the literal "no increase" rule).             */
int orc_gd_fit_accept(const orc_model* m, const double* const* cols, int64_t n,
                      double* theta, int32_t n_steps, double eta, double accept_ulps,
                      int32_t threads, double* nll, double* grad, double* eta_out,
                      double* trace);

/* orc_gd_fit over weighted events: the weighted NLL of orc_nll_weighted,
 * steps scaled by 1/W instead of 1/N (W <= 0: no scaling).              */
int orc_gd_fit_weighted(const orc_model* m, const double* const* cols, const double* w,
                        int64_t n, double* theta, int32_t n_steps, double eta,
                        int32_t threads, double* nll, double* grad, double* eta_out,
                        double* trace);

/* NLL, gradient and the BHHH matrix B = sum_i s_i s_i^T of the events'
 * scores s_i = d log p(x_i) / d theta (n_param x n_param, row-major,
 * symmetric), plus the Poisson term's second derivative N / nu^2 at
 * (nu, nu) in an extended model; rows and columns of fixed parameters 0.
 * (Berndt, Hall, Hall and Hausman, 1974: the outer product of the scores
 * approximates the Hessian of the NLL near the optimum.)                 */
int orc_nll_bhhh(const orc_model* m, const double* const* cols, int64_t n,
                 const double* theta, int32_t threads, double* nll, double* grad,
                 double* bhhh);

/* Damped BHHH minimiser (Levenberg-Marquardt on B): the proposal is
 * theta_acc + d with (B_acc + lambda D) d = -g_acc over the free
 * parameters, D = diag(B_acc) floored at 1e-12 of its largest entry,
 * solved by Cholesky.  Acceptance as in orc_gd_fit (finite, at most 4 ulps
 * above the last accepted NLL); on acceptance lambda = max(lambda / 10,
 * 1e-12), otherwise lambda *= 10.  A damped matrix that is not positive
 * definite is retried with ten times the damping, at most 8 times, else
 * the proposal is theta_acc.  Exactly n_steps evaluations, the first at
 * the start point; outputs as orc_gd_fit (lambda_out: final damping).    */
int orc_bhhh_fit(const orc_model* m, const double* const* cols, int64_t n,
                 double* theta, int32_t n_steps, double lambda, int32_t threads,
                 double* nll, double* grad, double* lambda_out, double* trace);

/* The same minimiser run independently on every set (threads over sets). */
int orc_gd_fit_batched(const orc_model* m, const double* const* cols,
                       const int64_t* offsets, int32_t n_sets, double* theta,
                       int32_t n_steps, double eta, int32_t threads,
                       double* nll, double* grad, int32_t* status);

/* log K_nu(z), the modified Bessel function of the second kind of real
 * order nu at z > 0, by the integral the Hypatia2 density uses.         */
int orc_log_bessel_k(double nu, double z, double* out);

/* n-point Gauss-Legendre rule on [-1, 1] (nodes ascending). */
int orc_gl_rule(int32_t n, double* x, double* w);

#ifdef __cplusplus
}
#endif

#endif /* NLL_ORACLE_H */

"""Pins of the scalar FP64 oracle against things other than itself.

Each test fixes the oracle to an external reference: a library routine
(scipy.stats densities, numpy Chebyshev and Legendre routines), an
independent numerical method (adaptive quadrature, extended-precision
summation, finite differences), a closed-form statistical result (the
Gaussian maximum-likelihood estimate) or an invariant of the definition.
The densities are the textbook ones the paper's models use (Sec. 3 and
5); the NLL is -sum_i log p(x_i) (Sec. 5.1).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import datagen
import oracle

OK, E_PARAM, E_DOMAIN, E_PDF = oracle.OK, oracle.E_PARAM, oracle.E_DOMAIN, oracle.E_PDF


def single_leaf_spec(kind, params, lo, hi, norm="analytic"):
    ps = [datagen.param(f"p{k}", v, -1e3, 1e3) for k, v in enumerate(params)]
    return {"obs": [{"name": "x", "lo": lo, "hi": hi}], "params": ps,
            "nodes": [{"kind": kind, "obs": 0, "params": list(range(len(params))), "norm": norm}],
            "root": 0}


# ---------------------------------------------------------------------------
# Library densities (scipy / numpy), truncated to the observable range
# ---------------------------------------------------------------------------

def lib_logpdf(kind, params, lo, hi, x):
    x = np.asarray(x, dtype=np.float64)
    if kind == "gauss":
        mu, s = params
        return stats.truncnorm.logpdf(x, (lo - mu) / s, (hi - mu) / s, loc=mu, scale=s)
    if kind == "exp":
        (c,) = params
        if c < 0:
            return stats.truncexpon.logpdf(x, b=(hi - lo) * -c, loc=lo, scale=-1.0 / c)
        # increasing exponential: mirror a decreasing one
        return stats.truncexpon.logpdf(hi + lo - x, b=(hi - lo) * c, loc=lo, scale=1.0 / c)
    if kind == "cb":
        m0, s, a, n = params
        d = stats.crystalball(a, n, loc=m0, scale=s)
        return d.logpdf(x) - np.log(d.cdf(hi) - d.cdf(lo))
    if kind == "argus":
        m0, c = params
        d = stats.argus(math.sqrt(-2.0 * c), scale=m0)
        top = min(hi, m0)
        return d.logpdf(x) - np.log(d.cdf(top) - d.cdf(lo))
    if kind == "johnson":
        mu, la, ga, de = params
        d = stats.johnsonsu(ga, de, loc=mu, scale=la)
        # mass inside the range from the side whose tail the range is in
        mass = d.sf(lo) - d.sf(hi) if d.cdf(lo) > 0.5 else d.cdf(hi) - d.cdf(lo)
        return d.logpdf(x) - np.log(mass)
    if kind == "chi2":
        (nu,) = params
        d = stats.chi2(nu)
        mass = d.sf(lo) - d.sf(hi) if d.cdf(lo) > 0.5 else d.cdf(hi) - d.cdf(lo)
        return d.logpdf(x) - np.log(mass)
    if kind == "cheb":
        coef = np.concatenate([[1.0], np.asarray(params, dtype=np.float64)])
        y = (2 * x - lo - hi) / (hi - lo)
        anti = np.polynomial.chebyshev.chebint(coef)
        z = 0.5 * (hi - lo) * (np.polynomial.chebyshev.chebval(1.0, anti)
                              - np.polynomial.chebyshev.chebval(-1.0, anti))
        return np.log(np.polynomial.chebyshev.chebval(y, coef)) - np.log(z)
    raise ValueError(kind)


LEAF_CASES = [
    ("gauss", (0.3, 1.5), -10.0, 10.0),
    ("gauss", (5.0, 0.4), 0.0, 10.0),
    ("gauss", (2.0, 0.7), 4.0, 9.0),      # both limits in the right tail
    ("gauss", (-3.0, 0.5), -10.0, -5.0),  # both limits in the left tail
    ("exp", (-0.7,), 0.0, 10.0),
    ("exp", (0.35,), -2.0, 3.0),
    ("cb", (5.28, 0.003, 1.5, 3.0), 5.20, 5.30),
    ("cb", (0.0, 1.0, 1.0, 2.5), -8.0, 4.0),
    ("cb", (1.0, 0.5, 0.8, 6.0), 0.5, 3.0),  # range starts inside the core? no: t_lo=-1 < -0.8
    ("argus", (5.29, -20.0), 5.20, 5.30),
    ("argus", (1.0, -5.0), 0.1, 0.95),
    ("cheb", (-0.28, -0.27, -0.07, 0.10), -1.0, 1.0),
    ("cheb", (0.2, -0.1), 2.0, 6.0),
    ("johnson", (5.28, 0.02, -0.5, 1.5), 5.0, 5.6),   # skewed mass peak
    ("johnson", (0.0, 1.0, 0.8, 0.7), -10.0, 10.0),  # heavy tails, truncated
    ("johnson", (2.0, 0.5, 2.0, 2.0), 0.0, 3.0),
    ("johnson", (0.0, 1.0, 0.0, 1.0), 5.0, 30.0),   # both limits in the right tail
    ("chi2", (5.0,), 0.0, 40.0),
    ("chi2", (3.5,), 0.0, 12.0),
    ("chi2", (30.0,), 10.0, 60.0),
    ("chi2", (3.0,), 0.5, 8.0),
]


@pytest.mark.parametrize("kind,params,lo,hi", LEAF_CASES)
@pytest.mark.parametrize("norm", ["analytic", "gl256"])
def test_leaf_log_density_matches_library(kind, params, lo, hi, norm):
    spec = single_leaf_spec(kind, params, lo, hi, norm)
    o = oracle.Oracle(spec)
    top = min(hi, params[0]) if kind == "argus" else hi
    xs = np.concatenate([np.linspace(lo, top, 41)[:-1] if kind == "argus" else np.linspace(lo, hi, 41),
                         [lo + 0.37 * (top - lo), lo + 0.91 * (top - lo)]])
    if kind == "chi2":
        xs = xs[xs > 0.0]  # the density is 0 there (nu > 2)
    ref = lib_logpdf(kind, params, lo, hi, xs)
    got = np.array([o.log_density([x], params)[1] for x in xs])
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-12 * np.maximum(1.0, np.abs(ref)).max())


@pytest.mark.parametrize("kind,params,lo,hi", LEAF_CASES)
def test_leaf_integrates_to_one_adaptive_quadrature(kind, params, lo, hi):
    """int p dx = 1 with an independent adaptive Gauss-Kronrod integrator
    that is told where the density has kinks."""
    spec = single_leaf_spec(kind, params, lo, hi)
    o = oracle.Oracle(spec)
    pts = []
    if kind == "cb":
        pts = [params[0] - params[2] * params[1], params[0]]
    if kind == "gauss":
        pts = [params[0]]
    if kind == "argus":
        pts = [params[0]]
    pts = [p for p in pts if lo < p < hi]
    f = lambda x: math.exp(o.log_density([x], params)[1]) if (kind != "argus" or x < params[0]) else 0.0
    val, err = integrate.quad(f, lo, hi, points=pts or None, epsabs=0, epsrel=2e-14, limit=500)
    assert abs(val - 1.0) < 1e-12, (val, err)


@pytest.mark.parametrize("kind,params,lo,hi", LEAF_CASES)
def test_closed_form_norm_equals_split_quadrature(kind, params, lo, hi):
    """Closed-form Z and dZ/dtheta against 256-point Gauss-Legendre on analytic panels."""
    za = oracle.Oracle(single_leaf_spec(kind, params, lo, hi, "analytic")).leaf_norm(0, params)
    zq = oracle.Oracle(single_leaf_spec(kind, params, lo, hi, "gl256")).leaf_norm(0, params)
    assert za[0] == OK and zq[0] == OK
    assert abs(za[1] - zq[1]) <= 1e-13 * abs(za[1])
    scale = np.maximum(np.abs(za[2]), abs(za[1]) / np.maximum(np.abs(params), 1e-3))
    np.testing.assert_allclose(za[2], zq[2], rtol=0, atol=1e-12 * scale.max())


@pytest.mark.parametrize("kind,params,lo,hi", LEAF_CASES)
def test_norm_derivative_matches_finite_difference(kind, params, lo, hi):
    o = oracle.Oracle(single_leaf_spec(kind, params, lo, hi, "analytic"))
    st, Z, dZ = o.leaf_norm(0, params)
    for k in range(len(params)):
        h = 1e-5 * max(abs(params[k]), 1e-2)
        if kind == "cb" and k == 1:
            h = 1e-7 * params[1] / 1e-3 * 1e-3
        p1 = list(params); p1[k] += h
        p2 = list(params); p2[k] -= h
        fd = (o.leaf_norm(0, p1)[1] - o.leaf_norm(0, p2)[1]) / (2 * h)
        assert abs(fd - dZ[k]) <= 1e-6 * max(abs(dZ[k]), abs(Z) / max(abs(params[k]), 1e-2)), (k, fd, dZ[k])


def test_single_panel_quadrature_is_worse_at_kinks():
    """A single 256-point panel across the Crystal Ball junction and the ARGUS
    endpoint converges only algebraically (finding recorded in the design notes)."""
    cb = ("cb", (5.28, 0.003, 1.5, 3.0), 5.20, 5.30)
    ar = ("argus", (5.29, -20.0), 5.20, 5.30)
    for kind, params, lo, hi in (cb, ar):
        z_closed = oracle.Oracle(single_leaf_spec(kind, params, lo, hi, "analytic")).leaf_norm(0, params)[1]
        z_single = oracle.Oracle(single_leaf_spec(kind, params, lo, hi, "gl256_single")).leaf_norm(0, params)[1]
        rel = abs(z_single / z_closed - 1)
        assert 1e-9 < rel < 1e-3, (kind, rel)


def test_gauss_legendre_rule():
    x, w = oracle.gl_rule(256)
    xr, wr = np.polynomial.legendre.leggauss(256)
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, wr, rtol=0, atol=2e-14)
    # exact for all polynomials up to degree 511
    for k in range(0, 256, 15):
        approx = math.fsum(w * x ** (2 * k))
        assert abs(approx - 2.0 / (2 * k + 1)) < 1e-14 * max(1.0, 2.0 / (2 * k + 1)) * 4
        assert abs(math.fsum(w * x ** (2 * k + 1))) < 1e-15


# ---------------------------------------------------------------------------
# Whole models: composition, sufficient statistics, brute force
# ---------------------------------------------------------------------------

def lib_model_logpdf(spec, cols, theta):
    """log p of the three workload models from library densities."""
    names = [n["kind"] for n in spec["nodes"]]
    if names == ["gauss"]:
        lo, hi = spec["obs"][0]["lo"], spec["obs"][0]["hi"]
        return lib_logpdf("gauss", theta, lo, hi, cols[0])
    if names == ["gauss", "exp", "sum"]:
        lo, hi = spec["obs"][0]["lo"], spec["obs"][0]["hi"]
        f, mu, s, c = theta
        pg = np.exp(lib_logpdf("gauss", (mu, s), lo, hi, cols[0]))
        pe = np.exp(lib_logpdf("exp", (c,), lo, hi, cols[0]))
        return np.log(f * pg + (1 - f) * pe)
    if names == ["cb", "argus", "sum", "cheb", "prod"]:
        mlo, mhi = spec["obs"][0]["lo"], spec["obs"][0]["hi"]
        ylo, yhi = spec["obs"][1]["lo"], spec["obs"][1]["hi"]
        f = theta[0]
        pc = np.exp(lib_logpdf("cb", theta[1:5], mlo, mhi, cols[0]))
        m = cols[0]
        pa = np.where(m < theta[5], np.exp(lib_logpdf("argus", theta[5:7], mlo, mhi, np.minimum(m, theta[5] * (1 - 1e-16)))), 0.0)
        ly = lib_logpdf("cheb", theta[7:11], ylo, yhi, cols[1])
        return np.log(f * pc + (1 - f) * pa) + ly
    raise ValueError(names)


@pytest.mark.parametrize("config", [1, 2, 3])
def test_model_nll_matches_library_brute_force(config):
    """Tiny N (1, 2, 3, 16 events incl. range edges, the mode, the CB junction,
    the ARGUS endpoint region): NLL = -fsum(log p) from library densities."""
    w = datagen.workload(config, n=16)
    spec, theta = w["spec"], w["theta"]
    o = oracle.Oracle(spec)
    cols = [c.copy() for c in w["cols"]]
    if config == 1:
        cols[0][:4] = [-10.0, 10.0, 0.3, 0.3 + 1e-9]
    elif config == 2:
        cols[0][:4] = [0.0, 10.0, 5.0, 4.999]
    else:
        cols[0][:5] = [5.20, 5.30, 5.28 - 1.5 * 0.003, 5.289, 5.29]
        cols[1][:3] = [-1.0, 1.0, 0.0]
    for n in (1, 2, 3, 16):
        sub = [c[:n] for c in cols]
        ref = -math.fsum(lib_model_logpdf(spec, sub, theta))
        st, nll, _ = o.nll(sub, theta)
        assert st == OK
        assert abs(nll - ref) <= 2e-13 * max(1.0, abs(ref)), (n, nll, ref)


def test_gauss_nll_from_sufficient_statistics():
    """NLL = N log Z + sum (x - mu)^2 / (2 sigma^2), Z from the normal CDF,
    sum in extended precision; and NLL/N near 1/2 ln(2 pi e sigma^2)."""
    w = datagen.workload(1)
    x = w["cols"][0]
    for th in w["points"][:8]:
        mu, s = th
        st, nll, _ = oracle.Oracle(w["spec"]).nll(w["cols"], th)
        Z = s * math.sqrt(2 * math.pi) * (stats.norm.cdf((10 - mu) / s) - stats.norm.cdf((-10 - mu) / s))
        q = np.sum(((x.astype(np.longdouble) - mu) ** 2))
        ref = float(len(x) * np.longdouble(math.log(Z)) + q / (2 * np.longdouble(s) ** 2))
        assert abs(nll - ref) <= 1e-13 * abs(ref)
    st, nll, _ = oracle.Oracle(w["spec"]).nll(w["cols"], w["theta"])
    per_event = nll / len(x)
    assert abs(per_event - 0.5 * math.log(2 * math.pi * math.e * 1.5 ** 2)) < 5 * math.sqrt(0.5 / len(x))


def test_gauss_gd_fit_reaches_closed_form_mle():
    """Gradient descent on the wide-range Gaussian lands on the MLE
    mu = mean(x), sigma^2 = mean((x - mean)^2) (truncation at +-6.5 sigma
    shifts it by < 1e-9)."""
    w = datagen.workload(1)
    x = w["cols"][0].astype(np.longdouble)
    mu_hat = float(x.mean())
    s_hat = float(np.sqrt(((x - x.mean()) ** 2).mean()))
    st, th, nll, g, eta, tr = oracle.Oracle(w["spec"]).gd_fit(w["cols"], w["theta"], 50, 1.0, trace=True)
    assert st == OK
    assert abs(th[0] - mu_hat) <= 1e-8 * abs(mu_hat)
    assert abs(th[1] - s_hat) <= 1e-8 * s_hat
    assert np.all(np.diff(tr[:, 0]) <= 1e-9 * abs(nll))  # accepted every step: monotone
    assert np.max(np.abs(g)) / len(x) < 1e-10


def test_gd_acceptance_slack_reading():
    """Reading of "an increase halves the step" (the paper names no
    minimiser): an increase of the computed NLL within its own rounding,
    taken as 4 ulps of |NLL|, is not an increase of the function.  The
    literal rule (0 ulps) and this one are pinned against each other and
    against the closed-form optimum:
    - wherever the literal rule accepts every step, both trajectories are
      bitwise equal (c1 and most toys);
    - the literal rule can halve the step on rounding noise near the
      optimum and stall (here on a 122k-event toy: the step shrinks to
      2^-16 within 400 steps, 1e-9 short of stationarity), while the 4-ulp
      rule reaches a stationary point (|grad| / N <= 1e-12) in 50 steps on
      every toy, never above the literal rule's NLL by more than 4 ulps,
      and at the closed-form MLE within the truncation shift."""
    w = datagen.workload(1)
    o = oracle.Oracle(w["spec"])
    r0 = o.gd_fit(w["cols"], w["theta"], 50, 1.0, accept_ulps=0)
    r4 = o.gd_fit(w["cols"], w["theta"], 50, 1.0, accept_ulps=4)
    assert r0[0] == r4[0] == OK and np.array_equal(r0[1], r4[1]) and r0[2] == r4[2]
    x = w["cols"][0].astype(np.longdouble)
    assert abs(r4[1][0] - float(x.mean())) <= 1e-8 * abs(float(x.mean()))
    tw = datagen.toys_workload(n_sets=16, size_lo=1000, size_hi=200_000)
    stalled = 0
    for s in range(16):
        a, b = tw["offsets"][s], tw["offsets"][s + 1]
        xs = tw["cols"][0][a:b]
        n = b - a
        r0 = o.gd_fit([xs], tw["theta_start"], 50, 1.0, accept_ulps=0)
        r4 = o.gd_fit([xs], tw["theta_start"], 50, 1.0, accept_ulps=4)
        assert r0[0] == r4[0] == OK
        assert np.max(np.abs(r4[3])) / n <= 1e-12, s
        assert r4[2] <= r0[2] + 4 * 2.0 ** -52 * abs(r0[2]), s
        if r0[4] == 1.0:  # the literal rule never halved: the same trajectory
            assert np.array_equal(r0[1], r4[1]) and r0[2] == r4[2], s
        else:
            assert np.max(np.abs(r4[3])) <= np.max(np.abs(r0[3])), s
            r0_long = o.gd_fit([xs], tw["theta_start"], 400, 1.0, accept_ulps=0)
            if np.max(np.abs(r0_long[3])) / n > 1e-10:
                stalled += 1
        xl = xs.astype(np.longdouble)
        mle = np.array([float(xl.mean()), float(np.sqrt(((xl - xl.mean()) ** 2).mean()))])
        assert np.max(np.abs(r4[1] - mle)) <= 1e-7, s
    assert stalled >= 1  # the case that motivates the reading occurs in this sample


def test_gauss_mle_exact_on_very_wide_range():
    spec = datagen.gauss_spec(lo=-60.0, hi=60.0)
    cols = datagen.generate(spec, 20000, seed=11)
    x = cols[0].astype(np.longdouble)
    st, th, nll, g, eta = oracle.Oracle(spec).gd_fit(cols, datagen.theta_of(spec), 80, 1.0)
    assert abs(th[0] - float(x.mean())) < 1e-12
    assert abs(th[1] - float(np.sqrt(((x - x.mean()) ** 2).mean()))) < 1e-12


# ---------------------------------------------------------------------------
# Special cases and invariants
# ---------------------------------------------------------------------------

def test_mixture_endpoints_reduce_to_components():
    w = datagen.workload(2, n=5000)
    o = oracle.Oracle(w["spec"])
    f, mu, s, c = w["theta"]
    g_only = oracle.Oracle(datagen.gauss_spec(mu, s, 0.0, 10.0))
    e_only = oracle.Oracle(single_leaf_spec("exp", (c,), 0.0, 10.0))
    assert abs(o.nll(w["cols"], [1.0, mu, s, c])[1] - g_only.nll(w["cols"], [mu, s])[1]) < 1e-12 * 1e4
    assert abs(o.nll(w["cols"], [0.0, mu, s, c])[1] - e_only.nll(w["cols"], [c])[1]) < 1e-12 * 1e4


def test_flat_limits_give_uniform_nll():
    n = 3000
    cols = datagen.generate(datagen.mixture_spec(), n, seed=5)
    st, nll, _ = oracle.Oracle(single_leaf_spec("exp", (0.0,), 0.0, 10.0)).nll(cols, [0.0])
    assert abs(nll - n * math.log(10.0)) < 1e-11
    st, nll, _ = oracle.Oracle(single_leaf_spec("exp", (1e-14,), 0.0, 10.0)).nll(cols, [1e-14])
    assert abs(nll - n * math.log(10.0)) < n * 1e-14 * 10 + 1e-11
    ycols = [np.linspace(-1, 1, n)]
    st, nll, _ = oracle.Oracle(single_leaf_spec("cheb", (0.0, 0.0, 0.0, 0.0), -1.0, 1.0)).nll(ycols, [0.0] * 4)
    assert abs(nll - n * math.log(2.0)) < 1e-10


def test_cb_with_remote_tail_is_truncated_gauss():
    params = (0.3, 1.2, 50.0, 3.0)
    o = oracle.Oracle(single_leaf_spec("cb", params, -4.0, 5.0))
    xs = np.linspace(-4, 5, 31)
    got = np.array([o.log_density([x], params)[1] for x in xs])
    ref = lib_logpdf("gauss", (0.3, 1.2), -4.0, 5.0, xs)
    np.testing.assert_allclose(got, ref, atol=1e-13)


def test_product_with_flat_factor_adds_n_ln2():
    w = datagen.workload(3, n=4000)
    spec = w["spec"]
    theta = w["theta"].copy()
    theta[7:11] = 0.0
    st, nll2d, _ = oracle.Oracle(spec).nll(w["cols"], theta)
    mass = {"obs": [spec["obs"][0]], "params": spec["params"][:7], "nodes": spec["nodes"][:3], "root": 2}
    st, nll1d, _ = oracle.Oracle(mass).nll([w["cols"][0]], theta[:7])
    assert abs(nll2d - (nll1d + 4000 * math.log(2.0))) < 1e-12 * abs(nll2d)


@pytest.mark.parametrize("config", [1, 2, 3])
def test_permutation_and_additivity(config):
    w = datagen.workload(config, n=20000)
    o = oracle.Oracle(w["spec"])
    th = w["points"][1]
    st, full, g = o.nll(w["cols"], th)
    perm = np.random.default_rng(3).permutation(20000)
    st, pf, pg = o.nll([c[perm] for c in w["cols"]], th)
    assert abs(pf - full) <= 1e-13 * abs(full)
    np.testing.assert_allclose(pg, g, rtol=1e-11, atol=1e-9)
    a = o.nll([c[:7000] for c in w["cols"]], th)[1]
    b = o.nll([c[7000:] for c in w["cols"]], th)[1]
    assert abs(a + b - full) <= 1e-13 * abs(full)


def test_translation_and_scaling_of_gauss():
    spec = datagen.gauss_spec()
    cols = datagen.generate(spec, 10000, seed=9)
    o = oracle.Oracle(spec)
    th = np.array([0.25, 1.4])
    base = o.nll(cols, th)[1]
    shifted = datagen.gauss_spec(lo=-10 + 2.5, hi=10 + 2.5)
    assert abs(oracle.Oracle(shifted).nll([cols[0] + 2.5], th + [2.5, 0])[1] - base) < 1e-12 * abs(base) * 10
    sc = 4.0
    scaled = datagen.gauss_spec(lo=-10 * sc, hi=10 * sc)
    for p in scaled["params"]:
        p["lo"], p["hi"] = p["lo"] * sc, p["hi"] * sc
    v = oracle.Oracle(scaled).nll([cols[0] * sc], th * sc)[1]
    assert abs(v - (base + 10000 * math.log(sc))) < 1e-12 * abs(base) * 10


# ---------------------------------------------------------------------------
# Gradients against finite differences
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("config", [1, 2, 3])
def test_gradient_matches_central_differences(config):
    w = datagen.workload(config, n=4000)
    o = oracle.Oracle(w["spec"])
    th = w["points"][2]
    st, nll, g = o.nll(w["cols"], th)
    free = datagen.free_mask(w["spec"])
    for k in range(len(th)):
        if not free[k]:
            assert g[k] == 0.0
            continue
        h = 1e-4 * datagen.jitter_widths(w["spec"])[k]   # a small fraction of the parameter's scale

        def f(v):
            t = th.copy()
            t[k] = v
            return o.nll(w["cols"], t)[1]

        fd = (f(th[k] - 2 * h) - 8 * f(th[k] - h) + 8 * f(th[k] + h) - f(th[k] + 2 * h)) / (12 * h)
        bound = 50 * (2.2e-16 * abs(nll) / h) + 1e-6 * abs(g[k])
        assert abs(fd - g[k]) <= bound, (k, fd, g[k], bound)


@pytest.mark.parametrize("m", [5.2000, 5.2700, 5.28 - 1.5 * 0.003 - 1e-9, 5.28 - 1.5 * 0.003 + 1e-9,
                               5.2799, 5.2895, 5.28999, 5.2950, 5.3000])
def test_event_log_density_derivatives(m):
    """Per-event d log p / d theta against central differences at the
    Crystal Ball junction, in its core and tail, near the ARGUS endpoint."""
    spec = datagen.cb_argus_cheb_spec(cheb=(0.1, -0.2, 0.05, 0.02), norm="analytic")
    o = oracle.Oracle(spec)
    th = datagen.theta_of(spec)
    x = [m, 0.3]
    st, lp, d = o.log_density(x, th)
    assert st == OK
    m0, s, a = th[1], th[2], th[3]
    mj = m0 - a * s                      # Crystal Ball junction
    dist = {1: abs(m - mj), 2: abs(m - mj) / a, 3: abs(m - mj) / s}
    if m < th[5]:
        dist[5] = th[5] - m              # ARGUS endpoint
    for k in range(len(th)):
        scale = max(abs(th[k]), 1e-3)
        h = 1e-6 * scale
        if k in dist:
            h = max(min(h, 0.02 * dist[k]), 1e-12 * scale)

        def f(v):
            t = th.copy()
            t[k] = v
            return o.log_density(x, t)[1]

        fd = (f(th[k] - 2 * h) - 8 * f(th[k] - h) + 8 * f(th[k] + h) - f(th[k] + 2 * h)) / (12 * h)
        tol = 1e-6 * max(1.0, abs(d[k])) + 20 * 2.2e-16 * max(1.0, abs(lp)) / h
        assert abs(fd - d[k]) <= tol, (k, fd, d[k], h)


def test_cb_junction_is_continuous_with_zero_alpha_n_derivative():
    params = (5.28, 0.003, 1.5, 3.0)
    o = oracle.Oracle(single_leaf_spec("cb", params, 5.20, 5.30))
    mj = 5.28 - 1.5 * 0.003
    a = o.log_density([mj - 1e-14], params)
    b = o.log_density([mj + 1e-14], params)
    assert abs(a[1] - b[1]) < 1e-10
    np.testing.assert_allclose(a[2], b[2], atol=1e-5 * np.abs(a[2]).max())
    # on the junction d log g / d alpha and d log g / d n vanish on both sides;
    # what remains is -d log Z / d theta
    st, Z, dZ = o.leaf_norm(0, params)
    np.testing.assert_allclose(a[2][2:], -dZ[2:] / Z, rtol=1e-6)


def test_argus_near_endpoint_against_mpmath():
    """log g(m1) - log g(m2) for events within 1e-7 of the ARGUS endpoint,
    against a 40-digit evaluation (the normalisation cancels)."""
    import mpmath as mp
    mp.mp.dps = 40
    params = (5.29, -20.0)
    o = oracle.Oracle(single_leaf_spec("argus", params, 5.20, 5.30))
    m0, c = mp.mpf(params[0]), mp.mpf(params[1])

    def lg(m):
        m = mp.mpf(m)
        u = 1 - (m / m0) ** 2
        return mp.log(m) + mp.log(u) / 2 + c * u

    ref_m = 5.25
    for m in (5.2899999, 5.28999999999, 5.2899):
        got = o.log_density([m], params)[1] - o.log_density([ref_m], params)[1]
        want = float(lg(m) - lg(ref_m))
        assert abs(got - want) < 1e-13 * max(1.0, abs(want)), (m, got, want)


# ---------------------------------------------------------------------------
# Errors (Sec. 3, "Checking parameters")
# ---------------------------------------------------------------------------

def test_error_conventions():
    w = datagen.workload(2, n=100)
    o = oracle.Oracle(w["spec"])
    th = w["theta"]
    for bad in ([th[0], th[1], -0.1, th[3]], [1.2, th[1], th[2], th[3]], [float("nan"), th[1], th[2], th[3]]):
        st, nll, g = o.nll(w["cols"], bad)
        assert st == E_PARAM and nll == math.inf and np.all(g == 0)
    cols = [w["cols"][0].copy()]
    cols[0][7] = 10.5
    assert o.nll(cols, th)[0] == E_DOMAIN
    cols[0][7] = float("nan")
    assert o.nll(cols, th)[0] == E_DOMAIN
    cheb = oracle.Oracle(single_leaf_spec("cheb", (1.5, 0.0), -1.0, 1.0))
    st, nll, _ = cheb.nll([np.array([-0.9, 0.0, 0.9])], [1.5, 0.0])
    assert st == E_PDF and nll == math.inf
    st, nll, g = o.nll([np.zeros(0)], th)
    assert st == OK and nll == 0.0 and np.all(g == 0)


def test_batched_equals_single_sets():
    w = datagen.toys_workload(n_sets=12, size_lo=100, size_hi=3000)
    o = oracle.Oracle(w["spec"])
    th = np.tile(w["theta_start"], (12, 1)) * np.linspace(0.95, 1.05, 12)[:, None]
    st, nll, g, status = o.nll_batched(w["cols"], w["offsets"], th, threads=4)
    for s in range(12):
        a, b = w["offsets"][s], w["offsets"][s + 1]
        st1, v, gg = o.nll([w["cols"][0][a:b]], th[s])
        assert v == nll[s] and np.array_equal(gg, g[s]) and status[s] == OK


def test_batched_gd_matches_single_gd():
    w = datagen.toys_workload(n_sets=6, size_lo=1000, size_hi=5000)
    o = oracle.Oracle(w["spec"])
    th0 = np.tile(w["theta_start"], (6, 1))
    st, th, nll, g, status = o.gd_fit_batched(w["cols"], w["offsets"], th0, 50, 1.0, threads=3)
    for s in range(6):
        a, b = w["offsets"][s], w["offsets"][s + 1]
        x = w["cols"][0][a:b].astype(np.longdouble)
        r = o.gd_fit([w["cols"][0][a:b]], w["theta_start"], 50, 1.0)
        assert np.array_equal(r[1], th[s])
        assert abs(th[s][0] - float(x.mean())) < 1e-7 * max(1, abs(float(x.mean())))


def test_norms_against_40_digit_quadrature():
    """Closed-form and split-panel Z against mpmath's tanh-sinh quadrature at
    40 digits (tests/golden/mpmath_norms.json, written by make_mpmath_norms.py)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "mpmath_norms.json")
    cases = json.load(open(path))["cases"]
    for c in cases:
        want = float(c["Z"])
        for norm in ("analytic", "gl256"):
            o = oracle.Oracle(single_leaf_spec(c["kind"], c["params"], c["lo"], c["hi"], norm))
            st, Z, _ = o.leaf_norm(0, c["params"])
            assert st == OK
            assert abs(Z - want) <= 2e-14 * want, (c["kind"], norm, Z, want)


def test_extended_term_minimum_at_n_events():
    """With the Poisson yield term nu - N ln nu the NLL is minimal at nu = N
    and d NLL / d nu = 1 - N / nu (closed forms)."""
    spec = datagen.mixture_spec()
    spec["params"].append(datagen.param("nu", 1000.0, 1.0, 1e7))
    spec["extended"] = True
    spec["yield_param"] = 4
    cols = datagen.generate(datagen.mixture_spec(), 2500, seed=8)
    o = oracle.Oracle(spec)
    th = np.array([0.2, 5.0, 0.4, -0.7, 1000.0])
    st, v1, g1 = o.nll(cols, th)
    assert abs(g1[4] - (1 - 2500 / 1000.0)) < 1e-15
    th2 = th.copy()
    th2[4] = 2500.0
    st, v2, g2 = o.nll(cols, th2)
    assert g2[4] == 0.0 and v2 < v1
    base = oracle.Oracle(datagen.mixture_spec()).nll(cols, th[:4])[1]
    assert abs(v2 - (base + 2500 - 2500 * math.log(2500))) < 1e-12 * abs(v2)


@pytest.mark.parametrize("kind,params,lo,hi", [c for c in LEAF_CASES if c[0] in ("gauss", "exp", "cheb")])
def test_single_panel_quadrature_on_smooth_leaves(kind, params, lo, hi):
    za = oracle.Oracle(single_leaf_spec(kind, params, lo, hi, "analytic")).leaf_norm(0, params)
    zs = oracle.Oracle(single_leaf_spec(kind, params, lo, hi, "gl256_single")).leaf_norm(0, params)
    assert abs(za[1] - zs[1]) <= 1e-13 * za[1]
    np.testing.assert_allclose(zs[2], za[2], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# BHHH (outer product of the events' scores) and the damped BHHH minimiser
# ---------------------------------------------------------------------------

def _fd_scores(o, cols, th, h_rel=1e-6):
    """Per-event scores d log p(x_i) / d theta by central differences of the
    per-event log-density value alone (its analytic derivative unused)."""
    n, P = len(cols[0]), len(th)
    S = np.zeros((n, P))
    for k in range(P):
        h = h_rel * max(1.0, abs(th[k]))
        tp, tm = np.array(th, dtype=float), np.array(th, dtype=float)
        tp[k] += h
        tm[k] -= h
        for i in range(n):
            x = [c[i] for c in cols]
            S[i, k] = (o.log_density(x, tp)[1] - o.log_density(x, tm)[1]) / (2 * h)
    return S


@pytest.mark.parametrize("config", [1, 2, 3])
def test_bhhh_matrix_is_outer_product_of_fd_scores(config):
    """B = sum_i s_i s_i^T with s_i from finite differences of log p(x_i);
    symmetric, positive semi-definite."""
    w = datagen.workload(config, n=300)
    o = oracle.Oracle(w["spec"])
    th = w["points"][1]
    st, nll, g, B = o.nll_bhhh(w["cols"], th)
    assert st == OK
    S = _fd_scores(o, w["cols"], th)
    free = np.array([p.get("free", True) for p in w["spec"]["params"]], dtype=float)
    ref = (S.T @ S) * np.outer(free, free)  # fixed parameters: zero rows and columns
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(B - ref)) <= 1e-6 * scale, (B, ref)
    assert np.array_equal(B, B.T)
    assert np.min(np.linalg.eigvalsh(B)) >= -1e-12 * scale
    # the gradient is minus the sum of the same scores
    assert np.max(np.abs(g + free * S.sum(axis=0))) <= 1e-6 * max(1.0, np.max(np.abs(S).sum(axis=0)))


def test_bhhh_matrix_approaches_fisher_information():
    """For a Gaussian on a range of +-6.7 sigma, B / N at the truth tends to
    the Fisher information diag(1/sigma^2, 2/sigma^2) with 1/sqrt(N)
    fluctuations."""
    w = datagen.workload(1)
    o = oracle.Oracle(w["spec"])
    st, nll, g, B = o.nll_bhhh(w["cols"], w["theta"])
    n, s = len(w["cols"][0]), w["theta"][1]
    I = np.array([[1 / s**2, 0.0], [0.0, 2 / s**2]])
    assert np.max(np.abs(B / n - I)) <= 6 * np.sqrt(2.0 / n) * np.max(I)


def test_bhhh_extended_and_fixed_parameters():
    """The Poisson term adds N / nu^2 at (nu, nu); a fixed parameter's row
    and column are 0."""
    spec = datagen.mixture_spec()
    spec["params"].append(datagen.param("nu", 1000.0, 1.0, 1e7))
    spec["extended"] = True
    spec["yield_param"] = 4
    cols = datagen.generate(datagen.mixture_spec(), 400, seed=8)
    th = np.array([0.2, 5.0, 0.4, -0.7, 800.0])
    st, nll, g, B = oracle.Oracle(spec).nll_bhhh(cols, th)
    st4, nll4, g4, B4 = oracle.Oracle(datagen.mixture_spec()).nll_bhhh(cols, th[:4])
    assert np.array_equal(B[:4, :4], B4) and np.all(B[4, :4] == 0.0)
    assert B[4, 4] == 400 / 800.0**2
    spec2 = datagen.mixture_spec()
    spec2["params"][3]["free"] = False
    st, nll, g, B2 = oracle.Oracle(spec2).nll_bhhh(cols, th[:4])
    assert np.all(B2[3] == 0.0) and np.all(B2[:, 3] == 0.0)
    assert np.array_equal(B2[:3, :3], B4[:3, :3])


def test_bhhh_fit_reaches_closed_form_mle_in_few_steps():
    """Damped BHHH on the wide-range Gaussian lands on the MLE mu =
    mean(x), sigma^2 = mean((x - mean)^2) in far fewer steps than gradient
    descent (which needs ~50 here), with a monotone NLL."""
    w = datagen.workload(1)
    x = w["cols"][0].astype(np.longdouble)
    mu_hat = float(x.mean())
    s_hat = float(np.sqrt(((x - x.mean()) ** 2).mean()))
    st, th, nll, g, lam, tr = oracle.Oracle(w["spec"]).bhhh_fit(w["cols"], w["points"][0], 12, 1e-3, trace=True)
    assert st == OK
    assert abs(th[0] - mu_hat) <= 1e-8 * abs(mu_hat)
    assert abs(th[1] - s_hat) <= 1e-8 * s_hat
    acc = np.minimum.accumulate(tr[:, 0])
    assert np.all(np.diff(acc) <= 0.0)
    assert np.max(np.abs(g)) / len(x) < 1e-9


def test_bhhh_fit_mixture_converges_to_stationary_point():
    """On the signal+background mixture BHHH reaches a point whose gradient
    vanishes (relative to the per-event score scale), and the NLL there is
    no higher than gradient descent's after many more steps."""
    w = datagen.workload(2, n=20_000)
    o = oracle.Oracle(w["spec"])
    st, th, nll, g, lam = o.bhhh_fit(w["cols"], w["points"][0], 25, 1e-3, threads=4)
    assert st == OK
    st2, th2, nll2, g2, eta2 = o.gd_fit(w["cols"], w["points"][0], 400, 1.0, threads=4)
    _, _, _, stats = o.nll(w["cols"], th, stats=True)
    assert np.max(np.abs(g) / stats[1:]) < 1e-8
    assert nll <= nll2 + 1e-9 * abs(nll2)


# ---------------------------------------------------------------------------
# Johnson S_U (Sec. 3)
# ---------------------------------------------------------------------------

def test_johnson_large_delta_is_gaussian():
    """gamma = 0, lambda = delta sigma: as delta grows the S_U density tends
    to the Gaussian(mu, sigma) (asinh z -> z, sqrt(1 + z^2) -> 1), with
    log-density corrections (t^4/6 - t^2/2) / delta^2 to leading order,
    t = (x - mu)/sigma (from asinh z = z - z^3/6 and ln(1 + z^2) = z^2), plus
    a shift of the normalisation of the same order."""
    mu, sg, lo, hi = 0.3, 1.5, -6.0, 7.0
    for de in (1e3, 1e5):
        params = (mu, de * sg, 0.0, de)
        spec = single_leaf_spec("johnson", params, lo, hi)
        for p in spec["params"]:
            p["lo"], p["hi"] = -1e9, 1e9
        o = oracle.Oracle(spec)
        xs = np.linspace(lo, hi, 27)
        res = [o.log_density([x], params) for x in xs]
        assert all(r[0] == OK for r in res)
        got = np.array([r[1] for r in res])
        ref = lib_logpdf("gauss", (mu, sg), lo, hi, xs)
        t = (xs - mu) / sg
        bound = (1.2 * (t ** 4 / 6 + t ** 2 / 2) + 2.0) / de ** 2 + 1e-12
        assert np.all(np.abs(got - ref) <= bound), (de, np.abs(got - ref) / bound)


def test_johnson_mixture_nll_matches_library_brute_force():
    spec = datagen.johnson_spec()
    theta = datagen.theta_of(spec)
    cols = datagen.generate(spec, 16, seed=5)
    cols[0][:4] = [5.0, 5.6, 5.28, 5.2801]
    lo, hi = spec["obs"][0]["lo"], spec["obs"][0]["hi"]
    f = theta[0]
    o = oracle.Oracle(spec)
    for n in (1, 2, 3, 16):
        x = cols[0][:n]
        p = f * np.exp(lib_logpdf("johnson", theta[1:5], lo, hi, x)) + (1 - f) * np.exp(lib_logpdf("exp", theta[5:6], lo, hi, x))
        ref = -math.fsum(np.log(p))
        st, nll, _ = o.nll([x], theta)
        assert st == OK
        assert abs(nll - ref) <= 2e-13 * max(1.0, abs(ref)), (n, nll, ref)


@pytest.mark.parametrize("single", [False, True])
def test_johnson_gradient_matches_central_differences(single):
    w = datagen.johnson_workload(4000, single=single, n_points=3)
    o = oracle.Oracle(w["spec"])
    th = w["points"][2]
    st, nll, g = o.nll(w["cols"], th)
    assert st == OK
    widths = datagen.jitter_widths(w["spec"])
    for k in range(len(th)):
        h = 1e-3 * widths[k]

        def f(v):
            t = th.copy()
            t[k] = v
            return o.nll(w["cols"], t)[1]

        fd = (f(th[k] - 2 * h) - 8 * f(th[k] - h) + 8 * f(th[k] + h) - f(th[k] + 2 * h)) / (12 * h)
        bound = 50 * (2.2e-16 * abs(nll) / h) + 1e-6 * abs(g[k])
        assert abs(fd - g[k]) <= bound, (k, fd, g[k], bound)


def test_johnson_parameter_checks():
    spec = single_leaf_spec("johnson", (0.0, 1.0, 0.0, 1.0), -5.0, 5.0)
    o = oracle.Oracle(spec)
    for bad in ((0.0, 0.0, 0.0, 1.0), (0.0, -1.0, 0.0, 1.0), (0.0, 1.0, 0.0, 0.0), (0.0, 1.0, 0.0, -2.0)):
        assert o.log_density([0.1], bad)[0] == E_PARAM
    assert o.log_density([0.1], (0.0, 1.0, 0.0, 1.0))[0] == OK


# ---------------------------------------------------------------------------
# chi-square (the ChiSquarePdf of Sec. 5.2's speed-up figure)
# ---------------------------------------------------------------------------

def test_chi2_two_dof_is_exponential():
    """nu = 2: x^0 e^{-x/2}, the exponential with c = -1/2 (library truncexpon)."""
    lo, hi = 0.0, 9.0
    o = oracle.Oracle(single_leaf_spec("chi2", (2.0,), lo, hi))
    xs = np.linspace(lo, hi, 19)
    got = np.array([o.log_density([x], (2.0,))[1] for x in xs])
    np.testing.assert_allclose(got, lib_logpdf("exp", (-0.5,), lo, hi, xs), rtol=0, atol=1e-13)


@pytest.mark.parametrize("nu", [0.7, 2.0, 5.0, 17.3, 120.0])
def test_chi2_norm_is_scaled_lower_incomplete_gamma(nu):
    """Z over [0, hi] = 2^{nu/2} Gamma(nu/2) P(nu/2, hi/2) with scipy's
    regularised gamma P; dZ/dnu against a fourth-order central difference."""
    from scipy import special
    for hi in (0.3, 4.0, 40.0, 400.0):
        o = oracle.Oracle(single_leaf_spec("chi2", (nu,), 0.0, hi))
        st, Z, dZ = o.leaf_norm(0, (nu,))
        assert st == OK
        k = nu / 2
        ref = math.exp(k * math.log(2.0) + special.gammaln(k)) * special.gammainc(k, hi / 2)
        assert abs(Z - ref) <= 1e-13 * ref, (nu, hi, Z, ref)
        h = 1e-3 * min(nu, 1.0)
        z = lambda v: o.leaf_norm(0, (v,))[1]
        fd = (z(nu - 2 * h) - 8 * z(nu - h) + 8 * z(nu + h) - z(nu + 2 * h)) / (12 * h)
        assert abs(fd - dZ[0]) <= 1e-8 * max(abs(dZ[0]), Z), (nu, hi, fd, dZ)


def test_chi2_range_checks():
    """Observable ranges below 0 or beyond 1000 are not supported; nu <= 0 is
    outside the density's parameter domain."""
    for lo, hi in ((-1.0, 5.0), (0.0, 1000.5)):
        with pytest.raises(ValueError):
            oracle.Oracle(single_leaf_spec("chi2", (3.0,), lo, hi))
    o = oracle.Oracle(single_leaf_spec("chi2", (3.0,), 0.0, 5.0))
    assert o.log_density([1.0], (0.0,))[0] == E_PARAM
    assert o.log_density([1.0], (-1.0,))[0] == E_PARAM


def test_chi2_gradient_matches_central_differences():
    w = datagen.chi2_workload(5000, n_points=2)
    o = oracle.Oracle(w["spec"])
    th = w["points"][1]
    st, nll, g = o.nll(w["cols"], th)
    assert st == OK
    h = 1e-4
    f = lambda v: o.nll(w["cols"], np.array([v]))[1]
    fd = (f(th[0] - 2 * h) - 8 * f(th[0] - h) + 8 * f(th[0] + h) - f(th[0] + 2 * h)) / (12 * h)
    assert abs(fd - g[0]) <= 50 * 2.2e-16 * abs(nll) / h + 1e-7 * abs(g[0]), (fd, g)


# ---------------------------------------------------------------------------
# weighted events (binned datasets, sWeights)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("config", [1, 2, 3])
def test_integer_weights_equal_repeated_events(config):
    """Weights 0..4: the weighted NLL and gradient equal those of the dataset
    with every event repeated w_i times (also with an extended yield term)."""
    w = datagen.workload(config, n=3000)
    spec, th = w["spec"], w["points"][1]
    wt = np.floor(5 * datagen.uniforms(7, 3, 3000))
    rep = [np.repeat(c, wt.astype(np.int64)) for c in w["cols"]]
    o = oracle.Oracle(spec)
    st, v, g, s = o.nll(w["cols"], th, weights=wt, stats=True)
    st2, v2, g2, s2 = o.nll(rep, th, stats=True)
    assert st == OK and st2 == OK
    assert abs(v - v2) <= 1e-13 * abs(v2)
    np.testing.assert_allclose(g, g2, rtol=0, atol=1e-12 * max(np.abs(g2).max(), s2[1:].max()))
    ext = dict(spec)
    ext["params"] = list(spec["params"]) + [datagen.param("nu", 1000.0, 1.0, 1e7)]
    ext["extended"] = True
    ext["yield_param"] = len(ext["params"]) - 1
    the = np.append(th, 2100.0)
    oe = oracle.Oracle(ext)
    _, ve, ge = oe.nll(w["cols"], the, weights=wt)
    _, ve2, ge2 = oe.nll(rep, the)
    assert abs(ve - ve2) <= 1e-13 * abs(ve2)
    assert abs(ge[-1] - (1 - wt.sum() / 2100.0)) <= 1e-14 and abs(ge[-1] - ge2[-1]) <= 1e-14


def test_weighted_nll_matches_library():
    """-fsum(w_i log p(x_i)) from library densities, signed weights."""
    for config in (1, 2, 3):
        w = datagen.workload(config, n=16)
        wt = datagen.signed_weights(16, seed=config)
        ref = -math.fsum(wt * lib_model_logpdf(w["spec"], w["cols"], w["theta"]))
        st, v, _ = oracle.Oracle(w["spec"]).nll(w["cols"], w["theta"], weights=wt)
        assert st == OK and abs(v - ref) <= 2e-13 * max(1.0, abs(ref)), (config, v, ref)


def test_binned_gauss_fit_reaches_weighted_mle():
    """A binned fit (bin centres weighted by counts) of the wide-range
    Gaussian lands on the weighted-moment MLE mu = sum w x / W,
    sigma^2 = sum w (x - mu)^2 / W."""
    w = datagen.workload(1)
    xc, cnt = datagen.binned(w["cols"][0], -10.0, 10.0, 400)
    x = xc.astype(np.longdouble)
    W = cnt.astype(np.longdouble).sum()
    mu_hat = float((cnt * x).sum() / W)
    s_hat = float(np.sqrt((cnt * (x - mu_hat) ** 2).sum() / W))
    st, th, nll, g, eta = oracle.Oracle(w["spec"]).gd_fit([xc], w["theta"], 50, 1.0, weights=cnt)
    assert st == OK
    assert abs(th[0] - mu_hat) <= 1e-8 * abs(mu_hat)
    assert abs(th[1] - s_hat) <= 1e-8 * s_hat


# ---------------------------------------------------------------------------
# Sums of yields (extended models with one yield per component)
# ---------------------------------------------------------------------------

def yields_spec(extended=True):
    """nu_1 Gauss(2, 0.3) + nu_2 Gauss(7, 0.5) + nu_3 Exp(-0.2) on [0, 10],
    shapes fixed, yields free: p = sum nu_j p_j / sum nu_j."""
    P = datagen.param
    return {"obs": [{"name": "x", "lo": 0.0, "hi": 10.0}],
            "params": [P("n1", 300.0, 0.0, 1e7), P("n2", 500.0, 0.0, 1e7), P("n3", 1200.0, 0.0, 1e7),
                       P("mu1", 2.0, 0.0, 10.0, free=False), P("s1", 0.3, 0.01, 5.0, free=False),
                       P("mu2", 7.0, 0.0, 10.0, free=False), P("s2", 0.5, 0.01, 5.0, free=False),
                       P("c", -0.2, -5.0, 5.0, free=False)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [3, 4]}, {"kind": "gauss", "obs": 0, "params": [5, 6]},
                      {"kind": "exp", "obs": 0, "params": [7]},
                      {"kind": "sum", "params": [0, 1, 2], "children": [0, 1, 2]}],
            "root": 3, "extended": extended, "yield_param": -1}


def test_yields_nll_matches_library():
    """Extended NLL with yields = sum nu - sum_i log(sum_j nu_j p_j(x_i))
    (the Poisson term nu - N ln nu plus -sum log p), every p_j a scipy
    truncated density."""
    spec = yields_spec()
    th = np.array([310.0, 480.0, 1250.0, 2.0, 0.3, 7.0, 0.5, -0.2])
    x = datagen.generate(spec, 2000, seed=41)[0]
    dens = (th[0] * np.exp(lib_logpdf("gauss", (2.0, 0.3), 0.0, 10.0, x))
            + th[1] * np.exp(lib_logpdf("gauss", (7.0, 0.5), 0.0, 10.0, x))
            + th[2] * np.exp(lib_logpdf("exp", (-0.2,), 0.0, 10.0, x)))
    ref = math.fsum(th[:3]) - math.fsum(np.log(dens))
    st, v, g = oracle.Oracle(spec).nll([x], th)
    assert st == OK
    assert abs(v - ref) <= 1e-12 * abs(ref)
    # without the Poisson term: the normalised mixture with fractions nu_j / sum nu
    st, v0, g0 = oracle.Oracle(yields_spec(extended=False)).nll([x], th)
    ref0 = -math.fsum(np.log(dens / math.fsum(th[:3])))
    assert abs(v0 - ref0) <= 1e-12 * abs(ref0)


def test_yields_gradient_vanishes_at_the_counts_of_separated_components():
    """Components with (numerically) disjoint support: at nu_j = n_j (the
    number of events drawn from component j) the extended NLL is stationary,
    and d NLL / d nu_j = 1 - n_j / nu_j elsewhere (closed forms)."""
    P = datagen.param
    spec = {"obs": [{"name": "x", "lo": 0.0, "hi": 10.0}],
            "params": [P("n1", 400.0, 0.0, 1e7), P("n2", 600.0, 0.0, 1e7), P("mu1", 2.0, 0.0, 10.0),
                       P("s1", 0.1, 0.01, 5.0), P("mu2", 8.0, 0.0, 10.0), P("s2", 0.1, 0.01, 5.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [2, 3]}, {"kind": "gauss", "obs": 0, "params": [4, 5]},
                      {"kind": "sum", "params": [0, 1], "children": [0, 1]}],
            "root": 2, "extended": True, "yield_param": -1}
    x = datagen.generate(spec, 1000, seed=42)[0]
    n1, n2 = int(np.sum(x < 5.0)), int(np.sum(x >= 5.0))
    o = oracle.Oracle(spec)
    st, v, g = o.nll([x], np.array([n1, n2, 2.0, 0.1, 8.0, 0.1]))
    assert st == OK and abs(g[0]) < 1e-12 and abs(g[1]) < 1e-12
    st, v2, g2 = o.nll([x], np.array([n1 + 40.0, n2 - 25.0, 2.0, 0.1, 8.0, 0.1]))
    assert abs(g2[0] - (1.0 - n1 / (n1 + 40.0))) < 1e-12
    assert abs(g2[1] - (1.0 - n2 / (n2 - 25.0))) < 1e-12
    assert v2 > v


def test_yields_equal_fractions_plus_poisson_term():
    """The sum of yields equals the fraction form with f_j = nu_j / sum nu
    (a different path through the oracle) plus nu - N ln nu."""
    spec = yields_spec()
    th = np.array([310.0, 480.0, 1250.0, 2.0, 0.3, 7.0, 0.5, -0.2])
    x = datagen.generate(spec, 3000, seed=43)[0]
    P = datagen.param
    frac = {"obs": spec["obs"],
            "params": [P("f1", 0.1, 0.0, 1.0), P("f2", 0.1, 0.0, 1.0)] + spec["params"][3:],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [2, 3]}, {"kind": "gauss", "obs": 0, "params": [4, 5]},
                      {"kind": "exp", "obs": 0, "params": [6]},
                      {"kind": "sum", "params": [0, 1], "children": [0, 1, 2]}],
            "root": 3}
    S = th[:3].sum()
    thf = np.concatenate([[th[0] / S, th[1] / S], th[3:]])
    vf = oracle.Oracle(frac).nll([x], thf)[1]
    v = oracle.Oracle(spec).nll([x], th)[1]
    assert abs(v - (vf + S - 3000 * math.log(S))) <= 1e-12 * abs(v)


def test_yields_gradient_matches_central_differences():
    spec = yields_spec()
    for p in spec["params"]:
        p["free"] = True
    th = np.array([310.0, 480.0, 1250.0, 2.1, 0.28, 6.9, 0.55, -0.25])
    x = datagen.generate(spec, 3000, seed=44)[0]
    o = oracle.Oracle(spec)
    st, nll, g = o.nll([x], th)
    for k in range(len(th)):
        h = 1e-4 * max(abs(th[k]), 0.1)

        def f(v):
            t = th.copy()
            t[k] = v
            return o.nll([x], t)[1]

        fd = (f(th[k] - 2 * h) - 8 * f(th[k] - h) + 8 * f(th[k] + h) - f(th[k] + 2 * h)) / (12 * h)
        bound = 50 * (2.2e-16 * abs(nll) / h) + 1e-6 * abs(g[k])
        assert abs(fd - g[k]) <= bound, (k, fd, g[k], bound)


def test_yields_checks_and_product_root():
    """Negative yields or a zero total are out of range; a product whose one
    child is a sum of yields takes that sum's total as the expected count."""
    spec = yields_spec()
    o = oracle.Oracle(spec)
    x = datagen.generate(spec, 500, seed=45)[0]
    th = np.array([310.0, 480.0, 1250.0, 2.0, 0.3, 7.0, 0.5, -0.2])
    bad = th.copy()
    bad[1] = -1.0
    assert o.nll([x], bad)[0] == E_PARAM
    zero = th.copy()
    zero[:3] = 0.0
    assert o.nll([x], zero)[0] == E_PARAM
    P = datagen.param
    prod = {"obs": [{"name": "x", "lo": 0.0, "hi": 10.0}, {"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": spec["params"] + [P("a1", 0.0, -1.0, 1.0)],
            "nodes": spec["nodes"] + [{"kind": "cheb", "obs": 1, "params": [8]},
                                      {"kind": "prod", "children": [3, 4]}],
            "root": 5, "extended": True, "yield_param": -1}
    y = np.linspace(-1.0, 1.0, 500)
    st, v, g = oracle.Oracle(prod).nll([x, y], np.concatenate([th, [0.0]]))
    v1 = o.nll([x], th)[1]
    assert st == OK and abs(v - (v1 + 500 * math.log(2.0))) <= 1e-12 * abs(v)


# ---------------------------------------------------------------------------
# Hypatia2 (generalised hyperbolic core, power-law tails on both sides)
# ---------------------------------------------------------------------------

HYP_NAMES = ["mu", "sigma", "lambda", "zeta", "beta", "a_l", "n_l", "a_r", "n_r"]
HYP_CASES = [([5.28, 0.003, -2.0, 0.5, 0.0, 2.0, 3.0, 2.5, 4.0], 5.20, 5.35),
             ([0.0, 1.0, -1.2, 0.05, 0.1, 1.5, 2.0, 1.8, 6.0], -8.0, 8.0),
             ([1.0, 0.5, 1.0, 2.0, -0.2, 2.5, 1.5, 3.0, 3.0], -3.0, 5.0),
             ([0.0, 1.0, 3.0, 20.0, 0.0, 3.0, 5.0, 3.0, 5.0], -6.0, 6.0)]


def hypatia_spec(th, lo, hi):
    return {"obs": [{"name": "m", "lo": lo, "hi": hi}],
            "params": [datagen.param(n, v, -1e3, 1e3) for n, v in zip(HYP_NAMES, th)],
            "nodes": [{"kind": "hypatia", "obs": 0, "params": list(range(9)), "norm": "gl256"}], "root": 0}


def test_log_bessel_k_against_mpmath():
    """The oracle's K_nu(z) (trapezoidal rule on its integral over cosh)
    against mpmath's besselk at 30 digits, orders -3.3..4.2, z 1e-3..700."""
    import mpmath as mp
    mp.mp.dps = 30
    for nu in (-3.3, -1.7, -0.5, 0.0, 0.3, 0.5, 1.0, 2.5, 4.2):
        for z in (1e-3, 0.05, 0.3, 1.0, 3.0, 10.0, 50.0, 300.0, 700.0):
            ref = float(mp.log(mp.besselk(nu, z)))
            assert abs(oracle.log_bessel_k(nu, z) - ref) <= 2e-15 * max(1.0, abs(ref)), (nu, z)


def test_hypatia_density_against_mpmath():
    """log p of the oracle against the same definition written with mpmath
    (besselk, numerical slope at the junctions, tanh-sinh quadrature for Z)
    at 30 digits, over the core, both tails and the range ends."""
    import mpmath as mp
    mp.mp.dps = 30
    for th, lo, hi in HYP_CASES:
        mu, sg, la, ze, be, al, nl, ar, nr = [mp.mpf(v) for v in th]
        nu = la - mp.mpf(1) / 2
        d2 = ze * mp.besselk(la, ze) / mp.besselk(la + 1, ze) * sg * sg
        alpha = ze / mp.sqrt(d2)

        def lG(d):
            r2 = d * d + d2
            return nu / 2 * mp.log(r2) + be * d + mp.log(mp.besselk(nu, alpha * mp.sqrt(r2)))
        dl, dh = -al * sg, ar * sg
        Gl, sl, Gh, sh = lG(dl), mp.diff(lG, dl), lG(dh), mp.diff(lG, dh)

        def lg(d):
            if d < dl:
                return Gl - nl * mp.log(1 + sl * (dl - d) / nl)
            if d > dh:
                return Gh - nr * mp.log(1 - sh * (d - dh) / nr)
            return lG(d)
        cuts = [lo] + [p for p in (mu + dl, mu, mu + dh) if lo < p < hi] + [hi]
        logZ = mp.log(mp.quad(lambda x: mp.exp(lg(x - mu) - Gl), cuts)) + Gl
        o = oracle.Oracle(hypatia_spec(th, lo, hi))
        for x in np.linspace(lo, hi, 13):
            ref = float(lg(mp.mpf(x) - mu) - logZ)
            st, lp, _ = o.log_density([x], np.array(th))
            assert st == OK and abs(lp - ref) <= 4e-15 * max(1.0, abs(ref)), (th, x, lp, ref)


def test_hypatia_lambda_one_is_hyperbolic():
    """lambda = 1 gives K_{1/2}(z) = sqrt(pi / 2z) e^{-z}: the core is the
    hyperbolic density, log G = beta d - alpha sqrt(d^2 + delta^2) + const;
    alpha and delta from scipy's kv (only in A^2 = zeta K_1 / K_2)."""
    from scipy.special import kv
    th = [0.4, 0.8, 1.0, 1.3, 0.15, 2.5, 3.0, 2.0, 4.0]
    mu, sg, la, ze, be = th[:5]
    delta = np.sqrt(ze * kv(la, ze) / kv(la + 1.0, ze)) * sg
    alpha = ze / delta
    o = oracle.Oracle(hypatia_spec(th, -5.0, 5.0))
    xs = np.linspace(mu - 1.9 * sg, mu + 1.5 * sg, 9)
    lp = np.array([o.log_density([x], np.array(th))[1] for x in xs])
    d = xs - mu
    ref = be * d - alpha * np.sqrt(d * d + delta * delta)
    np.testing.assert_allclose(lp - lp[0], ref - ref[0], rtol=0, atol=2e-14)


def test_hypatia_tails_continue_value_and_slope():
    """At both junctions the tails continue the core with equal value and
    slope (one-sided differences of log p on either side)."""
    for th, lo, hi in HYP_CASES:
        o = oracle.Oracle(hypatia_spec(th, lo, hi))
        mu, sg = th[0], th[1]
        for xj in (mu - th[5] * sg, mu + th[7] * sg):
            if not (lo < xj < hi):
                continue
            h = 1e-5 * sg
            f = lambda x: o.log_density([x], np.array(th))[1]
            left = (f(xj) - f(xj - h)) / h
            right = (f(xj + h) - f(xj)) / h
            assert abs(f(xj - 1e-12 * sg) - f(xj + 1e-12 * sg)) < 1e-9
            assert abs(left - right) <= 1e-4 * max(1.0, abs(left)), (th, xj, left, right)


def test_hypatia_gradient_matches_central_differences():
    """d NLL / d theta (complex steps through the Bessel integral, the
    junctions, the tails and the normalisation) against fourth-order central
    differences of the oracle's NLL, all nine parameters free."""
    th, lo, hi = HYP_CASES[1]
    spec = hypatia_spec(th, lo, hi)
    rng = np.random.default_rng(51)
    x = np.clip(rng.standard_t(3, 2000) * 1.2 + 0.1, lo, hi)
    o = oracle.Oracle(spec)
    st, nll, g = o.nll([x], np.array(th))
    assert st == OK
    for k in range(9):
        h = 1e-4 * max(abs(th[k]), 0.05)

        def f(v):
            t = np.array(th, dtype=float)
            t[k] = v
            return o.nll([x], t)[1]

        fd = (f(th[k] - 2 * h) - 8 * f(th[k] - h) + 8 * f(th[k] + h) - f(th[k] + 2 * h)) / (12 * h)
        bound = 50 * (2.2e-16 * abs(nll) / h) + 1e-6 * abs(g[k])
        assert abs(fd - g[k]) <= bound, (HYP_NAMES[k], fd, g[k], bound)


def test_hypatia_parameter_checks():
    """sigma, zeta, a_l, a_r > 0 and n_l, n_r > 1; a tail whose junction
    slope does not fall away from the core (a strong skew beta) is out of
    range."""
    th, lo, hi = HYP_CASES[1]
    o = oracle.Oracle(hypatia_spec(th, lo, hi))
    x = np.linspace(lo, hi, 50)
    assert o.nll([x], np.array(th))[0] == OK
    for k, v in ((1, 0.0), (3, 0.0), (5, -1.0), (6, 1.0), (7, 0.0), (8, 0.5), (4, 5.0)):
        t = np.array(th, dtype=float)
        t[k] = v
        assert o.nll([x], t)[0] == E_PARAM, (HYP_NAMES[k], v)

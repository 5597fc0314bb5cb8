"""Pins of the binned (HistFactory-type) oracle against things other than
itself: scipy's Poisson log-probability, the fixed points of the
interpolation codes (templates reproduced at alpha = +-1, linear / power
behaviour in between), the closed-form maximum of a one-sample fit, finite
differences, and the constraint and status conventions."""
import copy
import math

import numpy as np
import pytest
from scipy import special, stats

import datagen
from oracle import histfactory as hf


@pytest.fixture(scope="module")
def small():
    return datagen.hf_workload(n_bins=1000, n_samples=3, n_histosys=5, n_normsys=3, n_points=3)


def args(w):
    return w["spec"], w["counts"], w["nominal"], w["up"], w["down"]


def test_poisson_terms_match_scipy(small):
    spec, n, T, up, dn = args(small)
    for th in small["points"]:
        st, v, _ = hf.nll(spec, n, T, up, dn, th, grad=False)
        assert st == hf.OK
        nu, _ = hf.expected(spec, T, up, dn, th)
        cons = 0.5 * sum(th[p] ** 2 for p, par in enumerate(spec["params"]) if par["constrained"])
        ref = -math.fsum(stats.poisson.logpmf(n, nu)) - math.fsum(special.gammaln(n + 1)) + cons
        assert abs(v - ref) <= 1e-12 * abs(ref), (v, ref)


def test_interpolation_fixed_points(small):
    """One modifier moved at a time from the nominal point: histosys at
    alpha = +1 / -1 replaces its sample's nominal by the up / down template,
    and is linear on each side; normsys scales its sample by hi at +1, lo at
    -1 and by hi^(1/2) at +1/2."""
    spec, n, T, up, dn = args(small)
    th0 = datagen.theta_of(spec)
    nu0, _ = hf.expected(spec, T, up, dn, th0)
    h = 0
    for m in spec["modifiers"]:
        if m["type"] == "histosys":
            s, p = m["sample"], m["param"]
            for a, ref in ((1.0, up[h] - T[s]), (-1.0, dn[h] - T[s]), (0.37, 0.37 * (up[h] - T[s])),
                           (-0.6, 0.6 * (dn[h] - T[s]))):
                th = th0.copy()
                th[p] = a
                nu, _ = hf.expected(spec, T, up, dn, th)
                np.testing.assert_allclose(nu - nu0, ref, rtol=1e-12, atol=1e-12 * np.abs(nu0).max())
            h += 1
        elif m["type"] == "normsys":
            s, p = m["sample"], m["param"]
            for a, f in ((1.0, m["hi"]), (-1.0, m["lo"]), (0.5, math.sqrt(m["hi"]))):
                th = th0.copy()
                th[p] = a
                nu, _ = hf.expected(spec, T, up, dn, th)
                np.testing.assert_allclose(nu - nu0, (f - 1.0) * T[s], rtol=1e-12, atol=1e-12 * np.abs(nu0).max())


def test_one_sample_normfactor_maximum():
    """One sample scaled by mu: the maximum is mu = sum n / sum T."""
    w = datagen.hf_workload(n_bins=5000, n_samples=1, n_histosys=0, n_normsys=0)
    spec = {"n_bins": 5000, "samples": ["s0"], "params": [w["spec"]["params"][0]],
            "modifiers": [{"type": "normfactor", "sample": 0, "param": 0}]}
    n, T = w["counts"], w["nominal"]
    mu = math.fsum(n) / math.fsum(T[0])
    st, v, g = hf.nll(spec, n, T, [], [], [mu])
    assert st == hf.OK and abs(g[0]) <= 1e-9 * math.fsum(n) / mu
    for d in (1e-3, -1e-3):
        assert hf.nll(spec, n, T, [], [], [mu * (1 + d)], grad=False)[1] > v


def test_gradient_matches_central_differences(small):
    spec, n, T, up, dn = args(small)
    for th in small["points"]:
        st, v, g = hf.nll(spec, n, T, up, dn, th)
        assert st == hf.OK
        for p in range(len(th)):
            h = 1e-5

            def f(x):
                t = th.copy()
                t[p] = x
                return hf.nll(spec, n, T, up, dn, t, grad=False)[1]

            fd = (f(th[p] - 2 * h) - 8 * f(th[p] - h) + 8 * f(th[p] + h) - f(th[p] + 2 * h)) / (12 * h)
            assert abs(fd - g[p]) <= 50 * 2.2e-16 * abs(v) / h + 1e-7 * abs(g[p]), (p, fd, g[p])


def test_constraint_term_and_status(small):
    spec, n, T, up, dn = args(small)
    th = small["points"][0]
    free = copy.deepcopy(spec)
    for par in free["params"]:
        par["constrained"] = False
    v1 = hf.nll(spec, n, T, up, dn, th, grad=False)[1]
    v0 = hf.nll(free, n, T, up, dn, th, grad=False)[1]
    cons = 0.5 * sum(th[p] ** 2 for p, par in enumerate(spec["params"]) if par["constrained"])
    assert abs((v1 - v0) - cons) <= 1e-9 * abs(v1)
    bad = th.copy()
    bad[2] = 6.0
    assert hf.nll(spec, n, T, up, dn, bad)[0] == hf.E_PARAM
    one = {"n_bins": 1000, "samples": ["s0"], "params": [spec["params"][0]],
           "modifiers": [{"type": "normfactor", "sample": 0, "param": 0}]}
    assert hf.nll(one, n, T[:1], [], [], [0.0])[0] == hf.E_PDF


# ---------------------------------------------------------------------------
# per-bin statistical parameters (gamma_b of the flagged samples)
# ---------------------------------------------------------------------------

def _stat(n_bins, seed=5):
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(0.01, 0.1, n_bins)
    sigma[::7] = 0.0          # bins without a statistical parameter
    sigma[3::11] = np.inf     # not finite: none either
    gamma = 1.0 + rng.uniform(-0.05, 0.05, n_bins)
    return sigma, gamma


def test_stat_gamma_one_is_the_plain_model(small):
    """gamma = 1 everywhere: the plain NLL and gradient (no constraint
    contribution), and d NLL / d gamma_b = w_b times the flagged samples'
    part of nu_b."""
    spec, n, T, up, dn = args(small)
    sigma, _ = _stat(len(n))
    mask = 0b101
    th = small["points"][0]
    st0, v0, g0 = hf.nll(spec, n, T, up, dn, th)
    st, v, g, gg = hf.nll(spec, n, T, up, dn, th, stat=(mask, sigma, np.ones(len(n))))
    assert st == st0 == hf.OK
    assert v == v0 and np.array_equal(g, g0)
    nu, _ = hf.expected(spec, T, up, dn, th)
    # the flagged samples' part: switch the others off with a zero normfactor-free copy of the model
    spec_f = copy.deepcopy(spec)
    nu_f = np.zeros(len(n))
    for s in range(len(spec["samples"])):
        if (mask >> s) & 1:
            Ts = [T[k] if k == s else np.zeros(len(n)) for k in range(len(T))]
            ups = [u if m["sample"] == s else np.zeros(len(n)) for u, m in zip(up, hf.histosys_list(spec))]
            dns = [d if m["sample"] == s else np.zeros(len(n)) for d, m in zip(dn, hf.histosys_list(spec))]
            nu_f += hf.expected(spec_f, Ts, ups, dns, th)[0]
    w = np.where(n > 0, 1.0 - n / nu, 1.0)
    active = (sigma > 0) & np.isfinite(sigma)
    np.testing.assert_allclose(gg[active], (w * nu_f)[active], rtol=1e-12, atol=1e-12 * np.abs(nu_f).max())
    assert np.all(gg[~active] == 0.0)


def test_stat_poisson_terms_and_constraint_match_scipy():
    """One flagged sample scaled by a normfactor: nu_b = mu gamma_b T_b by
    hand, the NLL against scipy's Poisson log-probability plus the Gaussian
    constraints (gamma_b - 1)^2 / (2 sigma_b^2) of the bins that have one."""
    w = datagen.hf_workload(n_bins=2000, n_samples=1, n_histosys=0, n_normsys=0)
    spec = {"n_bins": 2000, "samples": ["s0"], "params": [w["spec"]["params"][0]],
            "modifiers": [{"type": "normfactor", "sample": 0, "param": 0}]}
    n, T = w["counts"], w["nominal"]
    sigma, gamma = _stat(2000, seed=9)
    mu = 1.07
    st, v, g, gg = hf.nll(spec, n, T, [], [], [mu], stat=(1, sigma, gamma))
    active = (sigma > 0) & np.isfinite(sigma)
    nu = mu * np.where(active, gamma, 1.0) * T[0]
    ref = (-math.fsum(stats.poisson.logpmf(n, nu)) - math.fsum(special.gammaln(n + 1))
           + math.fsum(0.5 * ((gamma - 1.0) / sigma)[active] ** 2))
    assert st == hf.OK and abs(v - ref) <= 1e-12 * abs(ref)
    # d/d mu and d/d gamma_b by hand
    wb = np.where(n > 0, 1.0 - n / nu, 1.0)
    assert abs(g[0] - math.fsum(wb * nu / mu)) <= 1e-10 * abs(g[0])
    np.testing.assert_allclose(gg[active], (wb * nu / gamma + (gamma - 1.0) / sigma ** 2)[active], rtol=1e-10)


def test_stat_one_bin_closed_form_minimum():
    """One bin, one flagged sample A gamma with a Gaussian constraint of width
    sigma: A - n / gamma + (gamma - 1) / sigma^2 = 0 has the positive root
    gamma = [tau - A + sqrt((A - tau)^2 + 4 tau n)] / (2 tau), tau = 1/sigma^2;
    the oracle's derivative vanishes there and the NLL rises on both sides."""
    spec = {"n_bins": 1, "samples": ["s0"],
            "params": [{"name": "mu", "value": 1.0, "lo": 0.0, "hi": 10.0, "free": False, "constrained": False}],
            "modifiers": [{"type": "normfactor", "sample": 0, "param": 0}]}
    for A, n_obs, sig in ((40.0, 52.0, 0.1), (7.5, 3.0, 0.3), (1000.0, 1100.0, 0.02)):
        tau = 1.0 / sig ** 2
        gam = (tau - A + math.sqrt((A - tau) ** 2 + 4.0 * tau * n_obs)) / (2.0 * tau)
        s = (1, np.array([sig]), np.array([gam]))
        st, v, _, gg = hf.nll(spec, np.array([n_obs]), [np.array([A])], [], [], [1.0], stat=s)
        assert st == hf.OK and abs(gg[0]) <= 1e-9 * (A + tau)
        for d in (1e-4, -1e-4):
            s2 = (1, np.array([sig]), np.array([gam * (1 + d)]))
            assert hf.nll(spec, np.array([n_obs]), [np.array([A])], [], [], [1.0], stat=s2)[1] > v


def test_stat_gradients_match_central_differences(small):
    spec, n, T, up, dn = args(small)
    sigma, gamma = _stat(len(n), seed=11)
    mask = 0b011
    th = small["points"][1]
    st, v, g, gg = hf.nll(spec, n, T, up, dn, th, stat=(mask, sigma, gamma))
    assert st == hf.OK
    h = 1e-6
    for b in (0, 1, 2, 7, 14, 500, 999):
        gp, gm = gamma.copy(), gamma.copy()
        gp[b] += h
        gm[b] -= h
        fd = (hf.nll(spec, n, T, up, dn, th, grad=False, stat=(mask, sigma, gp))[1]
              - hf.nll(spec, n, T, up, dn, th, grad=False, stat=(mask, sigma, gm))[1]) / (2 * h)
        assert abs(fd - gg[b]) <= 1e-5 * (1 + abs(gg[b])) + 20 * 2.2e-16 * abs(v) / h, (b, fd, gg[b])
    for p in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (hf.nll(spec, n, T, up, dn, tp, grad=False, stat=(mask, sigma, gamma))[1]
              - hf.nll(spec, n, T, up, dn, tm, grad=False, stat=(mask, sigma, gamma))[1]) / (2 * h)
        assert abs(fd - g[p]) <= 1e-5 * (1 + abs(g[p])) + 20 * 2.2e-16 * abs(v) / h, (p, fd, g[p])
    # bins without a statistical parameter ignore gamma_b
    inactive = np.flatnonzero(~((sigma > 0) & np.isfinite(sigma)))
    g2 = gamma.copy()
    g2[inactive] = 3.0
    assert hf.nll(spec, n, T, up, dn, th, grad=False, stat=(mask, sigma, g2))[1] == v


# ---------------------------------------------------------------------------
# smooth interpolation codes, shifted constraints (luminosity), shapesys
# ---------------------------------------------------------------------------

def _smooth(spec):
    s = copy.deepcopy(spec)
    for m in s["modifiers"]:
        if m["type"] in ("normsys", "histosys"):
            m["interp"] = "poly6"
    return s


@pytest.mark.parametrize("hi,lo", [(1.1, 0.9), (1.3, 0.85), (1.02, 0.99), (2.0, 0.6), (1.2, 1.1)])
def test_poly6_normsys_meets_the_exponential_smoothly(hi, lo):
    """Value, first and second derivative of eta at alpha = +1 and -1 from
    inside (one-sided differences of the polynomial branch) equal those of
    hi^alpha and lo^-alpha (closed forms); eta(0) = 1; eta > 0 on [-1, 1]."""
    m = {"type": "normsys", "hi": hi, "lo": lo, "interp": "poly6"}
    e = lambda a: hf.normsys_eta(m, a)[0]
    de = lambda a: hf.normsys_eta(m, a)[1]
    assert abs(e(0.0) - 1.0) <= 1e-15
    h = 1e-4
    for x, val, d1, d2 in ((1.0, hi, hi * math.log(hi), hi * math.log(hi) ** 2),
                           (-1.0, lo, -lo * math.log(lo), lo * math.log(lo) ** 2)):
        s = -1.0 if x > 0 else 1.0   # step into the interpolation region
        xi = x + s * 1e-12
        assert abs(e(xi) - val) <= 1e-11 * val
        # one-sided second-order differences inside the region
        d1_in = -s * (3 * e(xi) - 4 * e(xi + s * h) + e(xi + 2 * s * h)) / (2 * h)
        d2_in = (2 * e(xi) - 5 * e(xi + s * h) + 4 * e(xi + 2 * s * h) - e(xi + 3 * s * h)) / h ** 2
        assert abs(d1_in - d1) <= 1e-6 * max(1.0, abs(d1)), (x, d1_in, d1)
        assert abs(d2_in - d2) <= 2e-3 * max(1.0, abs(d2)), (x, d2_in, d2)
        assert abs(de(xi) - d1) <= 1e-10 * max(1.0, abs(d1))
    assert all(e(a) > 0 for a in np.linspace(-1, 1, 41))


def test_poly6_histosys_meets_the_linear_extrapolation_smoothly():
    """The polynomial delta reaches alpha du at +1 and -alpha dd at -1 with
    the linear branches' slopes (du, dd) and zero curvature (one-sided
    differences), vanishes at 0, and its derivative matches central
    differences inside."""
    rng = np.random.default_rng(3)
    du, dd = rng.normal(0, 1, 7), rng.normal(0, 1, 7)
    m = {"type": "histosys", "interp": "poly6"}
    D = lambda a: hf.histosys_delta(m, a, du, dd)[0]
    dD = lambda a: hf.histosys_delta(m, a, du, dd)[1]
    assert np.all(D(0.0) == 0.0)
    h = 1e-4
    for x, val, slope in ((1.0, du, du), (-1.0, -dd, dd)):
        s = -1.0 if x > 0 else 1.0
        xi = x + s * 1e-12
        np.testing.assert_allclose(D(xi), val, atol=1e-11)
        d1_in = -s * (3 * D(xi) - 4 * D(xi + s * h) + D(xi + 2 * s * h)) / (2 * h)
        d2_in = (2 * D(xi) - 5 * D(xi + s * h) + 4 * D(xi + 2 * s * h) - D(xi + 3 * s * h)) / h ** 2
        np.testing.assert_allclose(d1_in, slope, atol=1e-6)
        np.testing.assert_allclose(d2_in, 0.0, atol=2e-3)
    for a in (-0.7, -0.2, 0.1, 0.55, 0.93):
        np.testing.assert_allclose(dD(a), (D(a + 1e-6) - D(a - 1e-6)) / 2e-6, rtol=1e-7, atol=1e-8)
    # outside: linear, the same as the default code
    lin = {"type": "histosys"}
    for a in (1.5, -2.0, 1.0, -1.0):
        np.testing.assert_allclose(D(a), hf.histosys_delta(lin, a, du, dd)[0], rtol=1e-14, atol=1e-14)


def test_poly6_model_fixed_points_and_gradient(small):
    """The model with every normsys and histosys on the smooth codes: at
    alpha = +-1 it equals the default-code model (the templates and hi / lo
    are reproduced), and its gradient matches fourth-order central
    differences at the seeded points (interior alphas)."""
    spec, n, T, up, dn = args(small)
    sm = _smooth(spec)
    th0 = datagen.theta_of(spec)
    for m in spec["modifiers"]:
        if m["type"] in ("normsys", "histosys"):
            for a in (1.0, -1.0):
                th = th0.copy()
                th[m["param"]] = a
                np.testing.assert_allclose(hf.expected(sm, T, up, dn, th)[0], hf.expected(spec, T, up, dn, th)[0],
                                           rtol=1e-11)
    for th in small["points"]:
        st, v, g = hf.nll(sm, n, T, up, dn, th)
        assert st == hf.OK
        for p in range(len(th)):
            h = 1e-5

            def f(x):
                t = th.copy()
                t[p] = x
                return hf.nll(sm, n, T, up, dn, t, grad=False)[1]

            fd = (f(th[p] - 2 * h) - 8 * f(th[p] - h) + 8 * f(th[p] + h) - f(th[p] + 2 * h)) / (12 * h)
            assert abs(fd - g[p]) <= 50 * 2.2e-16 * abs(v) / h + 1e-7 * abs(g[p]), (p, fd, g[p])


def test_luminosity_constraint_one_bin_maximum():
    """One bin of A mu events, mu a luminosity-like normfactor constrained
    with mean 1 and width s: the minimum of A mu - n ln(A mu) +
    (mu - 1)^2 / (2 s^2) is the positive root of
    mu^2 + (A s^2 - 1) mu - n s^2 = 0; the oracle's derivative vanishes there
    and the constraint adds exactly (mu - 1)^2 / (2 s^2) to the NLL."""
    for A, n_obs, s in ((100.0, 120.0, 0.02), (5.0, 9.0, 0.1), (2000.0, 1900.0, 0.05)):
        spec = {"n_bins": 1, "samples": ["s0"],
                "params": [{"name": "lumi", "value": 1.0, "lo": 0.0, "hi": 10.0, "free": True, "constrained": True,
                            "constraint_mean": 1.0, "constraint_sigma": s}],
                "modifiers": [{"type": "normfactor", "sample": 0, "param": 0}]}
        b = A * s * s - 1.0
        mu = (-b + math.sqrt(b * b + 4.0 * n_obs * s * s)) / 2.0
        st, v, g = hf.nll(spec, np.array([n_obs]), [np.array([A])], [], [], [mu])
        assert st == hf.OK and abs(g[0]) <= 1e-10 * (A + n_obs / mu + 1.0 / s ** 2)
        free = copy.deepcopy(spec)
        free["params"][0]["constrained"] = False
        v0 = hf.nll(free, np.array([n_obs]), [np.array([A])], [], [], [mu], grad=False)[1]
        assert abs((v - v0) - 0.5 * ((mu - 1.0) / s) ** 2) <= 1e-12 * abs(v)


def test_shapesys_constraint_matches_scipy_poisson():
    """Poisson-constrained gammas (shapesys): with tau_b = 1/sigma_b^2
    integral, the constraint added to the NLL equals -log Poisson(tau_b |
    gamma_b tau_b) (scipy) without its constant ln Gamma(tau + 1) - tau ln tau;
    one bin's minimum is gamma = (n + tau) / (A + tau); gamma_b <= 0 in a
    bin with a parameter is an invalid density."""
    w = datagen.hf_workload(n_bins=600, n_samples=1, n_histosys=0, n_normsys=0)
    spec = {"n_bins": 600, "samples": ["s0"], "params": [w["spec"]["params"][0]],
            "modifiers": [{"type": "normfactor", "sample": 0, "param": 0}]}
    n, T = w["counts"], w["nominal"]
    rng = np.random.default_rng(21)
    tau = rng.integers(4, 400, 600).astype(float)
    sigma = 1.0 / np.sqrt(tau)
    sigma[::13] = 0.0
    active = sigma > 0
    gamma = 1.0 + rng.uniform(-0.1, 0.1, 600)
    mu = 0.97
    st, v, g, gg = hf.nll(spec, n, T, [], [], [mu], stat=(1, sigma, gamma, "poisson"))
    st0, v0, _, _ = hf.nll(spec, n, T, [], [], [mu], stat=(1, sigma, gamma, "gauss"))
    assert st == st0 == hf.OK
    gauss = math.fsum(0.5 * ((gamma - 1.0) / sigma)[active] ** 2)
    t = tau[active]
    ref = math.fsum(-stats.poisson.logpmf(t, gamma[active] * t) + (t * np.log(t) - special.gammaln(t + 1)))
    assert abs((v - (v0 - gauss)) - ref) <= 1e-10 * abs(ref)
    for A, n_obs, tb in ((40.0, 52.0, 25.0), (7.5, 3.0, 9.0), (1000.0, 1100.0, 400.0)):
        one = {"n_bins": 1, "samples": ["s0"],
               "params": [{"name": "mu", "value": 1.0, "lo": 0.0, "hi": 10.0, "free": False, "constrained": False}],
               "modifiers": [{"type": "normfactor", "sample": 0, "param": 0}]}
        gam = (n_obs + tb) / (A + tb)
        s = (1, np.array([1.0 / math.sqrt(tb)]), np.array([gam]), "poisson")
        st, v1, _, g1 = hf.nll(one, np.array([n_obs]), [np.array([A])], [], [], [1.0], stat=s)
        assert st == hf.OK and abs(g1[0]) <= 1e-9 * (A + tb)
    bad = gamma.copy()
    bad[1] = -0.01
    assert hf.nll(spec, n, T, [], [], [mu], stat=(1, sigma, bad, "poisson"))[0] == hf.E_PDF
    bad[1] = 0.0
    assert hf.nll(spec, n, T, [], [], [mu], stat=(1, sigma, bad, "poisson"))[0] == hf.E_PDF


def test_shapesys_gradients_match_central_differences(small):
    spec, n, T, up, dn = args(small)
    sm = _smooth(spec)
    sigma, gamma = _stat(len(n), seed=17)
    mask = 0b001
    th = small["points"][2]
    s = (mask, sigma, gamma, "poisson")
    st, v, g, gg = hf.nll(sm, n, T, up, dn, th, stat=s)
    assert st == hf.OK
    h = 1e-6
    for b in (0, 1, 2, 7, 14, 500, 999):
        gp, gm = gamma.copy(), gamma.copy()
        gp[b] += h
        gm[b] -= h
        fd = (hf.nll(sm, n, T, up, dn, th, grad=False, stat=(mask, sigma, gp, "poisson"))[1]
              - hf.nll(sm, n, T, up, dn, th, grad=False, stat=(mask, sigma, gm, "poisson"))[1]) / (2 * h)
        assert abs(fd - gg[b]) <= 1e-5 * (1 + abs(gg[b])) + 20 * 2.2e-16 * abs(v) / h, (b, fd, gg[b])
    for p in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (hf.nll(sm, n, T, up, dn, tp, grad=False, stat=s)[1]
              - hf.nll(sm, n, T, up, dn, tm, grad=False, stat=s)[1]) / (2 * h)
        assert abs(fd - g[p]) <= 1e-5 * (1 + abs(g[p])) + 20 * 2.2e-16 * abs(v) / h, (p, fd, g[p])

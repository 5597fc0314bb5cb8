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

"""Pins of the composite-model oracle with formula leaves (oracle.composite)
against things other than itself: the scalar C++ oracle's built-in models
(closed-form normalisations, pinned in test_oracle_pins), the same models
with their leaves written as formulas, the additivity of a product's NLL
over its factors, the identity between fractions and yields, and finite
differences of its complex-step gradient."""
import copy

import numpy as np
import pytest

import datagen
import oracle
from oracle import composite, jit

GAUSS = datagen.GAUSS_FORMULA
EXPO = "exp(p[0]*x)"


def as_formulas(spec):
    """The same model with every gauss/exp leaf written as its formula."""
    s = copy.deepcopy(spec)
    for nd in s["nodes"]:
        if nd["kind"] == "gauss":
            nd["kind"], nd["density"] = "jit", GAUSS
        elif nd["kind"] == "exp":
            nd["kind"], nd["density"] = "jit", EXPO
    return s


def close(v, g, v2, g2, nll_tol=1e-12, grad_tol=1e-8):
    assert abs(v - v2) <= nll_tol * abs(v2), (v, v2)
    assert np.max(np.abs(g - g2)) <= grad_tol * np.max(np.abs(g2)), (g, g2)


@pytest.mark.parametrize("sigma", [0.4, 0.02])
def test_mixture_matches_scalar_oracle(sigma):
    """f Gauss + (1 - f) Exp: built-in kinds and the same leaves as formulas,
    against the C++ oracle's closed forms; a 0.02-wide peak included."""
    spec = datagen.mixture_spec(sigma=sigma)
    x = datagen.generate(spec, 4000, seed=11)
    orc = oracle.Oracle(spec)
    for th in ([0.2, 5.0, sigma, -0.7], [0.35, 4.98, sigma * 1.05, -0.4]):
        th = np.array(th)
        st2, v2, g2 = orc.nll(x, th)
        for s in (spec, as_formulas(spec)):
            st, v, g = composite.nll(s, x, th)
            assert st == 0 and st2 == 0
            close(v, g, v2, g2)


def test_three_term_sum_matches_scalar_oracle():
    """Three children with two fractions (Gauss, Gauss, Exp)."""
    spec = {"obs": [{"name": "x", "lo": 0.0, "hi": 10.0}],
            "params": [datagen.param(n, v, lo, hi) for n, v, lo, hi in
                       (("f1", 0.3, 0, 1), ("f2", 0.2, 0, 1), ("mu1", 3.0, 0, 10), ("s1", 0.6, 0.01, 5),
                        ("mu2", 7.0, 0, 10), ("s2", 0.4, 0.01, 5), ("c", -0.3, -5, 5))],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [2, 3], "norm": "analytic"},
                      {"kind": "gauss", "obs": 0, "params": [4, 5], "norm": "analytic"},
                      {"kind": "exp", "obs": 0, "params": [6], "norm": "analytic"},
                      {"kind": "sum", "params": [0, 1], "children": [0, 1, 2]}],
            "root": 3}
    x = datagen.generate(spec, 3000, seed=12)
    th = datagen.theta_of(spec) * 1.03
    st2, v2, g2 = oracle.Oracle(spec).nll(x, th)
    st, v, g = composite.nll(as_formulas(spec), x, th)
    assert st == 0 and st2 == 0
    close(v, g, v2, g2)


def test_product_is_the_sum_of_its_factors():
    """A formula on x times a Gaussian on y: the NLL and gradient are those
    of the two 1-D models (the stand-alone formula oracle and the C++
    oracle) added."""
    w = datagen.jit_composite_workload("prod", n=3000, n_points=2)
    spec, (x, y) = w["spec"], w["cols"]
    gs = datagen.gauss_spec(mu=0.2, sigma=1.2, lo=-5.0, hi=5.0)
    for th in w["points"]:
        st, v, g = composite.nll(spec, [x, y], th)
        s1, v1, g1 = jit.nll(datagen.POWER_EXP, 0.5, 10.0, [0.0, -5.0], [5.0, 5.0], x, th[:2])
        s2, v2, g2 = oracle.Oracle(gs).nll([y], th[2:])
        assert st == s1 == s2 == 0
        close(v, g, v1 + v2, np.concatenate([g1, g2]))


def test_yields_equal_fractions():
    """nu1 d1 + nu2 d2 over nu1 + nu2 is the fraction model at f = nu1 /
    (nu1 + nu2); its yield gradient is the fraction gradient times df/dnu."""
    w = datagen.jit_composite_workload("two_jit", n=3000, n_points=2)
    spec, x = w["spec"], w["cols"]
    frac = copy.deepcopy(spec)
    frac["params"] = [datagen.param("f", 0.3, 0.0, 1.0)] + spec["params"][2:]
    frac["nodes"][2] = {"kind": "sum", "params": [0], "children": [0, 1]}
    for nd in frac["nodes"][:2]:
        nd["params"] = [q - 1 for q in nd["params"]]
    for th in w["points"]:
        n1, n2 = th[0], th[1]
        S = n1 + n2
        st, v, g = composite.nll(spec, x, th)
        stf, vf, gf = composite.nll(frac, x, np.concatenate([[n1 / S], th[2:]]))
        assert st == stf == 0
        assert abs(v - vf) <= 1e-13 * abs(vf)
        dfd = np.array([n2 / S ** 2, -n1 / S ** 2])
        ref = np.concatenate([gf[0] * dfd, gf[1:]])
        assert np.max(np.abs(g - ref)) <= 1e-9 * np.max(np.abs(ref)), (g, ref)


def test_complex_step_gradient_matches_finite_differences():
    w = datagen.jit_composite_workload("three", n=2000, n_points=1)
    spec, x, th = w["spec"], w["cols"], w["points"][0]
    st, v, g = composite.nll(spec, x, th)
    assert st == 0
    for k in range(len(th)):
        h = 1e-5 * max(abs(th[k]), 1e-2)
        f = lambda d: composite.nll(spec, x, th + d * np.eye(len(th))[k], grad=False)[1]
        fd = (f(-2 * h) - 8 * f(-h) + 8 * f(h) - f(2 * h)) / (12 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1.0), (k, fd, g[k])


def test_status():
    """A parameter outside its range and fractions summing above 1: -3; a
    formula that is negative at an event: -5; a formula that vanishes at an
    event where the other term does not: valid."""
    w = datagen.jit_composite_workload("three", n=500, n_points=1)
    spec, x, th = w["spec"], w["cols"], w["points"][0].copy()
    bad = th.copy()
    bad[3] = 9.0  # s1 above its range
    assert composite.nll(spec, x, bad)[0] == composite.E_PARAM
    bad = th.copy()
    bad[0], bad[1] = 0.7, 0.5
    assert composite.nll(spec, x, bad)[0] == composite.E_PARAM
    neg = copy.deepcopy(spec)
    neg["params"][6]["lo"] = -1.0
    bad = th.copy()
    bad[6], bad[7] = -0.5, 0.0  # 1 - x/2 < 0 for x > 2
    assert composite.nll(neg, x, bad)[0] == composite.E_PDF
    zero = {"obs": spec["obs"], "params": [datagen.param("f", 0.5, 0, 1), datagen.param("c", -0.5, -5, 5)],
            "nodes": [{"kind": "jit", "obs": 0, "params": [1], "density": "(x > 2.0) * exp(p[0]*x)"},
                      {"kind": "exp", "obs": 0, "params": [1], "norm": "analytic"},
                      {"kind": "sum", "params": [0], "children": [0, 1]}], "root": 2}
    assert composite.nll(zero, [np.array([1.0, 3.0, 5.0])], np.array([0.5, -0.5]))[0] == composite.OK

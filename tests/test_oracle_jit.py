"""Pins of the expression-string (just-in-time PDF) oracle against things
other than itself: the built-in Gaussian and exponential leaves of the
scalar oracle (pinned to scipy), 40-digit mpmath integrals, and finite
differences of its complex-step gradient."""
import math

import mpmath as mp
import numpy as np
import pytest

import datagen
import oracle
from oracle import jit

GAUSS = "exp(-0.5*((x-p[0])/p[1])*((x-p[0])/p[1]))"
EXPO = "exp(p[0]*x)"
POLYEXP = "(1.0 + p[0]*x*x) * exp(-x/p[1]) + p[2]"


def builtin(kind, params, lo, hi):
    ps = [datagen.param(f"p{k}", v, -1e3, 1e3) for k, v in enumerate(params)]
    return oracle.Oracle({"obs": [{"name": "x", "lo": lo, "hi": hi}], "params": ps,
                          "nodes": [{"kind": kind, "obs": 0, "params": list(range(len(params)))}], "root": 0})


@pytest.mark.parametrize("expr,kind,lo,hi", [(GAUSS, "gauss", -10.0, 10.0), (EXPO, "exp", 0.0, 10.0)])
def test_matches_builtin_leaves(expr, kind, lo, hi):
    spec = datagen.gauss_spec() if kind == "gauss" else None
    x = (datagen.generate(spec, 3000, seed=3)[0] if spec else
         datagen.generate({"obs": [{"name": "x", "lo": lo, "hi": hi}], "params": [datagen.param("c", -0.7, -5, 5)],
                           "nodes": [{"kind": "exp", "obs": 0, "params": [0]}], "root": 0}, 3000, seed=4)[0])
    pts = [[0.3, 1.5], [0.1, 1.2]] if kind == "gauss" else [[-0.7], [-0.4]]
    for th in pts:
        st, v, g = jit.nll(expr, lo, hi, [-1e3] * len(th), [1e3] * len(th), x, th)
        st2, v2, g2 = builtin(kind, th, lo, hi).nll([x], np.array(th))
        assert st == 0 and st2 == 0
        assert abs(v - v2) <= 1e-12 * abs(v2), (v, v2)
        np.testing.assert_allclose(g, g2, rtol=1e-9, atol=1e-9 * np.abs(g2).max())


def test_norm_against_40_digit_quadrature():
    mp.mp.dps = 40
    p = [0.3, 2.0, 0.05]
    Z, _ = jit.norm(POLYEXP, 0.0, 8.0, p)
    ref = mp.quad(lambda t: (1 + mp.mpf("0.3") * t * t) * mp.exp(-t / 2) + mp.mpf("0.05"), [0, 8])
    assert abs(Z - float(ref)) <= 1e-13 * float(ref)


def test_complex_step_gradient_matches_finite_differences():
    x = np.linspace(0.05, 7.95, 400)
    th = np.array([0.3, 2.0, 0.05])
    st, v, g = jit.nll(POLYEXP, 0.0, 8.0, [0, 0.1, 0], [5, 10, 1], x, th)
    assert st == 0
    for k in range(3):
        h = 1e-5 * max(abs(th[k]), 1e-2)
        f = lambda d: jit.nll(POLYEXP, 0.0, 8.0, [0, 0.1, 0], [5, 10, 1], x, th + d * np.eye(3)[k], grad=False)[1]
        fd = (f(-2 * h) - 8 * f(-h) + 8 * f(h) - f(2 * h)) / (12 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1.0), (k, fd, g[k])


def test_status_conventions():
    x = np.array([0.5, 1.0])
    assert jit.nll(GAUSS, -10, 10, [-5, 0.1], [5, 5], x, [0.0, 6.0])[0] == jit.E_PARAM
    assert jit.nll("x - p[0]", 0, 2, [-5], [5], x, [0.7])[0] == jit.E_PDF  # negative at x = 0.5


@pytest.mark.parametrize("sigma", [0.02, 0.005])
def test_narrow_peak_matches_builtin(sigma):
    """A Gaussian 1/500 to 1/2000 of the range wide: the normalisation and
    its derivatives (which vanish at the peak's centre) against the C++
    oracle's closed form."""
    spec = datagen.gauss_spec(5.0, sigma, 0.0, 10.0)
    spec["params"][1]["lo"] = 1e-4
    x = datagen.generate(spec, 3000, seed=5)[0]
    for th in ([5.0, sigma], [5.0 + 0.3 * sigma, 1.1 * sigma]):
        st, v, g = jit.nll(GAUSS, 0.0, 10.0, [0.0, 1e-4], [10.0, 5.0], x, th)
        st2, v2, g2 = oracle.Oracle(spec).nll([x], np.array(th))
        assert st == 0 and st2 == 0
        assert abs(v - v2) <= 1e-12 * abs(v2), (v, v2)
        assert np.max(np.abs(g - g2)) <= 1e-8 * np.max(np.abs(g2)), (g, g2)

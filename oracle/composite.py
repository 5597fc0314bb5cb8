"""Composite models with formula leaves -- TEST INFRASTRUCTURE ONLY.

Sec. 4 describes densities given as formula strings and compiled at run
time; Sec. 1 describes likelihood models as computation graphs of
observables, parameters, functions and densities, sums and products among
them.  The reading used here puts the two together: a formula density is a
leaf like any built-in one, so it may sit anywhere in a graph of sums and
products.  Written out plainly, for checking by eye:

  leaf l on observable o with parameters p = theta[params]:
      d_l(x) = g_l(x_o; p) / Z_l,   Z_l = int_{lo_o}^{hi_o} g_l dx_o;
  sum over children j = 1..k with fractions f_1..f_{k-1}:
      d(x) = sum_{j<k} f_j d_j(x) + (1 - sum_{j<k} f_j) d_k(x),
  or with yields nu_1..nu_k:
      d(x) = sum_j nu_j d_j(x) / sum_j nu_j;
  product over children on disjoint observables:
      d(x) = prod_j d_j(x);
  NLL = -sum_i log d(x_i)   (exactly rounded sum over the events).

Leaf kinds: "jit" (the node's "density", an expression in x and p[k] with
the functions of ``oracle.jit``) and, for models that mix formulas with
built-in densities, "gauss" (mu, sigma: exp(-((x - mu)/sigma)^2/2)) and
"exp" (c: exp(c x)) written from their definitions.  Every leaf is
normalised by scipy's adaptive Gauss-Kronrod quadrature (no closed forms,
nothing shared with the device's Gauss-Legendre rules).

The gradient is the complex step of the whole NLL,
    d NLL / d theta_k = Im NLL(theta + i h e_k) / h,
with every step above (the formulas, the quadratures of the real and
imaginary parts, the sums, the logarithm) taken in complex arithmetic;
exact to rounding for analytic expressions, and sharing nothing with the
device's dual numbers.

Status (as the library): -3 a parameter outside its range, a fraction
outside [0, 1] or fractions summing above 1, a negative yield or a yield
total <= 0; -5 a leaf value negative or not finite at an event, a leaf
normalisation <= 0 or not finite, or d(x_i) <= 0 or not finite.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate

from . import jit as _jit

OK, E_PARAM, E_PDF = 0, -3, -5
H = 1e-30  # complex step

BUILTIN = {"gauss": "exp(-0.5*((x-p[0])/p[1])*((x-p[0])/p[1]))", "exp": "exp(p[0]*x)"}


def leaf_expr(node):
    return node["density"] if node["kind"] == "jit" else BUILTIN[node["kind"]]


def _quad(f, lo, hi):
    """int_lo^hi f, adaptive, started from 64 equal subintervals: a rule
    over the whole range can miss a peak narrow against it altogether (the
    derivative integrands vanish at a symmetric peak's centre, where the
    first rule's middle node falls)."""
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        return integrate.quad(f, lo, hi, epsabs=0, epsrel=2e-14, limit=4000,
                              points=np.linspace(lo, hi, 65)[1:-1])[0]


def leaf_norm(expr, lo, hi, p):
    """Z of g(x; p) over [lo, hi]; p real or complex (then Z is complex, its
    real and imaginary parts integrated apart)."""
    p = np.asarray(p)
    re = _quad(lambda t: float(np.real(_jit.g(expr, np.array([t]), p))[0]), lo, hi)
    if not np.iscomplexobj(p) or not np.any(np.imag(p)):
        return complex(re, 0.0)
    im = _quad(lambda t: float(np.imag(_jit.g(expr, np.array([t]), p))[0]), lo, hi)
    return complex(re, im)


def density(spec, cols, theta, i, check):
    """d_i at the events (complex array) for node i; theta real or complex.
    check: list collecting invalid-density findings on the real path."""
    node = spec["nodes"][i]
    kind = node["kind"]
    if kind in ("sum", "prod"):
        ds = [density(spec, cols, theta, c, check) for c in node["children"]]
        if kind == "prod":
            out = ds[0]
            for d in ds[1:]:
                out = out * d
            return out
        coef = [theta[q] for q in node["params"]]
        if len(coef) == len(ds) - 1:
            coef = coef + [1.0 - sum(coef)]
            return sum(c * d for c, d in zip(coef, ds))
        total = sum(coef)
        return sum(c * d for c, d in zip(coef, ds)) / total
    o = node["obs"]
    lo, hi = float(spec["obs"][o]["lo"]), float(spec["obs"][o]["hi"])
    expr = leaf_expr(node)
    p = np.array([theta[q] for q in node["params"]])
    g = _jit.g(expr, np.asarray(cols[o], dtype=np.float64), p)
    Z = leaf_norm(expr, lo, hi, p)
    gr = np.real(g)
    if np.any(gr < 0) or not np.all(np.isfinite(gr)) or not (Z.real > 0) or not math.isfinite(Z.real):
        check.append(i)
    return g / Z


def params_ok(spec, theta):
    th = np.real(np.asarray(theta))
    for k, par in enumerate(spec["params"]):
        if not (par["lo"] <= th[k] <= par["hi"]):
            return False
    for node in spec["nodes"]:
        if node["kind"] != "sum":
            continue
        c = [th[q] for q in node["params"]]
        if len(c) == len(node["children"]) - 1:
            if any(v < 0 or v > 1 for v in c) or sum(c) > 1:
                return False
        elif any(v < 0 for v in c) or not (sum(c) > 0):
            return False
    return True


def nll_value(spec, cols, theta, check):
    d = density(spec, cols, theta, int(spec["root"]), check)
    lg = np.log(d.astype(np.complex128))
    return complex(-math.fsum(np.real(lg)), -math.fsum(np.imag(lg))), d


def nll(spec, cols, theta, grad=True):
    """(status, NLL, gradient) at theta (fixed parameters get 0)."""
    th = np.asarray(theta, dtype=np.float64)
    P = len(th)
    if not params_ok(spec, th):
        return E_PARAM, math.inf, np.zeros(P)
    check = []
    v, d = nll_value(spec, cols, th.astype(np.complex128), check)
    dr = np.real(d)
    if check or np.any(~(dr > 0)) or not np.all(np.isfinite(dr)) or not math.isfinite(v.real):
        return E_PDF, math.inf, np.zeros(P)
    g = np.zeros(P)
    if grad:
        for k in range(P):
            if not spec["params"][k].get("free", True):
                continue
            tc = th.astype(np.complex128)
            tc[k] += 1j * H
            g[k] = nll_value(spec, cols, tc, [])[0].imag / H
    return OK, v.real, g

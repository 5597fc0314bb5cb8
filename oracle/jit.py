"""Just-in-time densities from expression strings -- TEST INFRASTRUCTURE ONLY.

Sec. 4 describes PDFs given as formula strings and compiled at run time
(RooGenericPdf on TFormula and cling).  The reading used here: one
observable x on [lo, hi], a density expression g(x; p[0..P-1]) written in
C syntax with the functions below, normalised over the range,

    p(x) = g(x) / Z,  Z = int_lo^hi g dx,
    NLL  = -sum_i log g(x_i) + N log Z,

valid where every g(x_i) > 0.  This oracle evaluates the expression with
numpy (vectorised over the events), integrates with scipy's adaptive
Gauss-Kronrod quadrature (independent of the device's Gauss-Legendre rule),
and differentiates by the complex step d f/d p_k = Im f(p + i h e_k) / h
(exact to rounding for analytic expressions), which shares nothing with
the device's dual numbers.  Sums over events are exactly rounded.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate, special

OK, E_PARAM, E_PDF = 0, -3, -5
H = 1e-30  # complex step

FUNCS = {"exp": np.exp, "log": np.log, "sqrt": np.sqrt, "pow": np.power, "sin": np.sin, "cos": np.cos,
         "tan": np.tan, "atan": np.arctan, "tanh": np.tanh, "sinh": np.sinh, "cosh": np.cosh,
         "asinh": np.arcsinh, "erf": special.erf}


def g(expr: str, x, p):
    """The expression at x (array) and parameters p (real or complex)."""
    env = dict(FUNCS)
    env["x"] = x
    env["p"] = p
    return eval(expr, {"__builtins__": {}}, env) + 0.0 * x  # broadcast constants


def g_and_grad(expr: str, x, p):
    """g and dg/dp_k (complex step) at x."""
    p = np.asarray(p, dtype=np.float64)
    v = np.real(g(expr, x, p.astype(np.complex128)))
    d = []
    for k in range(len(p)):
        pc = p.astype(np.complex128)
        pc[k] += 1j * H
        d.append(np.imag(g(expr, x, pc)) / H)
    return v, d


def norm(expr: str, lo: float, hi: float, p):
    """Z and dZ/dp_k by adaptive quadrature (asked for 2e-14 relative: quad
    reports that rounding limits it there, which is the intent), started
    from 64 equal subintervals: one rule over the whole range can miss a
    peak narrow against it (the derivative integrands vanish at a symmetric
    peak's centre, where that rule's middle node falls)."""
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        return _norm(expr, lo, hi, p)


def _norm(expr: str, lo: float, hi: float, p):
    p = np.asarray(p, dtype=np.float64)
    f = lambda t: float(np.real(g(expr, np.array([t]), p.astype(np.complex128)))[0])
    pts = np.linspace(lo, hi, 65)[1:-1]
    Z = integrate.quad(f, lo, hi, epsabs=0, epsrel=2e-14, limit=4000, points=pts)[0]
    dZ = []
    for k in range(len(p)):
        def fk(t, k=k):
            pc = p.astype(np.complex128)
            pc[k] += 1j * H
            return float(np.imag(g(expr, np.array([t]), pc))[0]) / H
        dZ.append(integrate.quad(fk, lo, hi, epsabs=0, epsrel=2e-14, limit=4000, points=pts)[0])
    return Z, np.array(dZ)


def nll(expr: str, lo: float, hi: float, par_lo, par_hi, x, theta, free=None, grad=True):
    """(status, NLL, gradient)."""
    th = np.asarray(theta, dtype=np.float64)
    P = len(th)
    if not all(par_lo[k] <= th[k] <= par_hi[k] for k in range(P)):
        return E_PARAM, math.inf, np.zeros(P)
    x = np.asarray(x, dtype=np.float64)
    v, d = g_and_grad(expr, x, th)
    Z, dZ = norm(expr, lo, hi, th)
    if np.any(~(v > 0)) or not np.all(np.isfinite(v)) or not (Z > 0):
        return E_PDF, math.inf, np.zeros(P)
    n = len(x)
    value = -math.fsum(np.log(v)) + n * math.log(Z)
    gr = np.zeros(P)
    if grad:
        for k in range(P):
            if free is not None and not free[k]:
                continue
            gr[k] = -math.fsum(d[k] / v) + n * dZ[k] / Z
    return OK, value, gr

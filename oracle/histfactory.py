"""Binned template likelihood of HistFactory type -- TEST INFRASTRUCTURE ONLY.

The paper names HistFactory's binned models (built from histograms, Sec. 1)
as the next target of its work (Summary) without defining them.  This is
the reading used here, after the HistFactory definitions (Cranmer et al.,
CERN-OPEN-2012-016), written out plainly in numpy FP64 so that it can be
checked by eye:

  bins b (all channels concatenated), observed counts n_b >= 0;
  samples s with nominal expected counts T_sb;
  modifiers, each acting on one sample through one parameter:
    normfactor (parameter mu):     the sample times mu;
    normsys (alpha, hi, lo):       the sample times eta(alpha), with
                                   eta = hi^alpha (alpha >= 0), lo^-alpha (alpha < 0);
    histosys (alpha, up_b, down_b): the sample's bins plus
                                   alpha (up_b - T_sb)   (alpha >= 0),
                                   alpha (T_sb - down_b) (alpha < 0);
  a parameter may drive several modifiers (correlated across samples);
  nu_b = sum_s [prod normfactors] [prod normsys] (T_sb + sum histosys deltas);
  NLL = sum_b (nu_b - n_b ln nu_b) + 1/2 sum_{constrained p} ((theta_p - m_p) / s_p)^2
  (the Poisson terms without ln n_b!, Gaussian constraints of mean m_p and
  width s_p -- 0 and 1 unless the parameter gives "constraint_mean",
  "constraint_sigma" -- without their normalisation; a bin with n_b = 0
  contributes nu_b).  A luminosity parameter is a normfactor on the samples
  it scales, constrained with mean 1 and the luminosity's relative
  uncertainty as width.

Smooth interpolation codes (HistFactory's "code 4" for normsys, its
polynomial interpolation with linear extrapolation for histosys; modifier
"interp": "poly6"; the defaults above are "exp" and "linear"):
  normsys: for |alpha| < 1, eta = 1 + sum_{i=1..6} a_i alpha^i, the
    polynomial whose value, first and second derivatives at alpha = +1 and
    -1 equal those of hi^alpha and lo^-alpha there (six linear conditions,
    solved here with numpy); outside, hi^alpha / lo^-alpha;
  histosys: with du = up - T, dd = T - down, for |alpha| < 1 the delta is
    alpha (S + alpha A (15 + alpha^2 (3 alpha^2 - 10))), S = (du + dd) / 2,
    A = (du - dd) / 16 (an odd linear part and an even sixth-order part that
    meet alpha du at +1 and -alpha dd at -1 with equal first and second
    derivatives); outside, alpha du (alpha > 1) or alpha dd (alpha < -1).

Per-bin statistical parameters (HistFactory's "staterror", the
Barlow-Beeston-lite treatment of the templates' own statistical error):
samples flagged in a mask share one factor gamma_b per bin, with a
Gaussian constraint of width sigma_b (the templates' relative statistical
error in that bin):
  nu_b = gamma_b nu_b^(flagged) + nu_b^(others),
  NLL += 1/2 sum_b (gamma_b - 1)^2 / sigma_b^2,
  d NLL / d gamma_b = w_b nu_b^(flagged) + (gamma_b - 1) / sigma_b^2,
  w_b = 1 - n_b / nu_b (1 where n_b = 0).
Bins with sigma_b <= 0 (or not finite) have no gamma: gamma_b is taken as
1 there and its derivative is 0.  Reading: the constraint without its
normalisation, like the unit Gaussians.  The same gammas with a Poisson
constraint instead (HistFactory's "shapesys": the template's statistical
error as an auxiliary count tau_b = 1/sigma_b^2 observed for a Poisson mean
gamma_b tau_b): NLL += sum_b (tau_b gamma_b - tau_b ln gamma_b) (the
Poisson term without its constant ln Gamma(tau + 1) - tau ln tau), d / d gamma_b =
w_b nu_b^(flagged) + tau_b (1 - 1/gamma_b); gamma_b <= 0 in a bin with a
parameter is an invalid density (status -5).

Status codes as the unbinned oracle: 0 ok, -3 a parameter outside its
range, -5 an expected count nu_b <= 0 where n_b > 0, or nu_b < 0.
The derivative at alpha = 0 exactly is the alpha >= 0 side's.

Spec: {"n_bins": B, "samples": [names], "params": [{"name", "value", "lo",
"hi", "free", "constrained", ("constraint_mean", "constraint_sigma")}],
"modifiers": [{"type", "sample", "param", ("hi", "lo"), ("interp")}]}; data:
counts[B], nominal[S][B], and per histosys modifier (in the order of
"modifiers") its up and down templates.
"""
from __future__ import annotations

import math

import numpy as np

OK, E_PARAM, E_PDF = 0, -3, -5


def histosys_list(spec):
    return [m for m in spec["modifiers"] if m["type"] == "histosys"]


def normsys_poly6(hi, lo):
    """a_1..a_6 of the normsys interpolation polynomial: the six conditions
    eta(+-1), eta'(+-1), eta''(+-1) of 1 + sum a_i alpha^i equal to those of
    hi^alpha at +1 and lo^-alpha at -1."""
    A = np.zeros((6, 6))
    b = np.zeros(6)
    lh, ll = math.log(hi), math.log(lo)
    for row, (x, val, d1, d2) in enumerate(((1.0, hi - 1.0, hi * lh, hi * lh * lh),
                                            (-1.0, lo - 1.0, -lo * ll, lo * ll * ll))):
        for i in range(1, 7):
            A[3 * row, i - 1] = x ** i
            A[3 * row + 1, i - 1] = i * x ** (i - 1)
            A[3 * row + 2, i - 1] = i * (i - 1) * x ** (i - 2) if i >= 2 else 0.0
        b[3 * row], b[3 * row + 1], b[3 * row + 2] = val, d1, d2
    return np.linalg.solve(A, b)


def normsys_eta(m, a):
    """(eta, d eta / d alpha) of a normsys modifier at alpha = a."""
    hi, lo = m["hi"], m["lo"]
    if m.get("interp", "exp") == "poly6" and abs(a) < 1.0:
        c = normsys_poly6(hi, lo)
        return (1.0 + sum(c[i - 1] * a ** i for i in range(1, 7)),
                sum(i * c[i - 1] * a ** (i - 1) for i in range(1, 7)))
    if a >= 0:
        return hi ** a, math.log(hi) * hi ** a
    return lo ** (-a), -math.log(lo) * lo ** (-a)


def histosys_delta(m, a, du, dd):
    """(delta, d delta / d alpha) of a histosys modifier at alpha = a, with
    du = up - T and dd = T - down."""
    if m.get("interp", "linear") == "poly6" and abs(a) < 1.0:
        S, A = 0.5 * (du + dd), 0.0625 * (du - dd)
        return (a * (S + a * A * (15.0 + a * a * (3.0 * a * a - 10.0))),
                S + A * (30.0 * a - 40.0 * a ** 3 + 18.0 * a ** 5))
    if a >= 0:
        return a * du, du
    return a * dd, dd


def constraint(par, v):
    """(1/2 ((v - m) / s)^2, its derivative) of a constrained parameter."""
    mean, sig = par.get("constraint_mean", 0.0), par.get("constraint_sigma", 1.0)
    return 0.5 * ((v - mean) / sig) ** 2, (v - mean) / (sig * sig)


def expected(spec, nominal, up, down, theta, stat=None):
    """nu_b (and, per parameter, d nu_b / d theta_p) by the definition.
    stat = (mask, sigma, gamma): the flagged samples' contributions to bin b
    are multiplied by gamma_b where sigma_b > 0."""
    th = np.asarray(theta, dtype=np.float64)
    S, P = len(spec["samples"]), len(spec["params"])
    T = [np.asarray(nominal[s], dtype=np.float64) for s in range(S)]
    hs = histosys_list(spec)
    # each sample: its shape (nominal plus histosys deltas) and its factors
    shape = [t.copy() for t in T]
    dshape = {}  # (sample, param) -> d shape / d alpha
    k = 0
    for m in spec["modifiers"]:
        if m["type"] != "histosys":
            continue
        s, p = m["sample"], m["param"]
        delta, ddelta = histosys_delta(m, th[p], np.asarray(up[k]) - T[s], T[s] - np.asarray(down[k]))
        shape[s] = shape[s] + delta
        dshape[(s, p)] = dshape.get((s, p), 0.0) + ddelta
        k += 1
    assert k == len(hs)
    factor = np.ones(S)
    for m in spec["modifiers"]:
        s, p = m["sample"], m["param"]
        if m["type"] == "normfactor":
            factor[s] *= th[p]
        elif m["type"] == "normsys":
            factor[s] *= normsys_eta(m, th[p])[0]
    # per sample and bin: the gamma_b of flagged samples (else 1)
    gfac = [np.ones_like(T[0]) for _ in range(S)]
    if stat is not None:
        mask, sigma, gamma = stat[:3]
        sig = np.asarray(sigma, dtype=np.float64)
        active = (sig > 0) & np.isfinite(sig)
        g_eff = np.where(active, np.asarray(gamma, dtype=np.float64), 1.0)
        for s in range(S):
            if (mask >> s) & 1:
                gfac[s] = g_eff
    shape = [gfac[s] * shape[s] for s in range(S)]
    dshape = {k: gfac[k[0]] * v for k, v in dshape.items()}
    nu = np.zeros_like(T[0])
    for s in range(S):
        nu = nu + factor[s] * shape[s]
    # derivatives: product rule over each sample's factors and its shape
    dnu = [np.zeros_like(nu) for _ in range(P)]
    for s in range(S):
        mods = [m for m in spec["modifiers"] if m["sample"] == s]
        for i, m in enumerate(mods):
            p = m["param"]
            if m["type"] == "histosys":
                continue
            others = 1.0
            for j, o in enumerate(mods):
                if j == i or o["type"] == "histosys":
                    continue
                a = th[o["param"]]
                others *= a if o["type"] == "normfactor" else normsys_eta(o, a)[0]
            if m["type"] == "normfactor":
                d_factor = others
            else:
                d_factor = others * normsys_eta(m, th[p])[1]
            dnu[p] = dnu[p] + d_factor * shape[s]
        for (s2, p), ds in dshape.items():
            if s2 == s:
                dnu[p] = dnu[p] + factor[s] * ds
    return nu, dnu


def nll(spec, counts, nominal, up, down, theta, grad=True, stat=None):
    """(status, NLL, gradient) with exactly rounded sums over bins.  With
    stat = (mask, sigma, gamma[, kind]) (per-bin statistical parameters,
    kind "gauss" -- staterror, the default -- or "poisson" -- shapesys; see
    the header): (status, NLL, gradient, d NLL / d gamma_b per bin)."""
    th = np.asarray(theta, dtype=np.float64)
    P = len(spec["params"])
    n = np.asarray(counts, dtype=np.float64)
    bad = (E_PARAM, math.inf, np.zeros(P)) + ((np.zeros(len(n)),) if stat is not None else ())
    for p, par in enumerate(spec["params"]):
        if not (par["lo"] <= th[p] <= par["hi"]):
            return bad
    nu, dnu = expected(spec, nominal, up, down, th, stat)
    if np.any(nu < 0) or np.any((n > 0) & ~(nu > 0)) or not np.all(np.isfinite(nu)):
        return (E_PDF,) + bad[1:]
    kind = stat[3] if stat is not None and len(stat) > 3 else "gauss"
    if stat is not None and kind == "poisson":
        sig = np.asarray(stat[1], dtype=np.float64)
        act = (sig > 0) & np.isfinite(sig)
        if not np.all(np.asarray(stat[2], dtype=np.float64)[act] > 0):
            return (E_PDF,) + bad[1:]
    pos = n > 0
    terms = nu.copy()
    terms[pos] = nu[pos] - n[pos] * np.log(nu[pos])
    cons = [constraint(par, th[p])[0] for p, par in enumerate(spec["params"]) if par.get("constrained", False)]
    if stat is not None:
        mask, sigma, gamma = stat[:3]
        sig = np.asarray(sigma, dtype=np.float64)
        active = (sig > 0) & np.isfinite(sig)
        gam = np.asarray(gamma, dtype=np.float64)
        if kind == "poisson":
            tau = 1.0 / sig[active] ** 2
            cons.append(math.fsum(tau * gam[active] - tau * np.log(gam[active])))
        else:
            cons.append(math.fsum(0.5 * (gam[active] - 1.0) ** 2 / sig[active] ** 2))
    value = math.fsum(terms) + math.fsum(cons)
    g = np.zeros(P)
    w = np.ones_like(nu)
    w[pos] = 1.0 - n[pos] / nu[pos]
    if grad:
        for p, par in enumerate(spec["params"]):
            if not par.get("free", True):
                continue
            g[p] = math.fsum(w * dnu[p]) + (constraint(par, th[p])[1] if par.get("constrained", False) else 0.0)
    if stat is None:
        return OK, value, g
    # d nu_b / d gamma_b = the flagged samples' part of nu_b without gamma:
    # nu_b with the other samples multiplied by 0 and gamma = 1
    S = len(spec["samples"])
    others = (~mask) & ((1 << S) - 1)
    nu_flag = expected(spec, nominal, up, down, th, (others, np.ones(len(n)), np.zeros(len(n))))[0]
    sig1 = np.where(active, sig, 1.0)
    if kind == "poisson":
        dcons = (1.0 - 1.0 / np.where(active, gam, 1.0)) / sig1 ** 2
    else:
        dcons = (gam - 1.0) / sig1 ** 2
    gg = np.where(active, w * nu_flag + dcons, 0.0)
    return OK, value, g, gg

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
  NLL = sum_b (nu_b - n_b ln nu_b) + 1/2 sum_{constrained p} theta_p^2
  (the Poisson terms without ln n_b!, unit Gaussian constraints without
  their normalisation; a bin with n_b = 0 contributes nu_b).

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
normalisation, like the unit Gaussians.

Status codes as the unbinned oracle: 0 ok, -3 a parameter outside its
range, -5 an expected count nu_b <= 0 where n_b > 0, or nu_b < 0.
The derivative at alpha = 0 exactly is the alpha >= 0 side's.

Spec: {"n_bins": B, "samples": [names], "params": [{"name", "value", "lo",
"hi", "free", "constrained"}], "modifiers": [{"type", "sample", "param",
("hi", "lo")}]}; data: counts[B], nominal[S][B], and per histosys modifier
(in the order of "modifiers") its up and down templates.
"""
from __future__ import annotations

import math

import numpy as np

OK, E_PARAM, E_PDF = 0, -3, -5


def histosys_list(spec):
    return [m for m in spec["modifiers"] if m["type"] == "histosys"]


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
        a = th[p]
        delta = (np.asarray(up[k]) - T[s]) if a >= 0 else (T[s] - np.asarray(down[k]))
        shape[s] = shape[s] + a * delta
        dshape[(s, p)] = dshape.get((s, p), 0.0) + delta
        k += 1
    assert k == len(hs)
    factor = np.ones(S)
    for m in spec["modifiers"]:
        s, p = m["sample"], m["param"]
        if m["type"] == "normfactor":
            factor[s] *= th[p]
        elif m["type"] == "normsys":
            a = th[p]
            factor[s] *= m["hi"] ** a if a >= 0 else m["lo"] ** (-a)
    # per sample and bin: the gamma_b of flagged samples (else 1)
    gfac = [np.ones_like(T[0]) for _ in range(S)]
    if stat is not None:
        mask, sigma, gamma = stat
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
                if o["type"] == "normfactor":
                    others *= a
                else:
                    others *= o["hi"] ** a if a >= 0 else o["lo"] ** (-a)
            if m["type"] == "normfactor":
                d_factor = others
            else:
                a = th[p]
                d_factor = others * (math.log(m["hi"]) * m["hi"] ** a if a >= 0
                                     else -math.log(m["lo"]) * m["lo"] ** (-a))
            dnu[p] = dnu[p] + d_factor * shape[s]
        for (s2, p), ds in dshape.items():
            if s2 == s:
                dnu[p] = dnu[p] + factor[s] * ds
    return nu, dnu


def nll(spec, counts, nominal, up, down, theta, grad=True, stat=None):
    """(status, NLL, gradient) with exactly rounded sums over bins.  With
    stat = (mask, sigma, gamma) (per-bin statistical parameters, see the
    header): (status, NLL, gradient, d NLL / d gamma_b per bin)."""
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
    pos = n > 0
    terms = nu.copy()
    terms[pos] = nu[pos] - n[pos] * np.log(nu[pos])
    cons = [0.5 * th[p] ** 2 for p, par in enumerate(spec["params"]) if par.get("constrained", False)]
    if stat is not None:
        mask, sigma, gamma = stat
        sig = np.asarray(sigma, dtype=np.float64)
        active = (sig > 0) & np.isfinite(sig)
        gam = np.asarray(gamma, dtype=np.float64)
        cons.append(math.fsum(0.5 * (gam[active] - 1.0) ** 2 / sig[active] ** 2))
    value = math.fsum(terms) + math.fsum(cons)
    g = np.zeros(P)
    w = np.ones_like(nu)
    w[pos] = 1.0 - n[pos] / nu[pos]
    if grad:
        for p, par in enumerate(spec["params"]):
            if not par.get("free", True):
                continue
            g[p] = math.fsum(w * dnu[p]) + (th[p] if par.get("constrained", False) else 0.0)
    if stat is None:
        return OK, value, g
    # d nu_b / d gamma_b = the flagged samples' part of nu_b without gamma:
    # nu_b with the other samples multiplied by 0 and gamma = 1
    S = len(spec["samples"])
    others = (~mask) & ((1 << S) - 1)
    nu_flag = expected(spec, nominal, up, down, th, (others, np.ones(len(n)), np.zeros(len(n))))[0]
    gg = np.where(active, w * nu_flag + (gam - 1.0) / np.where(active, sig, 1.0) ** 2, 0.0)
    return OK, value, g, gg

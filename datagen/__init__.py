"""Seeded synthetic inputs shared by the tests and the benchmark.

This module only *generates inputs*: the model specifications (a neutral,
JSON-like dict that both the GPU binding and the oracle translate into their
own structures), the event columns, parameter points and toy sizes.  It
computes no likelihood, normalisation or gradient.

Randomness is Philox4x64-10 (counter-based, see ``datagen.cpp``) so every
value is reproducible independently of threading.  Seeds: master
2003012875; data seed = master + 1000 * config number; parameter-point seed
= data seed + 1; toy k of the batched workload uses stream (4 << 32) + k.

The five workloads stand in for the paper's benchmark models (its Fig. 1
covers 100k-300k events of "various likelihood models" whose definitions
are not given): a wide Gaussian, a Gaussian-plus-exponential mixture, a
2-D Crystal Ball / ARGUS mixture times a Chebyshev series, batched toy
datasets of the Gaussian, and the mixture at 1e8 events.  A sixth, a
Johnson S_U peak over an exponential background, exercises the Johnson
density the paper adds to the built-in ones (Sec. 3), and a seventh, one
chi-square density, the "ChiSquarePdf" entry of its speed-up figure.
"""
from __future__ import annotations

import copy
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdatagen.so")

MASTER_SEED = 2003012875
KIND = {"gauss": 1, "exp": 2, "cheb": 3, "cb": 4, "argus": 5, "sum": 6, "prod": 7, "johnson": 8, "chi2": 9,
        "hypatia": 10}


def build() -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
           os.path.join(_HERE, "datagen.cpp"), "-o", LIB_PATH + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class DgNode(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("obs", ctypes.c_int32), ("n_param", ctypes.c_int32),
                ("p", ctypes.c_double * 12), ("n_child", ctypes.c_int32), ("child", ctypes.c_int32 * 8)]


class DgModel(ctypes.Structure):
    _fields_ = [("n_obs", ctypes.c_int32), ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4),
                ("n_node", ctypes.c_int32), ("node", DgNode * 16), ("root", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.dg_philox4x64.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint64), P(ctypes.c_uint64)]
        L.dg_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P(ctypes.c_double)]
        L.dg_generate.argtypes = [P(DgModel), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                  P(P(ctypes.c_double)), ctypes.c_int32]
        L.dg_generate.restype = ctypes.c_int64
        L.dg_generate_sets.argtypes = [P(DgModel), ctypes.c_int32, P(ctypes.c_int64), ctypes.c_uint64,
                                       ctypes.c_uint64, P(P(ctypes.c_double)), ctypes.c_int32]
        L.dg_generate_sets.restype = ctypes.c_int64
        _lib = L
    return _lib


def default_threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


def philox4x64(ctr, key):
    c = (ctypes.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(v) for v in key])
    o = (ctypes.c_uint64 * 4)()
    lib().dg_philox4x64(c, k, o)
    return [int(v) for v in o]


def uniforms(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    lib().dg_uniforms(seed, stream, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


# --------------------------------------------------------------------------
# Model specifications (neutral dicts)
# --------------------------------------------------------------------------

def param(name, value, lo, hi, free=True, jitter=None):
    """A parameter; `jitter` is the half-width used for seeded parameter
    points (default 10 % of |value|)."""
    d = {"name": name, "value": float(value), "lo": float(lo), "hi": float(hi), "free": bool(free)}
    if jitter is not None:
        d["jitter"] = float(jitter)
    return d


def gauss_spec(mu=0.3, sigma=1.5, lo=-10.0, hi=10.0, norm="analytic"):
    """Config 1: one Gaussian on x in [-10, 10]."""
    return {"obs": [{"name": "x", "lo": lo, "hi": hi}],
            "params": [param("mu", mu, lo, hi), param("sigma", sigma, 0.05, 10.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [0, 1], "norm": norm}],
            "root": 0}


def mixture_spec(f=0.2, mu=5.0, sigma=0.4, c=-0.7, lo=0.0, hi=10.0, norm="analytic"):
    """Config 2 / 5: f * Gauss(mu, sigma) + (1 - f) * Exp(c) on x in [0, 10];
    parameters (f, mu, sigma, c)."""
    return {"obs": [{"name": "x", "lo": lo, "hi": hi}],
            "params": [param("f", f, 0.0, 1.0), param("mu", mu, lo, hi),
                       param("sigma", sigma, 0.01, 5.0), param("c", c, -5.0, 5.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [1, 2], "norm": norm},
                      {"kind": "exp", "obs": 0, "params": [3], "norm": norm},
                      {"kind": "sum", "params": [0], "children": [0, 1]}],
            "root": 2}


def johnson_spec(f=0.3, mu=5.28, lam=0.02, gam=-0.5, delta=1.5, c=-1.5, lo=5.0, hi=5.6, norm="analytic"):
    """f * Johnson S_U(m; mu, lambda, gamma, delta) + (1 - f) * Exp(m; c) on
    m in [5.0, 5.6]: a skewed mass peak over a falling background, the use
    the Johnson density is made for.  Parameters (f, mu, lambda, gamma,
    delta, c); seeded points jitter them by a fraction of the peak's scale."""
    return {"obs": [{"name": "m", "lo": lo, "hi": hi}],
            "params": [param("f", f, 0.0, 1.0, jitter=0.03), param("mu", mu, lo, hi, jitter=0.002),
                       param("lambda", lam, 1e-4, 1.0, jitter=0.002), param("gamma", gam, -10.0, 10.0, jitter=0.05),
                       param("delta", delta, 0.05, 20.0, jitter=0.15), param("c", c, -10.0, 10.0, jitter=0.15)],
            "nodes": [{"kind": "johnson", "obs": 0, "params": [1, 2, 3, 4], "norm": norm},
                      {"kind": "exp", "obs": 0, "params": [5], "norm": norm},
                      {"kind": "sum", "params": [0], "children": [0, 1]}],
            "root": 2}


def johnson_single_spec(mu=5.28, lam=0.02, gam=-0.5, delta=1.5, lo=5.0, hi=5.6, norm="analytic"):
    """The Johnson S_U peak of johnson_spec() alone; parameters (mu, lambda,
    gamma, delta)."""
    s = johnson_spec(mu=mu, lam=lam, gam=gam, delta=delta, lo=lo, hi=hi, norm=norm)
    return {"obs": s["obs"], "params": s["params"][1:5],
            "nodes": [{"kind": "johnson", "obs": 0, "params": [0, 1, 2, 3], "norm": norm}], "root": 0}


def chi2_spec(nu=5.0, lo=0.0, hi=40.0, norm="analytic"):
    """One chi-square density with nu degrees of freedom on x in [0, 40]
    (the "ChiSquarePdf" model of the paper's speed-up figure)."""
    return {"obs": [{"name": "x", "lo": lo, "hi": hi}],
            "params": [param("nu", nu, 0.1, 200.0)],
            "nodes": [{"kind": "chi2", "obs": 0, "params": [0], "norm": norm}],
            "root": 0}


def cheb_coefficients(seed: int, order: int = 4, lo: float = -1.0, hi: float = 1.0,
                      min_density: float = 0.05, max_tries: int = 1000) -> np.ndarray:
    """Chebyshev coefficients a_1..a_K ~ U[-0.3, 0.3], redrawn from the next
    stream until 1 + sum a_k T_k stays >= min_density on a 10001-point grid."""
    grid = np.linspace(-1.0, 1.0, 10001)
    for t in range(max_tries):
        a = -0.3 + 0.6 * uniforms(seed, 1000 + t, order)
        val = np.polynomial.chebyshev.chebval(grid, np.concatenate([[1.0], a]))
        if val.min() >= min_density:
            return a
    raise RuntimeError("no admissible Chebyshev coefficients")


def cb_argus_cheb_spec(cheb=(0.0, 0.0, 0.0, 0.0), f=0.1, m0=5.28, sigma=0.003, alpha=1.5, n=3.0,
                       am0=5.29, ac=-20.0, norm="gl256"):
    """Config 3: [f CB(m; m0, sigma, alpha, n) + (1-f) ARGUS(m; am0, ac)] x
    Cheb_4(y) on m in [5.20, 5.30], y in [-1, 1].  Parameters
    (f, m0, sigma, alpha, n, am0, ac, a1..a4); n and am0 fixed -> 9 free."""
    ps = [param("f", f, 0.0, 1.0, jitter=0.1 * f), param("cb_m0", m0, 5.20, 5.30, jitter=0.1 * sigma),
          param("cb_sigma", sigma, 1e-4, 0.05, jitter=0.1 * sigma),
          param("cb_alpha", alpha, 0.1, 10.0, jitter=0.1 * alpha), param("cb_n", n, 1.05, 50.0, free=False),
          param("ar_m0", am0, 5.2001, 6.0, free=False), param("ar_c", ac, -200.0, 0.0, jitter=0.1 * abs(ac))]
    for k, a in enumerate(cheb):
        ps.append(param(f"a{k + 1}", a, -1.0, 1.0))
    return {"obs": [{"name": "m", "lo": 5.20, "hi": 5.30}, {"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": ps,
            "nodes": [{"kind": "cb", "obs": 0, "params": [1, 2, 3, 4], "norm": norm},
                      {"kind": "argus", "obs": 0, "params": [5, 6], "norm": norm},
                      {"kind": "sum", "params": [0], "children": [0, 1]},
                      {"kind": "cheb", "obs": 1, "params": [7, 8, 9, 10], "norm": norm},
                      {"kind": "prod", "children": [2, 3]}],
            "root": 4}


def with_values(spec: dict, theta) -> dict:
    s = copy.deepcopy(spec)
    for p, v in zip(s["params"], theta):
        p["value"] = float(v)
    return s


def theta_of(spec: dict) -> np.ndarray:
    return np.array([p["value"] for p in spec["params"]], dtype=np.float64)


def _dg_model(spec: dict, theta=None) -> DgModel:
    th = theta_of(spec) if theta is None else np.asarray(theta, dtype=np.float64)
    m = DgModel()
    m.n_obs = len(spec["obs"])
    for k, o in enumerate(spec["obs"]):
        m.lo[k], m.hi[k] = o["lo"], o["hi"]
    m.n_node = len(spec["nodes"])
    for k, nd in enumerate(spec["nodes"]):
        d = m.node[k]
        d.kind = KIND[nd["kind"]]
        d.obs = int(nd.get("obs", -1))
        ps = nd.get("params", [])
        cs = nd.get("children", [])
        vals = [th[pi] for pi in ps]
        if nd["kind"] == "sum" and len(ps) == len(cs):
            # a sum of yields: the children are drawn with probabilities nu_j / sum nu
            tot = sum(vals)
            vals = [v / tot for v in vals[:-1]]
        d.n_param = len(vals)
        for j, v in enumerate(vals):
            d.p[j] = v
        d.n_child = len(cs)
        for j, c in enumerate(cs):
            d.child[j] = c
    m.root = spec["root"]
    return m


def generate(spec: dict, n: int, seed: int, stream: int = 0, theta=None, threads: int | None = None):
    """n events drawn from the model at `theta` (default: the spec values);
    returns a list of float64 columns (one per observable)."""
    m = _dg_model(spec, theta)
    cols = [np.empty(n, dtype=np.float64) for _ in spec["obs"]]
    arr = (ctypes.POINTER(ctypes.c_double) * 4)()
    for k, c in enumerate(cols):
        arr[k] = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    bad = lib().dg_generate(ctypes.byref(m), seed, stream, n, arr, threads or default_threads())
    if bad:
        raise RuntimeError(f"{bad} events could not be sampled")
    return cols


def generate_sets(spec: dict, thetas: np.ndarray, offsets: np.ndarray, seed: int, stream_base: int,
                  threads: int | None = None, out=None):
    """Concatenated datasets: set s is drawn at thetas[s] into
    [offsets[s], offsets[s+1])."""
    n_sets = len(offsets) - 1
    models = (DgModel * n_sets)()
    for s in range(n_sets):
        models[s] = _dg_model(spec, thetas[s])
    total = int(offsets[-1])
    cols = out if out is not None else [np.empty(total, dtype=np.float64) for _ in spec["obs"]]
    arr = (ctypes.POINTER(ctypes.c_double) * 4)()
    for k, c in enumerate(cols):
        arr[k] = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    bad = lib().dg_generate_sets(models, n_sets, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 seed, stream_base, arr, threads or default_threads())
    if bad:
        raise RuntimeError(f"{bad} events could not be sampled")
    return cols


def jittered_points(theta_true, n_points: int, seed: int, stream: int = 7, rel: float = 0.1,
                    free=None, widths=None) -> np.ndarray:
    """theta_true + w * U(-1, 1) per component with w = rel * |theta_true|
    unless explicit half-widths are given (fixed components kept)."""
    th = np.asarray(theta_true, dtype=np.float64)
    w = rel * np.abs(th) if widths is None else np.asarray(widths, dtype=np.float64)
    u = uniforms(seed, stream, n_points * len(th)).reshape(n_points, len(th))
    pts = th[None, :] + w[None, :] * (2.0 * u - 1.0)
    if free is not None:
        fixed = ~np.asarray(free, dtype=bool)
        pts[:, fixed] = th[fixed]
    return pts


def toy_sizes(n_sets: int, seed: int, lo: int = 1000, hi: int = 200000, stream: int = 3) -> np.ndarray:
    u = uniforms(seed, stream, n_sets)
    return lo + np.minimum((u * (hi - lo + 1)).astype(np.int64), hi - lo)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def binned(x: np.ndarray, lo: float, hi: float, n_bins: int):
    """A binned dataset: the centres of n_bins equal bins of [lo, hi] and the
    number of events of x in each (as float64 weights)."""
    counts, edges = np.histogram(x, bins=n_bins, range=(lo, hi))
    return 0.5 * (edges[:-1] + edges[1:]), counts.astype(np.float64)


def signed_weights(n: int, seed: int, lo: float = -0.5, hi: float = 1.5) -> np.ndarray:
    """n weights uniform in [lo, hi] (either sign, as sWeights have)."""
    return lo + (hi - lo) * uniforms(seed, 11, n)


HF_SEED = MASTER_SEED + 8000


def hf_workload(n_bins: int = 2_000_000, n_samples: int = 4, n_histosys: int = 16, n_normsys: int = 4,
                n_points: int = 4, seed: int = HF_SEED) -> dict:
    """A binned template model of HistFactory type: n_bins bins in channels
    of 100; sample 0 a Gaussian peak per channel (signal), the others
    exponentially falling backgrounds; histosys h on sample h % S with up and
    down templates tilted by +-(2..10) % across the channel; normsys k on
    sample k % S with hi = 1 + U[0.02, 0.1], lo = 1 - U[0.02, 0.1];
    normfactors mu_sig (sample 0) and mu_bkg (sample 1), unconstrained; the
    alphas constrained.  Counts are Poisson with means sum_s T_sb (all
    modifiers at their nominal values), from numpy's Philox generator.
    Parameter points: mu's jittered by 10 %, alphas uniform in [-1.5, 1.5]."""
    S, H, K = n_samples, n_histosys, n_normsys
    x = (np.arange(n_bins) % 100 + 0.5) / 100.0
    ch = np.arange(n_bins) // 100
    u = uniforms(seed, 21, 4 * S + 3 * H + 2 * K + 16)
    nominal = []
    for s in range(S):
        if s == 0:
            nominal.append(20.0 * np.exp(-0.5 * ((x - 0.5) / 0.08) ** 2))
        else:
            tau = 0.2 + 0.6 * u[s]
            amp = 50.0 + 100.0 * u[S + s]
            nominal.append(amp * np.exp(-x / tau) * (1.0 + 0.1 * np.cos(0.37 * ch)) + 1.0)
    up, down, mods = [], [], []
    params = [param("mu_sig", 1.0, 0.0, 10.0), param("mu_bkg", 1.0, 0.0, 10.0)]
    for k in range(2):
        params[k]["constrained"] = False
    mods.append({"type": "normfactor", "sample": 0, "param": 0})
    mods.append({"type": "normfactor", "sample": 1 % S, "param": 1})
    for h in range(H):
        s = h % S
        e_up, e_dn = 0.02 + 0.08 * u[2 * S + h], 0.02 + 0.08 * u[2 * S + H + h]
        tilt = (x - 0.5) * (1.0 if u[2 * S + 2 * H + h] < 0.5 else -1.0)
        up.append(nominal[s] * (1.0 + e_up * (1.0 + tilt)))
        down.append(nominal[s] * (1.0 - e_dn * (1.0 - tilt)))
        p = len(params)
        params.append(param(f"alpha_h{h}", 0.0, -5.0, 5.0, jitter=1.5))
        params[p]["constrained"] = True
        mods.append({"type": "histosys", "sample": s, "param": p})
    for k in range(K):
        p = len(params)
        params.append(param(f"alpha_n{k}", 0.0, -5.0, 5.0, jitter=1.5))
        params[p]["constrained"] = True
        mods.append({"type": "normsys", "sample": k % S, "param": p,
                     "hi": 1.02 + 0.08 * u[2 * S + 3 * H + k], "lo": 0.98 - 0.08 * u[2 * S + 3 * H + K + k]})
    spec = {"n_bins": n_bins, "samples": [f"s{s}" for s in range(S)], "params": params, "modifiers": mods}
    lam = np.sum(nominal, axis=0)
    counts = np.random.Generator(np.random.Philox(key=seed)).poisson(lam).astype(np.float64)
    theta = theta_of(spec)
    pts = jittered_points(theta, n_points, seed + 1, widths=jitter_widths(spec))
    return {"spec": spec, "counts": counts, "nominal": nominal, "up": up, "down": down,
            "theta": theta, "points": pts, "seed": seed}


def data_seed(config: int) -> int:
    return MASTER_SEED + 1000 * config


def free_mask(spec: dict) -> np.ndarray:
    return np.array([p.get("free", True) for p in spec["params"]], dtype=bool)


def jitter_widths(spec: dict, rel: float = 0.1) -> np.ndarray:
    return np.array([p.get("jitter", rel * abs(p["value"])) for p in spec["params"]], dtype=np.float64)


def parameter_points(spec: dict, n_points: int, seed: int) -> np.ndarray:
    """Seeded points around the spec values; points at which a Chebyshev
    series would not stay positive (min < 0.02 on a grid) are redrawn from
    the next stream."""
    pts = np.empty((n_points, len(spec["params"])))
    grid = np.linspace(-1.0, 1.0, 2001)
    cheb_nodes = [nd for nd in spec["nodes"] if nd["kind"] == "cheb"]
    filled, stream = 0, 7
    while filled < n_points:
        cand = jittered_points(theta_of(spec), n_points, seed, stream=stream, free=free_mask(spec),
                               widths=jitter_widths(spec))
        for row in cand:
            ok = all(np.polynomial.chebyshev.chebval(grid, np.concatenate([[1.0], row[nd["params"]]])).min() >= 0.02
                     for nd in cheb_nodes)
            if ok and filled < n_points:
                pts[filled] = row
                filled += 1
        stream += 1
    return pts


def workload(config: int, n: int | None = None, threads: int | None = None) -> dict:
    """Spec, columns and parameter points of workload 1, 2, 3 or 5
    (optionally with a smaller event count n)."""
    seed = data_seed(config)
    if config == 1:
        spec = gauss_spec()
        N = 100_000 if n is None else n
        pts = 64
    elif config in (2, 5):
        spec = mixture_spec()
        N = (10_000_000 if config == 2 else 100_000_000) if n is None else n
        pts = 8 if config == 2 else 32
    elif config == 3:
        spec = cb_argus_cheb_spec(cheb=cheb_coefficients(seed))
        N = 50_000_000 if n is None else n
        pts = 8
    else:
        raise ValueError("use toys_workload() for the batched configuration")
    cols = generate(spec, N, seed, threads=threads)
    theta = theta_of(spec)
    points = parameter_points(spec, pts, seed + 1)
    return {"config": config, "spec": spec, "cols": cols, "n": N, "theta": theta, "points": points,
            "seed": seed}


JOHNSON_SEED = MASTER_SEED + 6000


def johnson_workload(n: int = 10_000_000, single: bool = False, n_points: int = 8,
                     threads: int | None = None, norm: str = "analytic") -> dict:
    """The Johnson S_U mixture of johnson_spec() (or its peak alone) with n
    events: data seed master + 6000, parameter-point seed one more."""
    spec = johnson_single_spec(norm=norm) if single else johnson_spec(norm=norm)
    cols = generate(spec, n, JOHNSON_SEED, threads=threads)
    return {"spec": spec, "cols": cols, "n": n, "theta": theta_of(spec),
            "points": parameter_points(spec, n_points, JOHNSON_SEED + 1), "seed": JOHNSON_SEED}


JIT_COMPOSITE_SEED = MASTER_SEED + 11000

# formula densities used as leaves of composite models (C syntax; x and p[k])
BREIT_WIGNER = "1.0/((x-p[0])*(x-p[0]) + 0.25*p[1]*p[1])"
GAUSS_FORMULA = "exp(-0.5*((x-p[0])/p[1])*((x-p[0])/p[1]))"
QUADRATIC = "1.0 + p[0]*x + p[1]*x*x"
POWER_EXP = "pow(x, p[0])*exp(p[1]*x)"


def jit_composite_spec(kind: str) -> dict:
    """Composite models with formula leaves ("jit" nodes), for one or two
    observables; the events of each come from a built-in model of similar
    shape (jit_composite_workload), which parity does not need to match.
      "bw_exp":     f BW(x; m, G) + (1 - f) Exp(x; c) on [0, 10]
      "three":      f1 formula-Gauss(x; mu1, s1) + f2 Gauss(x; mu2, s2)
                    + (1 - f1 - f2) quadratic(x; a, b) on [0, 10]
      "two_jit":    yields nu1 BW(x; m, G) + nu2 power-exp(x; k, c) on [0.5, 10]
      "prod":       power-exp(x; k, c) x Gauss(y; mu, s), x in [0.5, 10], y in [-5, 5]
      "narrow":     f formula-Gauss(x; mu, 0.02-wide) + (1 - f) Exp(x; c) on [0, 10]
    """
    x = {"name": "x", "lo": 0.0, "hi": 10.0}
    if kind == "bw_exp":
        return {"obs": [x],
                "params": [param("f", 0.3, 0.0, 1.0, jitter=0.05), param("m", 5.0, 0.0, 10.0, jitter=0.1),
                           param("G", 0.8, 0.01, 5.0, jitter=0.1), param("c", -0.7, -5.0, 5.0, jitter=0.1)],
                "nodes": [{"kind": "jit", "obs": 0, "params": [1, 2], "density": BREIT_WIGNER},
                          {"kind": "exp", "obs": 0, "params": [3], "norm": "analytic"},
                          {"kind": "sum", "params": [0], "children": [0, 1]}],
                "root": 2}
    if kind == "three":
        return {"obs": [x],
                "params": [param("f1", 0.3, 0.0, 1.0, jitter=0.05), param("f2", 0.2, 0.0, 1.0, jitter=0.05),
                           param("mu1", 3.0, 0.0, 10.0, jitter=0.1), param("s1", 0.6, 0.01, 5.0, jitter=0.05),
                           param("mu2", 7.0, 0.0, 10.0, jitter=0.1), param("s2", 0.4, 0.01, 5.0, jitter=0.05),
                           param("a", 0.05, -0.09, 1.0, jitter=0.02), param("b", 0.01, 0.0, 1.0, jitter=0.005)],
                "nodes": [{"kind": "jit", "obs": 0, "params": [2, 3], "density": GAUSS_FORMULA},
                          {"kind": "gauss", "obs": 0, "params": [4, 5], "norm": "analytic"},
                          {"kind": "jit", "obs": 0, "params": [6, 7], "density": QUADRATIC},
                          {"kind": "sum", "params": [0, 1], "children": [0, 1, 2]}],
                "root": 3}
    if kind == "two_jit":
        return {"obs": [{"name": "x", "lo": 0.5, "hi": 10.0}],
                "params": [param("nu1", 3000.0, 0.0, 1e6, jitter=300.0), param("nu2", 7000.0, 0.0, 1e6, jitter=500.0),
                           param("m", 5.0, 0.5, 10.0, jitter=0.1), param("G", 0.8, 0.01, 5.0, jitter=0.1),
                           param("k", 1.5, 0.0, 5.0, jitter=0.1), param("c", -0.7, -5.0, 5.0, jitter=0.1)],
                "nodes": [{"kind": "jit", "obs": 0, "params": [2, 3], "density": BREIT_WIGNER},
                          {"kind": "jit", "obs": 0, "params": [4, 5], "density": POWER_EXP},
                          {"kind": "sum", "params": [0, 1], "children": [0, 1]}],
                "root": 2}
    if kind == "prod":
        return {"obs": [{"name": "x", "lo": 0.5, "hi": 10.0}, {"name": "y", "lo": -5.0, "hi": 5.0}],
                "params": [param("k", 1.5, 0.0, 5.0, jitter=0.1), param("c", -0.7, -5.0, 5.0, jitter=0.1),
                           param("mu", 0.2, -5.0, 5.0, jitter=0.1), param("s", 1.2, 0.05, 5.0, jitter=0.1)],
                "nodes": [{"kind": "jit", "obs": 0, "params": [0, 1], "density": POWER_EXP},
                          {"kind": "gauss", "obs": 1, "params": [2, 3], "norm": "analytic"},
                          {"kind": "prod", "children": [0, 1]}],
                "root": 2}
    if kind == "narrow":
        return {"obs": [x],
                "params": [param("f", 0.2, 0.0, 1.0, jitter=0.03), param("mu", 5.0, 0.0, 10.0, jitter=0.005),
                           param("s", 0.02, 0.001, 5.0, jitter=0.002), param("c", -0.7, -5.0, 5.0, jitter=0.1)],
                "nodes": [{"kind": "jit", "obs": 0, "params": [1, 2], "density": GAUSS_FORMULA},
                          {"kind": "exp", "obs": 0, "params": [3], "norm": "analytic"},
                          {"kind": "sum", "params": [0], "children": [0, 1]}],
                "root": 2}
    raise ValueError(kind)


def jit_composite_workload(kind: str, n: int = 100_000, n_points: int = 3, threads: int | None = None) -> dict:
    """The model jit_composite_spec(kind), n events from a built-in model of
    similar shape (a Gaussian peak over an exponential, or a product of two
    Gaussians), and seeded parameter points around the spec values."""
    spec = jit_composite_spec(kind)
    seed = JIT_COMPOSITE_SEED + {"bw_exp": 0, "three": 1, "two_jit": 2, "prod": 3, "narrow": 4}[kind]
    if kind == "prod":
        src = {"obs": spec["obs"],
               "params": [param("a", 4.0, 0.5, 10.0), param("b", 2.0, 0.1, 10.0), param("mu", 0.2, -5, 5),
                          param("s", 1.2, 0.05, 5.0)],
               "nodes": [{"kind": "gauss", "obs": 0, "params": [0, 1], "norm": "analytic"},
                         {"kind": "gauss", "obs": 1, "params": [2, 3], "norm": "analytic"},
                         {"kind": "prod", "children": [0, 1]}],
               "root": 2}
    else:
        lo, hi = spec["obs"][0]["lo"], spec["obs"][0]["hi"]
        mu, sig = (5.0, 0.02) if kind == "narrow" else (5.0, 0.6)
        src = mixture_spec(f=0.3, mu=mu, sigma=sig, c=-0.3, lo=lo, hi=hi)
    cols = generate(src, n, seed, threads=threads)
    return {"spec": spec, "cols": cols, "n": n, "theta": theta_of(spec),
            "points": parameter_points(spec, n_points, seed + 1), "seed": seed}


def hypatia_spec(f=0.4, lo=5.20, hi=5.35):
    """f * Hypatia2(m; 5.28, 0.003, -2, 0.5, 0, 2, 3, 2.5, 4) + (1 - f) *
    Exp(m; -1.5) on m in [5.20, 5.35]: a B-mass-like peak with power-law
    tails on both sides (the use the two-sided Hypatia is made for) over a
    falling background.  Parameters (f, mu, sigma, lambda, zeta, beta, a_l,
    n_l, a_r, n_r, c), all free; seeded points jitter each by a few per cent
    of the scale it acts on."""
    sg = 0.003
    return {"obs": [{"name": "m", "lo": lo, "hi": hi}],
            "params": [param("f", f, 0.0, 1.0, jitter=0.02), param("mu", 5.28, lo, hi, jitter=0.05 * sg),
                       param("sigma", sg, 1e-5, 0.1, jitter=0.05 * sg), param("lambda", -2.0, -6.0, 6.0, jitter=0.1),
                       param("zeta", 0.5, 1e-3, 100.0, jitter=0.025), param("beta", 0.0, -500.0, 500.0, jitter=0.02 / sg),
                       param("a_l", 2.0, 0.05, 20.0, jitter=0.1), param("n_l", 3.0, 1.001, 100.0, jitter=0.15),
                       param("a_r", 2.5, 0.05, 20.0, jitter=0.125), param("n_r", 4.0, 1.001, 100.0, jitter=0.2),
                       param("c", -1.5, -50.0, 50.0, jitter=0.15)],
            "nodes": [{"kind": "hypatia", "obs": 0, "params": list(range(1, 10))},
                      {"kind": "exp", "obs": 0, "params": [10]},
                      {"kind": "sum", "params": [0], "children": [0, 1]}],
            "root": 2}


HYPATIA_SEED = MASTER_SEED + 10000


def hypatia_workload(n: int = 10_000_000, n_points: int = 4, threads: int | None = None) -> dict:
    """hypatia_spec() with n events: data seed master + 10000, parameter-point
    seed one more."""
    spec = hypatia_spec()
    cols = generate(spec, n, HYPATIA_SEED, threads=threads)
    return {"spec": spec, "cols": cols, "n": n, "theta": theta_of(spec),
            "points": parameter_points(spec, n_points, HYPATIA_SEED + 1), "seed": HYPATIA_SEED}


CHI2_SEED = MASTER_SEED + 7000


def chi2_workload(n: int = 10_000_000, n_points: int = 8, threads: int | None = None,
                  norm: str = "analytic") -> dict:
    """chi2_spec() with n events: data seed master + 7000, parameter-point
    seed one more."""
    spec = chi2_spec(norm=norm)
    cols = generate(spec, n, CHI2_SEED, threads=threads)
    return {"spec": spec, "cols": cols, "n": n, "theta": theta_of(spec),
            "points": parameter_points(spec, n_points, CHI2_SEED + 1), "seed": CHI2_SEED}


def toys_workload(n_sets: int = 4096, size_lo: int = 1000, size_hi: int = 200000,
                  threads: int | None = None) -> dict:
    """Config 4: n_sets Gaussian datasets on [-10, 10] with sizes uniform in
    [size_lo, size_hi] and truths (0.3, 1.5) jittered by +-10 %."""
    seed = data_seed(4)
    spec = gauss_spec()
    sizes = toy_sizes(n_sets, seed, size_lo, size_hi)
    offsets = np.zeros(n_sets + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    truths = jittered_points(theta_of(spec), n_sets, seed + 1)
    cols = generate_sets(spec, truths, offsets, seed, 4 << 32, threads=threads)
    return {"config": 4, "spec": spec, "cols": cols, "offsets": offsets, "sizes": sizes,
            "truths": truths, "theta_start": theta_of(spec), "seed": seed}

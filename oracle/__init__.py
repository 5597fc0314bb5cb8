"""Scalar FP64 reference evaluator of unbinned NLLs -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never links,
loads or calls it, and it shares no source with the GPU path.

The C++ code (``oracle.cpp``) evaluates the likelihood the classic way the
paper describes in Sec. 5.1: event by event, recursively through the
computation graph, with each leaf normalised over its observable range
(closed forms or 256-point Gauss-Legendre, Sec. 3).  This module only
marshals arguments through ctypes.

Models are given as the neutral JSON-like dict used by the input
generators (``datagen``): ``{"obs": [...], "params": [...], "nodes": [...],
"root": r}``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

MAX_OBS, MAX_PAR, MAX_NODE, NODE_PAR, NODE_CHILD = 4, 32, 16, 12, 8

KIND = {"gauss": 1, "exp": 2, "cheb": 3, "cb": 4, "argus": 5, "sum": 6, "prod": 7, "johnson": 8, "chi2": 9,
        "hypatia": 10}
NORM = {"analytic": 0, "gl256": 1, "gl256_single": 2}

OK, E_ARG, E_UNSUPPORTED, E_PARAM, E_DOMAIN, E_PDF = 0, -1, -2, -3, -4, -5
STATUS_NAME = {OK: "ok", E_ARG: "arg", E_UNSUPPORTED: "unsupported", E_PARAM: "param_range",
               E_DOMAIN: "domain", E_PDF: "invalid_pdf"}


def build() -> str:
    """Compile liboracle.so with g++ -O2 (no fast-math)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
           os.path.join(_HERE, "oracle.cpp"), "-o", LIB_PATH + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class OrcNode(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("obs", ctypes.c_int32), ("n_param", ctypes.c_int32),
                ("param", ctypes.c_int32 * NODE_PAR), ("n_child", ctypes.c_int32),
                ("child", ctypes.c_int32 * NODE_CHILD), ("norm", ctypes.c_int32)]


class OrcModel(ctypes.Structure):
    _fields_ = [("n_obs", ctypes.c_int32), ("lo", ctypes.c_double * MAX_OBS),
                ("hi", ctypes.c_double * MAX_OBS), ("n_param", ctypes.c_int32),
                ("par_lo", ctypes.c_double * MAX_PAR), ("par_hi", ctypes.c_double * MAX_PAR),
                ("par_free", ctypes.c_uint8 * MAX_PAR), ("n_node", ctypes.c_int32),
                ("node", OrcNode * MAX_NODE), ("root", ctypes.c_int32),
                ("extended", ctypes.c_int32), ("yield_param", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        pd, pm = P(d), P(OrcModel)
        ppd = P(pd)
        L.orc_check_model.argtypes = [pm]
        L.orc_leaf_norm.argtypes = [pm, i32, pd, pd, pd]
        L.orc_log_density.argtypes = [pm, pd, pd, pd, pd]
        L.orc_nll.argtypes = [pm, ppd, i64, pd, i32, pd, pd, pd]
        L.orc_nll_batched.argtypes = [pm, ppd, P(i64), i32, pd, i32, pd, pd, P(i32)]
        L.orc_gd_fit.argtypes = [pm, ppd, i64, pd, i32, d, i32, pd, pd, pd, pd]
        L.orc_gd_fit_accept.argtypes = [pm, ppd, i64, pd, i32, d, d, i32, pd, pd, pd, pd]
        L.orc_nll_weighted.argtypes = [pm, ppd, pd, i64, pd, i32, pd, pd, pd, pd]
        L.orc_gd_fit_weighted.argtypes = [pm, ppd, pd, i64, pd, i32, d, i32, pd, pd, pd, pd]
        L.orc_nll_bhhh.argtypes = [pm, ppd, i64, pd, i32, pd, pd, pd]
        L.orc_bhhh_fit.argtypes = [pm, ppd, i64, pd, i32, d, i32, pd, pd, pd, pd]
        L.orc_gd_fit_batched.argtypes = [pm, ppd, P(i64), i32, pd, i32, d, i32, pd, pd, P(i32)]
        L.orc_gl_rule.argtypes = [i32, pd, pd]
        L.orc_log_bessel_k.argtypes = [d, d, pd]
        L.orc_log_bessel_k.restype = ctypes.c_int
        for f in ("orc_check_model", "orc_leaf_norm", "orc_log_density", "orc_nll",
                  "orc_nll_batched", "orc_gd_fit", "orc_gd_fit_accept", "orc_gd_fit_batched", "orc_gl_rule"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def model_from_spec(spec: dict) -> OrcModel:
    m = OrcModel()
    obs, params, nodes = spec["obs"], spec["params"], spec["nodes"]
    m.n_obs = len(obs)
    for k, o in enumerate(obs):
        m.lo[k], m.hi[k] = float(o["lo"]), float(o["hi"])
    m.n_param = len(params)
    for k, p in enumerate(params):
        m.par_lo[k], m.par_hi[k] = float(p["lo"]), float(p["hi"])
        m.par_free[k] = 1 if p.get("free", True) else 0
    m.n_node = len(nodes)
    for k, nd in enumerate(nodes):
        n = m.node[k]
        n.kind = KIND[nd["kind"]]
        n.obs = int(nd.get("obs", -1))
        ps, cs = list(nd.get("params", [])), list(nd.get("children", []))
        n.n_param, n.n_child = len(ps), len(cs)
        for j, v in enumerate(ps):
            n.param[j] = int(v)
        for j, v in enumerate(cs):
            n.child[j] = int(v)
        n.norm = NORM[nd.get("norm", "analytic")]
    m.root = int(spec["root"])
    m.extended = 1 if spec.get("extended", False) else 0
    m.yield_param = int(spec.get("yield_param", -1))
    return m


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cols(cols):
    cols = [np.ascontiguousarray(c, dtype=np.float64) for c in cols]
    arr = (ctypes.POINTER(ctypes.c_double) * MAX_OBS)()
    for k, c in enumerate(cols):
        arr[k] = _dptr(c)
    return cols, arr


class Oracle:
    """Thin ctypes front end over one model."""

    def __init__(self, spec: dict):
        self.spec = spec
        self.m = model_from_spec(spec)
        self.n_param = len(spec["params"])
        st = lib().orc_check_model(ctypes.byref(self.m))
        if st != OK:
            raise ValueError(f"oracle rejects model: {STATUS_NAME.get(st, st)}")

    def theta0(self) -> np.ndarray:
        return np.array([p["value"] for p in self.spec["params"]], dtype=np.float64)

    def leaf_norm(self, node: int, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        Z = ctypes.c_double()
        dZ = np.zeros(self.n_param)
        st = lib().orc_leaf_norm(ctypes.byref(self.m), node, _dptr(th), ctypes.byref(Z), _dptr(dZ))
        return st, Z.value, dZ

    def log_density(self, x, theta):
        xv = np.ascontiguousarray(x, dtype=np.float64)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        lp = ctypes.c_double()
        d = np.zeros(self.n_param)
        st = lib().orc_log_density(ctypes.byref(self.m), _dptr(xv), _dptr(th), ctypes.byref(lp), _dptr(d))
        return st, lp.value, d

    def nll(self, cols, theta, threads: int = 1, grad: bool = True, stats: bool = False, weights=None):
        """weights (optional, one per event): the weighted NLL -sum w_i log p_i."""
        keep, arr = _cols(cols)
        n = len(keep[0])
        th = np.ascontiguousarray(theta, dtype=np.float64)
        out = ctypes.c_double()
        g = np.zeros(self.n_param)
        s = np.zeros(self.n_param + 1)
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.float64)
            assert len(w) == n
            st = lib().orc_nll_weighted(ctypes.byref(self.m), arr, _dptr(w), n, _dptr(th), threads,
                                        ctypes.byref(out), _dptr(g) if grad else None,
                                        _dptr(s) if stats else None, None)
        else:
            st = lib().orc_nll(ctypes.byref(self.m), arr, n, _dptr(th), threads, ctypes.byref(out),
                               _dptr(g) if grad else None, _dptr(s) if stats else None)
        res = (st, out.value, g if grad else None)
        return res + ((s,) if stats else ())

    def nll_batched(self, cols, offsets, theta, threads: int = 1, grad: bool = True):
        keep, arr = _cols(cols)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n_sets = len(off) - 1
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(n_sets, self.n_param)
        nll = np.zeros(n_sets)
        g = np.zeros((n_sets, self.n_param))
        status = np.zeros(n_sets, dtype=np.int32)
        st = lib().orc_nll_batched(ctypes.byref(self.m), arr, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   n_sets, _dptr(th), threads, _dptr(nll), _dptr(g) if grad else None,
                                   status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return st, nll, (g if grad else None), status

    def gd_fit(self, cols, theta, n_steps: int, eta: float = 1.0, threads: int = 1, trace: bool = False,
               weights=None, accept_ulps=None):
        """Gradient descent (status, theta, NLL, gradient, final step[, trace]).
        accept_ulps: acceptance slack in ulps of the accepted NLL (default 4;
        0 is the literal no-increase rule)."""
        keep, arr = _cols(cols)
        n = len(keep[0])
        th = np.array(theta, dtype=np.float64)
        out = ctypes.c_double()
        eta_out = ctypes.c_double()
        g = np.zeros(self.n_param)
        tr = np.zeros((max(n_steps, 1), self.n_param + 1))
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.float64)
            assert len(w) == n
            st = lib().orc_gd_fit_weighted(ctypes.byref(self.m), arr, _dptr(w), n, _dptr(th), n_steps, eta,
                                           threads, ctypes.byref(out), _dptr(g), ctypes.byref(eta_out),
                                           _dptr(tr) if trace else None)
        elif accept_ulps is not None:
            st = lib().orc_gd_fit_accept(ctypes.byref(self.m), arr, n, _dptr(th), n_steps, eta,
                                         float(accept_ulps), threads, ctypes.byref(out), _dptr(g),
                                         ctypes.byref(eta_out), _dptr(tr) if trace else None)
        else:
            st = lib().orc_gd_fit(ctypes.byref(self.m), arr, n, _dptr(th), n_steps, eta, threads,
                                  ctypes.byref(out), _dptr(g), ctypes.byref(eta_out),
                                  _dptr(tr) if trace else None)
        res = (st, th, out.value, g, eta_out.value)
        return res + ((tr[:n_steps],) if trace else ())

    def nll_bhhh(self, cols, theta, threads: int = 1):
        """(status, NLL, gradient, BHHH matrix sum_i s_i s_i^T)."""
        keep, arr = _cols(cols)
        n = len(keep[0])
        th = np.ascontiguousarray(theta, dtype=np.float64)
        out = ctypes.c_double()
        g = np.zeros(self.n_param)
        B = np.zeros((self.n_param, self.n_param))
        st = lib().orc_nll_bhhh(ctypes.byref(self.m), arr, n, _dptr(th), threads, ctypes.byref(out), _dptr(g),
                                _dptr(B))
        return st, out.value, g, B

    def bhhh_fit(self, cols, theta, n_steps: int, lam: float = 1e-3, threads: int = 1, trace: bool = False):
        """Damped BHHH fit: (status, theta, NLL, gradient, final damping[, trace])."""
        keep, arr = _cols(cols)
        n = len(keep[0])
        th = np.array(theta, dtype=np.float64)
        out = ctypes.c_double()
        lam_out = ctypes.c_double()
        g = np.zeros(self.n_param)
        tr = np.zeros((max(n_steps, 1), self.n_param + 1))
        st = lib().orc_bhhh_fit(ctypes.byref(self.m), arr, n, _dptr(th), n_steps, lam, threads,
                                ctypes.byref(out), _dptr(g), ctypes.byref(lam_out), _dptr(tr) if trace else None)
        res = (st, th, out.value, g, lam_out.value)
        return res + ((tr[:n_steps],) if trace else ())

    def gd_fit_batched(self, cols, offsets, theta, n_steps: int, eta: float = 1.0, threads: int = 1):
        keep, arr = _cols(cols)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n_sets = len(off) - 1
        th = np.array(theta, dtype=np.float64).reshape(n_sets, self.n_param).copy()
        nll = np.zeros(n_sets)
        g = np.zeros((n_sets, self.n_param))
        status = np.zeros(n_sets, dtype=np.int32)
        st = lib().orc_gd_fit_batched(ctypes.byref(self.m), arr, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      n_sets, _dptr(th), n_steps, eta, threads, _dptr(nll), _dptr(g),
                                      status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return st, th, nll, g, status


def log_bessel_k(nu: float, z: float) -> float:
    out = ctypes.c_double()
    if lib().orc_log_bessel_k(ctypes.c_double(nu), ctypes.c_double(z), ctypes.byref(out)) != OK:
        raise ValueError("z must be positive")
    return out.value


def gl_rule(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    st = lib().orc_gl_rule(n, _dptr(x), _dptr(w))
    if st != OK:
        raise ValueError("bad rule size")
    return x, w

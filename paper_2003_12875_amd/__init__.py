"""nllmi: batched unbinned negative log-likelihoods on AMD MI355X (gfx950).

Thin Python front end of ``libnllmi.so`` (C ABI in ``include/nll.h``):
argument marshalling only -- every step of the likelihood runs in the HIP
kernels.  PyTorch provides device memory (tensors) and streams.

    model = Model.from_spec(spec)          # PDF graph (see ``Model.from_spec``)
    model.set_data([x_tensor])             # SoA float64 columns on the GPU
    nll, grad = model.eval_grad(theta)     # one fused pass
    nll = NLL.apply(theta, model)          # autograd: backward uses the same pass

Reference: S. Hageboeck, "A Faster, More Intuitive RooFit" (arXiv:2003.12875):
the computation graph of Sec. 1, the batched likelihood evaluation of
Sec. 5, the built-in densities of Sec. 3.
"""
from __future__ import annotations

import ctypes
import os

from ._native import (HF_MODIFIER, HFDesc, HFModifier, JitDesc, MAX_NODE_CHILDREN, MAX_NODE_PARAMS, NLLError, NodeDesc,
                      ModelDesc, Schedule, Info,
                      STATUS, check, lib, LIB_PATH)

KIND = {"gauss": 1, "exp": 2, "cheb": 3, "cb": 4, "argus": 5, "sum": 6, "prod": 7, "johnson": 8, "chi2": 9,
        "hypatia": 10, "jit": 11}
NORM = {"analytic": 0, "gl256": 1, "gl256_single": 2}
PRECISION = {"fp64": 0, "fp32c": 1}

__all__ = ["Model", "NLL", "NLLError", "STATUS", "lib", "LIB_PATH"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_tensor(t, dtype, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t, dtype=dtype)
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if t.device != device:
        t = t.to(device)
    return t.contiguous()


def _buf(t, dtype, device, numel, name):
    """A caller-supplied buffer the library reads or writes: checked for
    type, device, contiguity and size (the C ABI takes bare pointers)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor on {device}")
    if t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return t


class Model:
    """One likelihood model on one device (``nll_model``)."""

    def __init__(self, desc_args: dict, device: int = 0):
        torch = _torch()
        self.device = torch.device("cuda", device)
        self.n_param = desc_args["n_param"]
        self.n_obs = desc_args["n_obs"]
        self._keep = desc_args["keep"]
        d = desc_args["desc"]
        d.device = device
        d.stream = ctypes.c_void_p(self._stream())
        handle = ctypes.c_void_p()
        check(lib().nll_create_model(ctypes.byref(d), ctypes.byref(handle)), "nll_create_model")
        self._h = handle
        self._cols = None
        self.n_events = -1

    # -- construction ------------------------------------------------------
    @classmethod
    def from_spec(cls, spec: dict, precision: str = "fp64", device: int = 0) -> "Model":
        """Build from a graph specification::

            {"obs": [{"name", "lo", "hi"}...],
             "params": [{"name", "value", "lo", "hi", "free"}...],
             "nodes": [{"kind": "gauss"|"exp"|"cheb"|"cb"|"argus"|"johnson"|"chi2"|
                                "hypatia"|"jit"|"sum"|"prod",
                        "obs": int, "params": [...], "children": [...],
                        "norm": "analytic"|"gl256"|"gl256_single",
                        "density": str (jit: a formula in x and p[k])}...],
             "root": int, "extended": bool, "yield_param": int}
        """
        obs, params, nodes = spec["obs"], spec["params"], spec["nodes"]
        n_obs, n_param, n_node = len(obs), len(params), len(nodes)
        lo = (ctypes.c_double * n_obs)(*[float(o["lo"]) for o in obs])
        hi = (ctypes.c_double * n_obs)(*[float(o["hi"]) for o in obs])
        plo = (ctypes.c_double * n_param)(*[float(p["lo"]) for p in params])
        phi = (ctypes.c_double * n_param)(*[float(p["hi"]) for p in params])
        pfree = (ctypes.c_uint8 * n_param)(*[1 if p.get("free", True) else 0 for p in params])
        nd = (NodeDesc * n_node)()
        dens = []  # the formulas' bytes, alive until the model is created
        for i, n in enumerate(nodes):
            ps, cs = list(n.get("params", [])), list(n.get("children", []))
            if len(ps) > MAX_NODE_PARAMS or len(cs) > MAX_NODE_CHILDREN:
                raise NLLError(-1, "node has too many parameters or children")
            nd[i].kind = KIND[n["kind"]]
            nd[i].obs = int(n.get("obs", -1))
            nd[i].n_param = len(ps)
            nd[i].n_child = len(cs)
            for j, v in enumerate(ps):
                nd[i].param[j] = int(v)
            for j, v in enumerate(cs):
                nd[i].child[j] = int(v)
            nd[i].norm = NORM[n.get("norm", "analytic")]
            if n["kind"] == "jit":
                dens.append(str(n["density"]).encode())
                nd[i].density = dens[-1]
        d = ModelDesc()
        d.n_obs, d.obs_lo, d.obs_hi = n_obs, lo, hi
        d.n_param, d.param_lo, d.param_hi, d.param_free = n_param, plo, phi, pfree
        d.n_node, d.nodes, d.root = n_node, nd, int(spec["root"])
        d.precision = PRECISION[precision]
        d.extended = 1 if spec.get("extended", False) else 0
        d.yield_param = int(spec.get("yield_param", -1)) if spec.get("extended", False) else 0
        return cls({"desc": d, "n_param": n_param, "n_obs": n_obs, "keep": (lo, hi, plo, phi, pfree, nd, dens)},
                   device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().nll_destroy_model(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------
    def _stream(self) -> int:
        return _torch().cuda.current_stream(self.device).cuda_stream

    def _bind_stream(self):
        check(lib().nll_set_stream(self._h, ctypes.c_void_p(self._stream())), "nll_set_stream")

    # -- data ----------------------------------------------------------------
    def set_data(self, cols):
        """Attach SoA float64 event columns (device tensors, one per
        observable).  Validates every event against the observable ranges."""
        torch = _torch()
        cols = [_dev_tensor(c, torch.float64, self.device) for c in cols]
        if len(cols) != self.n_obs or len({c.numel() for c in cols}) != 1:
            raise NLLError(-1, "one column of equal length per observable required")
        n = cols[0].numel()
        arr = (ctypes.c_void_p * 4)(*[c.data_ptr() for c in cols])
        self._bind_stream()
        check(lib().nll_set_data(self._h, arr, ctypes.c_int64(n)), "nll_set_data")
        self._cols = cols
        self._weights = None
        self.n_events = n

    def set_weights(self, weights):
        """Attach per-event float64 weights (device tensor, one per event) to
        the attached data, or detach them with None: the NLL becomes
        -sum w_i log p(x_i) (a binned dataset: bin centres weighted by the
        counts).  Cleared by set_data."""
        ptr = None
        if weights is not None:
            weights = _dev_tensor(weights, _torch().float64, self.device)
            if weights.numel() != self.n_events:
                raise NLLError(-1, "one weight per attached event required")
            ptr = weights.data_ptr()
        self._bind_stream()
        check(lib().nll_set_weights(self._h, ptr), "nll_set_weights")
        self._weights = weights

    # -- evaluation ------------------------------------------------------------
    def eval(self, theta, out=None):
        torch = _torch()
        theta = _buf(_dev_tensor(theta, torch.float64, self.device), torch.float64, self.device, self.n_param, "theta")
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        _buf(out, torch.float64, self.device, 1, "out")
        self._bind_stream()
        check(lib().nll_eval(self._h, _ptr(theta), _ptr(out)), "nll_eval")
        return out

    def eval_grad(self, theta, out=None, grad=None):
        torch = _torch()
        theta = _buf(_dev_tensor(theta, torch.float64, self.device), torch.float64, self.device, self.n_param, "theta")
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        grad = torch.empty(self.n_param, dtype=torch.float64, device=self.device) if grad is None else grad
        _buf(out, torch.float64, self.device, 1, "out")
        _buf(grad, torch.float64, self.device, self.n_param, "grad")
        self._bind_stream()
        check(lib().nll_eval_grad(self._h, _ptr(theta), _ptr(out), _ptr(grad)), "nll_eval_grad")
        return out, grad

    def eval_batched(self, offsets, theta, grad: bool = True):
        torch = _torch()
        offsets = _dev_tensor(offsets, torch.int64, self.device)
        n_sets = offsets.numel() - 1
        theta = _dev_tensor(theta, torch.float64, self.device)
        _buf(theta, torch.float64, self.device, n_sets * self.n_param, "theta")
        nll = torch.empty(n_sets, dtype=torch.float64, device=self.device)
        g = torch.empty(n_sets, self.n_param, dtype=torch.float64, device=self.device) if grad else None
        status = torch.empty(n_sets, dtype=torch.int32, device=self.device)
        self._bind_stream()
        check(lib().nll_eval_batched(self._h, n_sets, _ptr(offsets), _ptr(theta), _ptr(nll), _ptr(g), _ptr(status)),
              "nll_eval_batched")
        return nll, g, status

    def eval_points(self, theta, grad: bool = True):
        """The attached dataset at each row of theta ([n_points, n_param]) in
        one pass (see nll_eval_points).  Returns (nll, grad or None, status)."""
        torch = _torch()
        theta = _dev_tensor(theta, torch.float64, self.device)
        n_points = theta.numel() // self.n_param if self.n_param else 0
        _buf(theta, torch.float64, self.device, n_points * self.n_param, "theta")
        nll = torch.empty(n_points, dtype=torch.float64, device=self.device)
        g = torch.empty(n_points, self.n_param, dtype=torch.float64, device=self.device) if grad else None
        status = torch.empty(n_points, dtype=torch.int32, device=self.device)
        self._bind_stream()
        check(lib().nll_eval_points(self._h, n_points, _ptr(theta), _ptr(nll), _ptr(g), _ptr(status)),
              "nll_eval_points")
        return nll, g, status

    def fit_batched(self, offsets, theta, n_steps: int, eta: float = 1.0, out=None):
        """Gradient-descent fits of every set (see nll_fit_batched).  Returns
        (theta, nll, grad, status) at the last accepted points."""
        torch = _torch()
        offsets = _dev_tensor(offsets, torch.int64, self.device)
        n_sets = offsets.numel() - 1
        if out is None:
            th = _dev_tensor(theta, torch.float64, self.device).reshape(n_sets, self.n_param).clone()
            nll = torch.empty(n_sets, dtype=torch.float64, device=self.device)
            g = torch.empty(n_sets, self.n_param, dtype=torch.float64, device=self.device)
            status = torch.empty(n_sets, dtype=torch.int32, device=self.device)
        else:
            th, nll, g, status = out
            th.copy_(_dev_tensor(theta, torch.float64, self.device).reshape(n_sets, self.n_param))
        _buf(th, torch.float64, self.device, n_sets * self.n_param, "theta")
        _buf(nll, torch.float64, self.device, n_sets, "nll")
        _buf(g, torch.float64, self.device, n_sets * self.n_param, "grad")
        _buf(status, torch.int32, self.device, n_sets, "status")
        self._bind_stream()
        check(lib().nll_fit_batched(self._h, n_sets, _ptr(offsets), _ptr(th), int(n_steps), float(eta), _ptr(nll),
                                    _ptr(g), _ptr(status)), "nll_fit_batched")
        return th, nll, g, status

    def fit(self, theta, n_steps: int, eta: float = 1.0, out=None):
        """Gradient-descent fit on all attached events (see nll_fit).  Pass
        out=(theta, nll, grad, status) tensors to reuse buffers (and the
        recorded graph) across calls."""
        torch = _torch()
        if out is None:
            th = _dev_tensor(theta, torch.float64, self.device).clone()
            nll = torch.empty(1, dtype=torch.float64, device=self.device)
            g = torch.empty(self.n_param, dtype=torch.float64, device=self.device)
            status = torch.empty(1, dtype=torch.int32, device=self.device)
        else:
            th, nll, g, status = out
            th.copy_(_dev_tensor(theta, torch.float64, self.device))
        _buf(th, torch.float64, self.device, self.n_param, "theta")
        _buf(nll, torch.float64, self.device, 1, "nll")
        _buf(g, torch.float64, self.device, self.n_param, "grad")
        _buf(status, torch.int32, self.device, 1, "status")
        self._bind_stream()
        check(lib().nll_fit(self._h, _ptr(th), int(n_steps), float(eta), _ptr(nll), _ptr(g), _ptr(status)), "nll_fit")
        return th, nll, g, status

    def eval_bhhh(self, theta):
        """(NLL, gradient, BHHH matrix [n_param, n_param]) at theta (see
        nll_eval_bhhh)."""
        torch = _torch()
        theta = _dev_tensor(theta, torch.float64, self.device)
        _buf(theta, torch.float64, self.device, self.n_param, "theta")
        nll = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty(self.n_param, dtype=torch.float64, device=self.device)
        B = torch.empty(self.n_param, self.n_param, dtype=torch.float64, device=self.device)
        self._bind_stream()
        check(lib().nll_eval_bhhh(self._h, _ptr(theta), _ptr(nll), _ptr(g), _ptr(B)), "nll_eval_bhhh")
        return nll, g, B

    def fit_bhhh(self, theta, n_steps: int, lam: float = 1e-3, out=None):
        """Damped BHHH fit on all attached events (see nll_fit_bhhh); the
        same buffers and return values as fit()."""
        torch = _torch()
        if out is None:
            th = _dev_tensor(theta, torch.float64, self.device).clone()
            nll = torch.empty(1, dtype=torch.float64, device=self.device)
            g = torch.empty(self.n_param, dtype=torch.float64, device=self.device)
            status = torch.empty(1, dtype=torch.int32, device=self.device)
        else:
            th, nll, g, status = out
            th.copy_(_dev_tensor(theta, torch.float64, self.device))
        _buf(th, torch.float64, self.device, self.n_param, "theta")
        _buf(nll, torch.float64, self.device, 1, "nll")
        _buf(g, torch.float64, self.device, self.n_param, "grad")
        _buf(status, torch.int32, self.device, 1, "status")
        self._bind_stream()
        check(lib().nll_fit_bhhh(self._h, _ptr(th), int(n_steps), float(lam), _ptr(nll), _ptr(g), _ptr(status)),
              "nll_fit_bhhh")
        return th, nll, g, status

    def sync(self) -> int:
        """Synchronise and return (and clear) the device status (0 = ok)."""
        st = ctypes.c_int32(0)
        self._bind_stream()
        lib().nll_sync(self._h, ctypes.byref(st))
        return st.value

    # -- schedule / info -------------------------------------------------------
    @property
    def schedule(self) -> dict:
        s = Schedule()
        check(lib().nll_get_schedule(self._h, ctypes.byref(s)), "nll_get_schedule")
        return {"unroll": s.unroll, "blocks_per_cu": s.blocks_per_cu, "tile_events": s.tile_events,
                "sets_blocks_per_cu": s.sets_blocks_per_cu, "sets_unroll": s.sets_unroll}

    def set_schedule(self, **kw):
        cur = self.schedule
        cur.update(kw)
        s = Schedule(cur["unroll"], cur["blocks_per_cu"], cur["tile_events"], cur["sets_blocks_per_cu"],
                     cur["sets_unroll"])
        check(lib().nll_set_schedule(self._h, ctypes.byref(s)), "nll_set_schedule")

    def autotune(self, theta, offsets=None):
        torch = _torch()
        self._bind_stream()
        if offsets is None:
            theta = _dev_tensor(theta, torch.float64, self.device)
            check(lib().nll_autotune(self._h, 1, 0, None, _ptr(theta)), "nll_autotune")
        else:
            offsets = _dev_tensor(offsets, torch.int64, self.device)
            n_sets = offsets.numel() - 1
            theta = _dev_tensor(theta, torch.float64, self.device).reshape(n_sets, self.n_param).contiguous()
            check(lib().nll_autotune(self._h, 2, n_sets, _ptr(offsets), _ptr(theta)), "nll_autotune")
        return self.schedule

    def set_option(self, option: str, value):
        """"graph": bool; "step_timing": False/0, True/1 (whole steps) or
        "kernel"/2 (the streaming kernel of each step)."""
        code = {"graph": 1, "step_timing": 2}[option]
        v = 2 if value == "kernel" else int(value)
        check(lib().nll_set_option(self._h, code, v), "nll_set_option")

    def step_times(self, cap: int = 1 << 16):
        """Per-step (or per-streaming-kernel) durations (ms) of the last fit
        run with step timing on."""
        buf = (ctypes.c_float * cap)()
        n = ctypes.c_int32(0)
        self._bind_stream()
        check(lib().nll_step_times(self._h, buf, cap, ctypes.byref(n)), "nll_step_times")
        return [buf[i] for i in range(n.value)]

    @property
    def info(self) -> dict:
        i = Info()
        check(lib().nll_get_info(self._h, ctypes.byref(i)), "nll_get_info")
        return {"variant": i.variant.decode(), "n_leaf": i.n_leaf, "n_term": i.n_term,
                "n_accumulators": i.n_accumulators, "precision": i.precision, "n_cu": i.n_cu,
                "n_events": i.n_events, "per_set_bytes": i.per_set_bytes}


class HFModel:
    """A binned template likelihood of HistFactory type on one device
    (``nll_hf_model``), bound to the current torch stream at creation.
    ``NLL.apply(theta, model)`` takes it as it takes a ``Model``."""

    def __init__(self, spec: dict, device: int = 0):
        """spec: {"n_bins": B, "samples": [names], "params": [{"name",
        "value", "lo", "hi", "free", "constrained", ("constraint_mean",
        "constraint_sigma")}...], "modifiers": [{"type":
        "normfactor"|"normsys"|"histosys", "sample": s, "param": p, ("hi",
        "lo" for normsys), ("interp": "poly6" for the smooth codes)}...]}"""
        torch = _torch()
        self.device = torch.device("cuda", device)
        params, mods = spec["params"], spec["modifiers"]
        P, M = len(params), len(mods)
        self.n_param, self.n_samples, self.n_bins = P, len(spec["samples"]), int(spec["n_bins"])
        self.n_histosys = sum(1 for m in mods if m["type"] == "histosys")
        plo = (ctypes.c_double * P)(*[float(p["lo"]) for p in params])
        phi = (ctypes.c_double * P)(*[float(p["hi"]) for p in params])
        pfree = (ctypes.c_uint8 * P)(*[1 if p.get("free", True) else 0 for p in params])
        pcon = (ctypes.c_uint8 * P)(*[1 if p.get("constrained", False) else 0 for p in params])
        pmean = (ctypes.c_double * P)(*[float(p.get("constraint_mean", 0.0)) for p in params])
        psig = (ctypes.c_double * P)(*[float(p.get("constraint_sigma", 1.0)) for p in params])
        md = (HFModifier * max(M, 1))()
        for i, m in enumerate(mods):
            md[i].type = HF_MODIFIER[m["type"]]
            md[i].sample, md[i].param = int(m["sample"]), int(m["param"])
            md[i].hi, md[i].lo = float(m.get("hi", 1.0)), float(m.get("lo", 1.0))
            md[i].interp = {"exp": 0, "linear": 0, "poly6": 1}[m.get("interp", "linear" if m["type"] == "histosys"
                                                                   else "exp")]
        d = HFDesc()
        d.n_bins, d.n_samples, d.n_param = self.n_bins, self.n_samples, P
        d.param_lo, d.param_hi, d.param_free, d.param_constrained = plo, phi, pfree, pcon
        d.param_mean, d.param_sigma = pmean, psig
        d.n_modifiers, d.modifiers = M, md
        d.device = device
        d.stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        handle = ctypes.c_void_p()
        check(lib().nll_hf_create(ctypes.byref(d), ctypes.byref(handle)), "nll_hf_create")
        self._h = handle
        self._keep = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().nll_hf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_data(self, counts, nominal, up=(), down=()):
        """counts[B], nominal: one [B] per sample, up/down: one [B] per
        histosys modifier in modifier order (float64, moved to the device)."""
        torch = _torch()
        f64 = torch.float64
        counts = _dev_tensor(counts, f64, self.device)
        nominal = [_dev_tensor(t, f64, self.device) for t in nominal]
        up = [_dev_tensor(t, f64, self.device) for t in up]
        down = [_dev_tensor(t, f64, self.device) for t in down]
        if len(nominal) != self.n_samples or len(up) != self.n_histosys or len(down) != self.n_histosys:
            raise NLLError(-1, "one nominal per sample and one up/down pair per histosys required")
        if any(t.numel() != self.n_bins for t in [counts, *nominal, *up, *down]):
            raise NLLError(-1, "every template needs n_bins entries")
        ptrs = lambda ts: (ctypes.c_void_p * max(len(ts), 1))(*[t.data_ptr() for t in ts])
        check(lib().nll_hf_set_data(self._h, counts.data_ptr(), ptrs(nominal), ptrs(up), ptrs(down)),
              "nll_hf_set_data")
        self._keep = (counts, nominal)  # borrowed by the library

    def eval(self, theta, out=None):
        torch = _torch()
        theta = _dev_tensor(theta, torch.float64, self.device)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        check(lib().nll_hf_eval(self._h, theta.data_ptr(), out.data_ptr(), None), "nll_hf_eval")
        return out

    def eval_grad(self, theta, out=None, grad=None):
        torch = _torch()
        theta = _dev_tensor(theta, torch.float64, self.device)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        grad = torch.empty(self.n_param, dtype=torch.float64, device=self.device) if grad is None else grad
        check(lib().nll_hf_eval(self._h, theta.data_ptr(), out.data_ptr(), grad.data_ptr()), "nll_hf_eval")
        return out, grad

    def set_staterror(self, samples, sigma):
        """Per-bin statistical parameters gamma_b shared by `samples` (sample
        indices), with Gaussian constraints of widths sigma[B] (relative
        statistical error per bin; <= 0: no parameter in that bin)."""
        torch = _torch()
        mask = 0
        for s in samples:
            mask |= 1 << int(s)
        sigma = _dev_tensor(sigma, torch.float64, self.device)
        if sigma.numel() != self.n_bins:
            raise NLLError(-1, "sigma needs n_bins entries")
        check(lib().nll_hf_set_staterror(self._h, mask, sigma.data_ptr()), "nll_hf_set_staterror")
        self._keep_sigma = sigma  # read on the stream; kept until that is done

    def set_shapesys(self, samples, sigma):
        """As set_staterror with Poisson constraints (shapesys): tau_b =
        1/sigma_b^2 auxiliary counts for the means gamma_b tau_b."""
        torch = _torch()
        mask = 0
        for s in samples:
            mask |= 1 << int(s)
        sigma = _dev_tensor(sigma, torch.float64, self.device)
        if sigma.numel() != self.n_bins:
            raise NLLError(-1, "sigma needs n_bins entries")
        check(lib().nll_hf_set_shapesys(self._h, mask, sigma.data_ptr()), "nll_hf_set_shapesys")
        self._keep_sigma = sigma

    def eval_stat(self, theta, gamma, grad=True):
        """(NLL, gradient or None, d NLL / d gamma or None) at theta and the
        per-bin statistical parameters gamma[B]."""
        torch = _torch()
        f64 = torch.float64
        theta = _dev_tensor(theta, f64, self.device)
        gamma = _dev_tensor(gamma, f64, self.device)
        if gamma.numel() != self.n_bins:
            raise NLLError(-1, "gamma needs n_bins entries")
        out = torch.empty(1, dtype=f64, device=self.device)
        g = torch.empty(self.n_param, dtype=f64, device=self.device) if grad else None
        gg = torch.empty(self.n_bins, dtype=f64, device=self.device) if grad else None
        check(lib().nll_hf_eval_stat(self._h, theta.data_ptr(), gamma.data_ptr(), out.data_ptr(),
                                     g.data_ptr() if grad else None, gg.data_ptr() if grad else None),
              "nll_hf_eval_stat")
        return out, g, gg

    def sync(self) -> int:
        st = ctypes.c_int32(0)
        check(lib().nll_hf_sync(self._h, ctypes.byref(st)), "nll_hf_sync")
        return st.value


class JITModel:
    """A density given as a C expression in x and p[k], compiled for the
    device at construction (``nll_jit_model``); bound to the current torch
    stream then.  ``NLL.apply(theta, model)`` takes it as it takes a
    ``Model``."""

    def __init__(self, density: str, lo: float, hi: float, params, device: int = 0):
        """params: [{"name", "value", "lo", "hi", "free"}...]."""
        torch = _torch()
        self.device = torch.device("cuda", device)
        P = len(params)
        self.n_param = P
        plo = (ctypes.c_double * P)(*[float(p["lo"]) for p in params])
        phi = (ctypes.c_double * P)(*[float(p["hi"]) for p in params])
        pfree = (ctypes.c_uint8 * P)(*[1 if p.get("free", True) else 0 for p in params])
        d = JitDesc()
        d.density = density.encode()
        d.obs_lo, d.obs_hi = float(lo), float(hi)
        d.n_param, d.param_lo, d.param_hi, d.param_free = P, plo, phi, pfree
        d.device = device
        d.stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        log = ctypes.create_string_buffer(8192)
        handle = ctypes.c_void_p()
        st = lib().nll_jit_create(ctypes.byref(d), ctypes.byref(handle), log, len(log))
        self.compile_log = log.value.decode(errors="replace")
        if st != 0:
            raise NLLError(st, "nll_jit_create" + (": " + self.compile_log if self.compile_log else ""))
        self._h = handle
        self._x = None
        self.n_events = -1

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().nll_jit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_data(self, x):
        torch = _torch()
        x = _dev_tensor(x, torch.float64, self.device)
        check(lib().nll_jit_set_data(self._h, x.data_ptr(), ctypes.c_int64(x.numel())), "nll_jit_set_data")
        self._x = x
        self.n_events = x.numel()

    def eval(self, theta, out=None):
        torch = _torch()
        theta = _dev_tensor(theta, torch.float64, self.device)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        check(lib().nll_jit_eval(self._h, theta.data_ptr(), out.data_ptr(), None), "nll_jit_eval")
        return out

    def eval_grad(self, theta, out=None, grad=None):
        torch = _torch()
        theta = _dev_tensor(theta, torch.float64, self.device)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        grad = torch.empty(self.n_param, dtype=torch.float64, device=self.device) if grad is None else grad
        check(lib().nll_jit_eval(self._h, theta.data_ptr(), out.data_ptr(), grad.data_ptr()), "nll_jit_eval")
        return out, grad

    def sync(self) -> int:
        st = ctypes.c_int32(0)
        check(lib().nll_jit_sync(self._h, ctypes.byref(st)), "nll_jit_sync")
        return st.value


def _nll_function():
    torch = _torch()

    class _NLL(torch.autograd.Function):
        """NLL(theta) with the analytic gradient of the same fused pass:
        forward calls nll_eval_grad and keeps the gradient; backward scales it."""

        @staticmethod
        def forward(ctx, theta, model):
            nll, grad = model.eval_grad(theta.detach())
            ctx.save_for_backward(grad)
            return nll[0]

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return g * grad, None

    return _NLL


class _LazyNLL:
    _fn = None

    def apply(self, theta, model):
        if _LazyNLL._fn is None:
            _LazyNLL._fn = _nll_function()
        return _LazyNLL._fn.apply(theta, model)


NLL = _LazyNLL()

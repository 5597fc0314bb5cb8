#!/usr/bin/env python3
"""Benchmark of the batched unbinned NLL on one MI355X.

Headline workload (one JSON line on stdout): 4096 toy datasets drawn from
the 1-D Gaussian model (x in [-10, 10], sizes uniform in [1000, 200000],
4.13e8 FP64 events in all, truths jittered by +-10 %), each fitted by
gradient descent from the nominal point.  One step = one gradient-descent
iteration of every toy on the device: NLL and the adjoint gradient of both
parameters of every toy in one persistent streaming launch over (toy, tile)
work items, then one finishing block per toy (its reduction, the update with
step halving, the next proposal's constants) -- all in the library's HIP
kernels, the K steps recorded once into a HIP graph and replayed.  `value`
is the whole job's throughput: events x steps over the wall time of one
replay of K steps (median of REPS replays, inputs resident in HBM).

Also reported, on the same GPU:
  * roofline     -- the dominant kernel (k_sets, the streaming launch of each
    step): algorithmic bytes per launch (8 bytes per event) over its average
    launch duration, measured in the same run with HIP start/stop events
    attached to its launch on the library's stream in every step of an eager
    K-step fit, against the 8 TB/s HBM peak; `traffic` is the HBM byte count
    per launch from the FETCH_SIZE and WRITE_SIZE summary under profiles/
    (scaled by the same counters on a calibration kernel of known traffic),
    reported only while the kernel sources still hash to what was profiled;
    `achievable_read` is the read rate of the library's streaming read probe
    (nll_read_probe) on a 4 GiB buffer in the same run;
  * fd_baseline  -- the same fit with forward-only FP64 NLLs and central
    finite-difference gradients (2P+1 batched NLL passes per step);
  * cpu_baseline -- the scalar FP64 oracle (test infrastructure) on the host
    cores: the same gradient-descent fits on a sample of the toys;
  * extra        -- the other workloads (each first autotuned unless
    --no-tune): the mixture with 1e7 events (fit steps, NLL+gradient hot and
    with the last-level cache flushed, its kernel's VALU/HBM roofline), the
    1-D Gaussian at 64 points, the precision study (1e8 events, FP64 and
    FP32-compensated), the 2-D Crystal Ball/ARGUS x Chebyshev model (5e7
    events), BHHH, extended, Johnson, chi-square, weighted, binned-template
    and expression-string densities; and `parity`: the worst NLL and gradient
    errors against the oracle per configuration.

    python bench.py [--steps K] [--warmup W] [--quick] [--no-cpu-baseline] [--no-tune]

Profiling helpers (used to write the summaries under profiles/):
    python bench.py --probe pmc          # calibration kernel + eager fit steps of both kernels
    python bench.py --summarize-trace DIR [--workload-name NAME]
    python bench.py --summarize-pmc FETCH_DIR WRITE_DIR --kernel {toys,mixture}
    python bench.py --summarize-valu DIR
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NLL+grad events/s per MI355X and % HBM roofline vs plain FP64 NLL+FD grad"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2003_12875_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
COPY_BYTES = 1 << 30  # calibration kernel: reads and writes 1 GiB
REPS = 5              # timed replays of the K-step headline fit (median reported)
# the fastest of the autotuner's candidates for the 4096-toy workload (a
# sweep of them on MI355X), fixed so that the profiled kernel is the timed one
TOYS_SCHEDULE = {"tile_events": 32768, "sets_blocks_per_cu": 4, "sets_unroll": 8}
KERNELS = {
    # name: (summary files, kernel-name test, algorithmic bytes per launch, workload)
    "toys": ("k_sets_gauss_4096toys", lambda k: "k_sets<" in k, None,
             "4096 Gaussian toy datasets, 4.13e8 FP64 events"),
    "mixture": ("k_single_fit_gauss_exp_1e7", lambda k: "k_single_fit<" in k, 8.0e7,
                "gauss+exp mixture, 1e7 FP64 events"),
}
VALU_COUNTERS = ["SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                 "SQ_INSTS_VALU_TRANS_F64", "SQ_WAVES"]
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: FP64 VALU lane-instructions/s
FP64_PEAK_FLOPS = 78.6e12


def csrc_hash():
    """sha256 over the device and host sources of the library (sorted)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if f.endswith((".h", ".hip", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _summary(path):
    """`- key: value` lines of a committed summary, or {} if absent or taken
    on different kernel sources."""
    kv = {}
    try:
        with open(path) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    kv[k.strip()] = v.strip().strip("`")
    except OSError:
        return {}
    return kv if kv.get("csrc_sha256") == csrc_hash() else {}


def profiled_traffic(which):
    kv = _summary(os.path.join(PROFILES, KERNELS[which][0] + "_traffic.txt"))
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def profiled_valu():
    """(VALU lane-instructions, FP64 FLOPs) per launch of the mixture's fit
    kernel from the committed counter summary, or None."""
    kv = _summary(os.path.join(PROFILES, KERNELS["mixture"][0] + "_valu.txt"))
    try:
        return float(kv["valu_lane_instructions_per_launch"]), float(kv["fp64_flops_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def median(v):
    v = sorted(v)
    n = len(v)
    return 0.5 * (v[(n - 1) // 2] + v[n // 2]) if n else float("nan")


def time_launches(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def time_flushed(torch, fn, reps, flush):
    """Median time (ms) of fn with the last-level cache flushed before each
    call (an in-place pass over a buffer four times its size); HIP events on
    the stream bracket fn alone."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        flush.add_(1.0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        ts.append(ev0.elapsed_time(ev1))
    return median(ts)


def read_probe(torch, nllmi, nbytes=4 << 30):
    """Achievable HBM read rate: the library's streaming read probe over a
    4 GiB buffer at several grid sizes, best median of 10 launches."""
    L = nllmi.lib()
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.empty(256 * 32, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    res = {}
    for bpc in (1, 2, 3, 4, 8):
        blocks = 256 * bpc

        def run():
            st = L.nll_read_probe(x.data_ptr(), n, out.data_ptr(), blocks, stream)
            if st != 0:
                raise RuntimeError(f"nll_read_probe: {st}")
        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(10):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            run()
            ev1.record()
            torch.cuda.synchronize()
            ts.append(ev0.elapsed_time(ev1))
        res[blocks] = nbytes / (median(ts) * 1e-3) / 1e9
    if abs(float(out[:blocks].sum().item()) - n) > 0.5:  # the last grid's block sums
        raise RuntimeError("read probe: wrong sum")
    best = max(res, key=res.get)
    del x, out
    torch.cuda.empty_cache()
    return {"GBs": res[best], "blocks": best, "bytes": nbytes, "GBs_by_blocks": res}


# ---------------------------------------------------------------------------
# headline: 4096 toys x K gradient-descent steps
# ---------------------------------------------------------------------------
def toys_setup(torch, nllmi, datagen):
    log("toys: generating 4096 datasets (4.13e8 events)")
    w = datagen.toys_workload()
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    m.set_schedule(**TOYS_SCHEDULE)
    offs = torch.from_numpy(w["offsets"]).cuda()
    start = torch.as_tensor(w["theta_start"], dtype=torch.float64, device="cuda").repeat(len(w["sizes"]), 1)
    return w, m, offs, start


def headline(torch, nllmi, datagen, args):
    w, m, offs, start = toys_setup(torch, nllmi, datagen)
    S = len(w["sizes"])
    n = int(w["offsets"][-1])
    P = m.n_param
    bufs = (start.clone(), torch.empty(S, dtype=torch.float64, device="cuda"),
            torch.empty(S, P, dtype=torch.float64, device="cuda"), torch.empty(S, dtype=torch.int32, device="cuda"))
    if args.warmup > 0:
        m.fit_batched(offs, start, args.warmup, 1.0)
    m.fit_batched(offs, start, args.steps, 1.0, out=bufs)  # records the K-step graph for these buffers
    torch.cuda.synchronize()
    log(f"toys: timing {REPS} replays of the {args.steps}-step fit")
    walls, gpus = [], []
    for _ in range(REPS):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        t0 = time.perf_counter()
        m.fit_batched(offs, start, args.steps, 1.0, out=bufs)
        ev1.record()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        gpus.append(ev0.elapsed_time(ev1))
    wall = median(walls)
    status_ok = bool((bufs[3] == 0).all().item())
    theta_fit = bufs[0].cpu().numpy()
    nll_fit = bufs[1].cpu().numpy()
    # the streaming kernel alone: HIP events attached to its launch in every
    # step of an eager fit of the same K steps; then whole steps likewise
    m.set_option("step_timing", "kernel")
    m.fit_batched(offs, start, args.steps, 1.0)
    kern = m.step_times()
    m.set_option("step_timing", True)
    m.fit_batched(offs, start, args.steps, 1.0)
    steps_eager = m.step_times()
    m.set_option("step_timing", False)
    kern_ms = sum(kern) / len(kern)
    bytes_per_launch = 8.0 * n
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9
    log("toys: read probe")
    probe = read_probe(torch, nllmi)
    # same-GPU baseline: forward-only batched NLL, 2P+1 passes per step
    th = start.clone()
    nll1 = torch.empty(S, dtype=torch.float64, device="cuda")
    stat = torch.empty(S, dtype=torch.int32, device="cuda")
    L = nllmi.lib()

    def fwd():
        L.nll_eval_batched(m._h, S, offs.data_ptr(), th.data_ptr(), nll1.data_ptr(), None, stat.data_ptr())

    def fwd_grad():
        L.nll_eval_batched(m._h, S, offs.data_ptr(), th.data_ptr(), nll1.data_ptr(), bufs[2].data_ptr(),
                           stat.data_ptr())
    m._bind_stream()
    t_fwd = time_launches(torch, fwd, 10)
    t_grad = time_launches(torch, fwd_grad, 10)
    fd_step_ms = (2 * P + 1) * t_fwd
    ms_per_step = 1e3 * wall / args.steps
    res = {
        "metric": METRIC, "value": n * args.steps / wall, "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4096 toy datasets of the 1-D Gaussian model on x in [-10,10] (sizes uniform in "
                               "[1000,200000], 413048672 FP64 events, truths +-10 %), each fitted by gradient "
                               "descent from (0.3, 1.5): per step NLL + adjoint gradient of both parameters of "
                               "every toy in one persistent launch, then the update (HIP-graph replay)",
                   "n_sets": S, "n_events": n, "n_params": P, "schedule": m.schedule,
                   "variant": m.info["variant"],
                   "timing": f"median of {REPS} replays of the {args.steps}-step graph; wall clock, "
                             "synchronised before and after each"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic("toys"),
                     "kernel": f"k_sets<gauss, grad, {m.schedule['sets_unroll']}>: the streaming launch of a "
                               "step (NLL and gradient of "
                               "every toy over (toy, tile) work items)",
                     "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": kern_ms,
                     "launches_timed": len(kern), "eager_step_ms": sum(steps_eager) / len(steps_eager),
                     "graph_step_ms": median(gpus) / args.steps,
                     "achievable_read": probe, "frac_of_achievable": achieved / probe["GBs"],
                     "csrc_sha256": csrc_hash()},
        "fd_baseline": {"forward_batched_ms": t_fwd, "passes_per_step": 2 * P + 1, "fd_step_ms": fd_step_ms,
                        "eval_grad_batched_ms": t_grad, "speedup_per_fit": fd_step_ms / ms_per_step},
        "fit": {"status_ok": status_ok, "replay_wall_ms": [1e3 * t for t in walls],
                "replay_gpu_ms": gpus},
    }
    return res, (w, theta_fit, nll_fit)


def toys_checks(datagen, w, theta_fit, nll_fit, steps, threads):
    """Fitted toys against the oracle's own gradient-descent fits (same
    start, same steps) on 8 toys, and every toy's fitted point against its
    closed-form maximum-likelihood estimate (mean and standard deviation;
    the truncation of the range moves it by ~1e-9)."""
    import numpy as np
    import oracle
    off = w["offsets"]
    x = w["cols"][0]
    picks = np.linspace(0, len(off) - 2, 8).astype(int)
    o = oracle.Oracle(w["spec"])
    sub_cols, sub_off = [], [0]
    for s in picks:
        sub_cols.append(x[off[s]:off[s + 1]])
        sub_off.append(sub_off[-1] + len(sub_cols[-1]))
    xs = np.concatenate(sub_cols)
    th0 = np.tile(w["theta_start"], (len(picks), 1))
    t0 = time.perf_counter()
    st, th_o, nll_o, g_o, stat_o = o.gd_fit_batched([xs], np.array(sub_off), th0, steps, 1.0, threads=threads)
    t_orc = time.perf_counter() - t0
    sizes = np.diff(off)
    mean = np.add.reduceat(x, off[:-1]) / sizes
    var = np.add.reduceat(x * x, off[:-1]) / sizes - mean ** 2
    mle = np.stack([mean, np.sqrt(var)], axis=1)
    return {"oracle_toys": [int(s) for s in picks],
            "max_nll_rel_err_vs_oracle_fit": float(np.max(np.abs(nll_fit[picks] / nll_o - 1.0))),
            "max_theta_abs_err_vs_oracle_fit": float(np.max(np.abs(theta_fit[picks] - th_o))),
            "max_theta_abs_err_vs_closed_form_mle": float(np.max(np.abs(theta_fit - mle))),
            "oracle_fit_s": t_orc}


def cpu_baseline(datagen, w, steps, budget_s=12.0):
    """The oracle's gradient-descent fits of a sample of the toys (every
    32nd; the same sizes, starts and step count) on all host cores, and of
    every 1024th toy on one core."""
    import numpy as np
    import oracle
    o = oracle.Oracle(w["spec"])
    off = w["offsets"]
    x = w["cols"][0]
    T = cores()

    def sample(every):
        picks = np.arange(0, len(off) - 1, every)
        cols = [x[off[s]:off[s + 1]] for s in picks]
        so = np.zeros(len(picks) + 1, dtype=np.int64)
        so[1:] = np.cumsum([len(c) for c in cols])
        return np.concatenate(cols), so, picks

    xs, so, picks = sample(32)
    th0 = np.tile(w["theta_start"], (len(picks), 1))
    t0 = time.perf_counter()
    o.gd_fit_batched([xs], so, th0, steps, 1.0, threads=T)
    dt = time.perf_counter() - t0
    x1, so1, p1 = sample(1024)
    t0 = time.perf_counter()
    o.gd_fit_batched([x1], so1, np.tile(w["theta_start"], (len(p1), 1)), steps, 1.0, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": int(so[-1]) * steps / dt, "unit": "events/s", "cores": T, "kind": "oracle",
            "sample": f"{len(picks)} of the 4096 toys (every 32nd, {int(so[-1])} events), {steps} gradient-descent "
                      f"steps each (NLL + analytic gradient + update), scalar FP64 C++ oracle, {T} threads over "
                      f"toys: {dt:.1f} s",
            "single_thread_value": int(so1[-1]) * steps / dt1,
            "single_thread_sample": f"{len(p1)} toys (every 1024th, {int(so1[-1])} events), {steps} steps, "
                                    f"one thread: {dt1:.1f} s"}


# ---------------------------------------------------------------------------
# the other workloads
# ---------------------------------------------------------------------------
def timed_fit(torch, model, theta0, steps, warmup, step_timing=False):
    """Warm up, record the K-step graph, then time one replay (or, with
    step_timing, one eager run with an event after every step)."""
    dev = model.device
    P = model.n_param
    bufs = (torch.empty(P, dtype=torch.float64, device=dev), torch.empty(1, dtype=torch.float64, device=dev),
            torch.empty(P, dtype=torch.float64, device=dev), torch.empty(1, dtype=torch.int32, device=dev))
    th0 = torch.as_tensor(theta0, dtype=torch.float64, device=dev)
    model.set_option("step_timing", step_timing)
    if step_timing:
        model.set_option("graph", False)
    if warmup > 0:
        model.fit(th0, warmup)
    model.fit(th0, steps, out=bufs)  # records the graph for these buffers
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    model.fit(th0, steps, out=bufs)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    step_ms = model.step_times() if step_timing else [gpu_ms / steps]
    st = int(bufs[3].item())
    model.set_option("step_timing", False)
    model.set_option("graph", True)
    return {"wall_s": wall, "gpu_ms": gpu_ms, "step_ms": step_ms, "status": st,
            "theta": bufs[0].cpu().numpy(), "nll": float(bufs[1].item())}


def tune(torch, model, theta, args, offsets=None):
    """The library's autotuner on this workload (unless --no-tune): every
    candidate schedule is checked against the default's NLL, the fastest
    kept.  No cache file: it tunes afresh."""
    if args.no_tune:
        return
    os.environ.pop("NLLMI_TUNE_CACHE", None)
    th = torch.as_tensor(theta, dtype=torch.float64, device="cuda")
    model.autotune(th, offsets=offsets)
    log(f"tuned schedule: {model.schedule}")


class Parity:
    """Worst NLL and gradient errors of the device against the oracle, per
    configuration (NLL relative; gradient max-norm over the oracle's)."""

    def __init__(self, threads):
        self.threads = threads
        self.out = {}
        self.orc_time = {}

    def check(self, name, spec, cols, points, gpu_vals, n_events):
        import numpy as np
        import oracle
        o = oracle.Oracle(spec)
        en, eg = 0.0, 0.0
        t0 = time.perf_counter()
        for th, (v, g) in zip(points, gpu_vals):
            st, ref, gref = o.nll(cols, np.asarray(th), threads=self.threads)
            if st != 0:
                raise RuntimeError(f"{name}: oracle status {st}")
            en = max(en, abs(v / ref - 1.0))
            eg = max(eg, float(np.max(np.abs(g - gref)) / np.max(np.abs(gref))))
        dt = time.perf_counter() - t0
        self.out[name] = {"points": len(points), "max_nll_rel_err": en, "max_grad_err_rel_max_norm": eg}
        self.orc_time[name] = {"events_per_s": n_events * len(points) / dt, "threads": self.threads,
                               "points": len(points), "n_events": n_events}


def mixture_1e7(torch, nllmi, datagen, args, parity):
    """The 1e7-event mixture: gradient-descent fit steps (one launch per
    step) with its kernel's roofline, NLL+gradient hot and with the
    last-level cache flushed, the finite-difference baseline."""
    log("mixture: 1e7 events")
    w = datagen.workload(2)
    spec, n = w["spec"], w["n"]
    cols = [torch.from_numpy(c).cuda() for c in w["cols"]]
    model = nllmi.Model.from_spec(spec)
    model.set_data(cols)
    theta0 = w["points"][0]
    r = timed_fit(torch, model, theta0, 200, 20)
    if r["status"] != 0:
        raise RuntimeError(f"fit status {r['status']}")
    kt = timed_fit(torch, model, theta0, 200, 0, step_timing="kernel")
    kern_ms = sum(kt["step_ms"]) / len(kt["step_ms"])
    valu = profiled_valu()
    th = torch.as_tensor(theta0, dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(model.n_param, dtype=torch.float64, device="cuda")
    t_fwd = time_launches(torch, lambda: model.eval(th, out=out), 50)
    t_grad = time_launches(torch, lambda: model.eval_grad(th, out=out, grad=grad), 50)
    flush = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB, 4x the last-level cache
    t_grad_flushed = time_flushed(torch, lambda: model.eval_grad(th, out=out, grad=grad), 20, flush)
    t_fwd_flushed = time_flushed(torch, lambda: model.eval(th, out=out), 20, flush)
    del flush
    fd_passes = 2 * model.n_param + 1
    step_ms = r["gpu_ms"] / 200
    vals = [(float(a.item()), b.cpu().numpy()) for a, b in (model.eval_grad(torch.from_numpy(p)) for p in w["points"])]
    parity.check("c2_mixture_1e7", spec, w["cols"], w["points"], vals, n)
    res = {"n_events": n, "fit_steps": 200, "fit_ms_per_step": 1e3 * r["wall_s"] / 200, "fit_gpu_step_ms": step_ms,
           "fit_events_per_s": n * 200 / r["wall_s"], "schedule": model.schedule,
           "kernel": {"name": "k_single_fit<gauss+exp, 4>: the previous step's update and this proposal's "
                              "constants in every block, then the NLL/gradient pass",
                      "avg_launch_ms": kern_ms,
                      "hbm": {"achieved_GBs": 8.0 * n / (kern_ms * 1e-3) / 1e9,
                              "frac": 8.0 * n / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "traffic": profiled_traffic("mixture")},
                      "valu": ({"lane_instructions_per_event": valu[0] / n,
                                "achieved_T_lane_ops": valu[0] / (kern_ms * 1e-3) / 1e12,
                                "peak_T_lane_ops": VALU_PEAK_LANE_OPS / 1e12,
                                "frac": valu[0] / (kern_ms * 1e-3) / VALU_PEAK_LANE_OPS,
                                "fp64_tflops": valu[1] / (kern_ms * 1e-3) / 1e12} if valu else None)},
           "eval_grad_ms": {"hot": t_grad, "cache_flushed": t_grad_flushed},
           "eval_ms": {"hot": t_fwd, "cache_flushed": t_fwd_flushed},
           "eval_grad_GBs": {"hot": 8.0 * n / (t_grad * 1e-3) / 1e9,
                             "cache_flushed": 8.0 * n / (t_grad_flushed * 1e-3) / 1e9},
           "fd_baseline": {"forward_ms": t_fwd, "passes_per_step": fd_passes, "fd_step_ms": fd_passes * t_fwd,
                           "speedup_per_fit": fd_passes * t_fwd / step_ms}}
    # the oracle on one core, for a per-core figure: 1e6 events, one point
    import numpy as np
    import oracle
    o = oracle.Oracle(spec)
    t0 = time.perf_counter()
    o.nll([w["cols"][0][:1_000_000]], np.asarray(theta0), threads=1)
    parity.orc_time["c2_mixture_1e7_single_thread"] = {"events_per_s": 1e6 / (time.perf_counter() - t0),
                                                       "threads": 1, "points": 1, "n_events": 1_000_000}
    del model, cols
    torch.cuda.empty_cache()
    return res


def extras(torch, nllmi, datagen, args, parity):
    import numpy as np
    ex = {}
    ex["mixture_1e7"] = mixture_1e7(torch, nllmi, datagen, args, parity)
    # 1-D Gaussian, 1e5 events: 64 parameter points, then fit steps (both
    # launch-latency bound at this size)
    w = datagen.workload(1)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    pts = torch.from_numpy(w["points"]).cuda()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.n_param, dtype=torch.float64, device="cuda")
    t64 = time_launches(torch, lambda: [m.eval(pts[i], out=out) for i in range(64)], 5)
    tpts = time_launches(torch, lambda: m.eval_points(pts, grad=False), 20)
    tptsg = time_launches(torch, lambda: m.eval_points(pts, grad=True), 20)
    r = timed_fit(torch, m, w["theta"], 50, 5)
    vals = [(float(a.item()), b.cpu().numpy()) for a, b in (m.eval_grad(pts[i]) for i in range(64))]
    parity.check("c1_gauss_1e5", w["spec"], w["cols"], w["points"], vals, w["n"])
    ex["gauss_1e5"] = {"eval_64_points_ms": t64, "eval_us": 1e3 * t64 / 64,
                       "eval_points_64_one_pass_ms": tpts, "eval_grad_points_64_one_pass_ms": tptsg,
                       "fit_steps": 50,
                       "fit_ms_per_step": 1e3 * r["wall_s"] / 50, "fit_avg_step_us": 1e3 * r["gpu_ms"] / 50,
                       "fit_events_per_s": w["n"] * 50 / r["wall_s"]}
    del m
    # precision study: 1e8 events of the mixture, FP64 and FP32-compensated
    # event passes; NLL+gradient timing and fp32c-vs-fp64 differences at the
    # 32 seeded points; both against the oracle at 4 of them
    log("c5: generating 1e8 events")
    w = datagen.workload(5)
    cols = [torch.from_numpy(c).cuda() for c in w["cols"]]
    pts = torch.from_numpy(w["points"]).cuda()
    res5 = {}
    vals = {}
    out5 = torch.empty(1, dtype=torch.float64, device="cuda")
    g5 = torch.empty(len(w["spec"]["params"]), dtype=torch.float64, device="cuda")
    for prec in ("fp64", "fp32c"):
        m = nllmi.Model.from_spec(w["spec"], precision=prec)
        m.set_data(cols)
        tune(torch, m, pts[0], args)
        tg = time_launches(torch, lambda: m.eval_grad(pts[0], out=out5, grad=g5), 10)
        vals[prec] = [(float(a.item()), b.cpu().numpy()) for a, b in (m.eval_grad(pts[i]) for i in range(32))]
        res5[prec] = {"eval_grad_ms": tg, "events_per_s": w["n"] / (tg * 1e-3),
                      "achieved_GBs": 8.0 * w["n"] / (tg * 1e-3) / 1e9,
                      "hbm_frac": 8.0 * w["n"] / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS, "variant": m.info["variant"],
                      "schedule": m.schedule}
        del m
    nerr = [abs(a[0] / b[0] - 1.0) for a, b in zip(vals["fp32c"], vals["fp64"])]
    gerr = [float(np.max(np.abs(a[1] - b[1])) / max(np.max(np.abs(b[1])), 1e-300))
            for a, b in zip(vals["fp32c"], vals["fp64"])]
    res5["fp32c_vs_fp64_gpu"] = {"points": 32, "max_nll_rel_err": max(nerr),
                                 "max_grad_err_rel_max_norm": max(gerr)}
    parity.check("c5_fp64_1e8", w["spec"], w["cols"], w["points"][:4], vals["fp64"][:4], w["n"])
    parity.check("c5_fp32c_1e8", w["spec"], w["cols"], w["points"][:4], vals["fp32c"][:4], w["n"])
    ex["precision_study_1e8"] = res5
    del cols, w
    torch.cuda.empty_cache()
    # 2-D CB/ARGUS x Chebyshev, 5e7 events, 9 free parameters
    log("c3: generating 5e7 events")
    w = datagen.workload(3)
    m = nllmi.Model.from_spec(w["spec"])
    cols = [torch.from_numpy(c).cuda() for c in w["cols"]]
    m.set_data(cols)
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.n_param, dtype=torch.float64, device="cuda")
    tune(torch, m, th, args)
    tg = time_launches(torch, lambda: m.eval_grad(th, out=out, grad=g), 10)
    tf = time_launches(torch, lambda: m.eval(th, out=out), 10)
    vals = [(float(a.item()), b.cpu().numpy()) for a, b in (m.eval_grad(torch.from_numpy(p)) for p in w["points"][:2])]
    parity.check("c3_cb_argus_cheb_5e7", w["spec"], w["cols"], w["points"][:2], vals, w["n"])
    n_free = int(sum(1 for p in w["spec"]["params"] if p.get("free", True)))
    ex["cb_argus_cheb_5e7"] = {"eval_grad_ms": tg, "eval_ms": tf, "events_per_s": w["n"] / (tg * 1e-3),
                               "achieved_GBs": 16.0 * w["n"] / (tg * 1e-3) / 1e9,
                               "hbm_frac": 16.0 * w["n"] / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "fd_step_ms": (2 * n_free + 1) * tf, "speedup_vs_fd": (2 * n_free + 1) * tf / tg,
                               "schedule": m.schedule}
    del m, cols, w
    torch.cuda.empty_cache()
    # second-order fit on the mixture: damped BHHH from the same start, steps
    # until the NLL is within 1e-9 (relative) of its final value, against
    # gradient descent's 200 steps
    w = datagen.workload(2)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    th0 = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    P = m.n_param
    bb = (torch.empty(P, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.float64, device="cuda"),
          torch.empty(P, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
    m.fit_bhhh(th0, 30, 1e-3, out=bb)
    torch.cuda.synchronize()
    t_bh = time_launches(torch, lambda: m.fit_bhhh(th0, 30, 1e-3, out=bb), 3)
    f_bh = float(bb[1].item())
    trace = []
    for k in (1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 20, 25, 30):
        trace.append((k, float(m.fit_bhhh(th0, k, 1e-3)[1].item())))
    steps_to = next((k for k, f in trace if abs(f - f_bh) <= 1e-9 * abs(f_bh)), None)
    gd = m.fit(th0, 200)
    ex["bhhh_c2_1e7"] = {"steps": 30, "ms_per_step": t_bh / 30, "nll": f_bh, "status": int(bb[3].item()),
                         "steps_to_1e-9": steps_to, "gd_200_steps_nll": float(gd[1].item()),
                         "nll_by_steps": trace}
    del m
    torch.cuda.empty_cache()
    # extended model (the mixture with a Poisson yield term nu - N ln nu,
    # 5 parameters) on the same events: NLL+gradient and a 200-step fit
    spec = dict(w["spec"])
    spec["params"] = list(spec["params"]) + [datagen.param("nu", 0.9 * w["n"], 1.0, 1e12)]
    spec["extended"] = True
    spec["yield_param"] = len(spec["params"]) - 1
    m = nllmi.Model.from_spec(spec)
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    thx = list(w["points"][0]) + [0.9 * w["n"]]
    th = torch.as_tensor(thx, dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.n_param, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: m.eval_grad(th, out=out, grad=g), 20)
    r = timed_fit(torch, m, thx, 200, 10)
    ex["extended_c2_1e7"] = {"eval_grad_ms": tg, "events_per_s": w["n"] / (tg * 1e-3),
                             "fit_ms_per_step": 1e3 * r["wall_s"] / 200, "fit_events_per_s": w["n"] * 200 / r["wall_s"],
                             "fit_status": r["status"], "n_events": w["n"]}
    del m
    torch.cuda.empty_cache()
    # weighted events on the mixture: the 1e7 events with weights in
    # [0.5, 1.5] (16 bytes per event, one logarithm more), and a binned fit
    # of the same events (1e4 bins of [0, 10], centres weighted by the counts)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    m.set_weights(torch.from_numpy(0.5 + datagen.uniforms(5, 12, w["n"])).cuda())
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.n_param, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: m.eval_grad(th, out=out, grad=g), 20)
    r = timed_fit(torch, m, w["points"][0], 50, 5)
    xc, cnt = datagen.binned(w["cols"][0], 0.0, 10.0, 10_000)
    mb = nllmi.Model.from_spec(w["spec"])
    mb.set_data([torch.from_numpy(xc).cuda()])
    mb.set_weights(torch.from_numpy(cnt).cuda())
    tb = time_launches(torch, lambda: mb.eval_grad(th, out=out, grad=g), 50)
    rb = timed_fit(torch, mb, w["points"][0], 200, 10)
    ex["weighted_c2_1e7"] = {"n_events": w["n"], "eval_grad_ms": tg, "events_per_s": w["n"] / (tg * 1e-3),
                             "achieved_GBs": 16.0 * w["n"] / (tg * 1e-3) / 1e9,
                             "fit_ms_per_step": 1e3 * r["wall_s"] / 50, "fit_status": r["status"],
                             "binned_10000_bins": {"eval_grad_us": 1e3 * tb,
                                                   "fit_us_per_step": 1e6 * rb["wall_s"] / 200,
                                                   "fit_status": rb["status"]}}
    del m, mb
    torch.cuda.empty_cache()
    # Johnson S_U peak over an exponential background (the Johnson density
    # of Sec. 3), 1e7 events: NLL+gradient and NLL alone; then the peak
    # alone (4 score features) fitted by damped BHHH from a seeded start
    w = datagen.johnson_workload()
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.n_param, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: m.eval_grad(th, out=out, grad=g), 20)
    tf = time_launches(torch, lambda: m.eval(th, out=out), 20)
    res_j = {"variant": m.info["variant"], "n_events": w["n"], "eval_grad_ms": tg, "eval_ms": tf,
             "events_per_s": w["n"] / (tg * 1e-3), "achieved_GBs": 8.0 * w["n"] / (tg * 1e-3) / 1e9,
             "schedule": m.schedule}
    del m
    w = datagen.johnson_workload(single=True)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    th0 = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    P = m.n_param
    bb = (torch.empty(P, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.float64, device="cuda"),
          torch.empty(P, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
    m.fit_bhhh(th0, 20, 1e-3, out=bb)
    torch.cuda.synchronize()
    t_bh = time_launches(torch, lambda: m.fit_bhhh(th0, 20, 1e-3, out=bb), 3)
    f_bh = float(bb[1].item())
    trace = [(k, float(m.fit_bhhh(th0, k, 1e-3)[1].item())) for k in (1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 20)]
    res_j["peak_alone_bhhh"] = {"variant": m.info["variant"], "steps": 20, "ms_per_step": t_bh / 20,
                                "nll": f_bh, "status": int(bb[3].item()),
                                "steps_to_1e-9": next((k for k, f in trace if abs(f - f_bh) <= 1e-9 * abs(f_bh)), None)}
    ex["johnson_exp_1e7"] = res_j
    del m
    torch.cuda.empty_cache()
    # chi-square (the ChiSquarePdf model of the paper's speed-up figure),
    # 1e7 events: NLL+gradient, NLL alone, and damped BHHH to convergence
    w = datagen.chi2_workload()
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(1, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: m.eval_grad(th, out=out, grad=g), 20)
    tf = time_launches(torch, lambda: m.eval(th, out=out), 20)
    bb = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.float64, device="cuda"),
          torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
    m.fit_bhhh(th, 10, 1e-3, out=bb)
    torch.cuda.synchronize()
    t_bh = time_launches(torch, lambda: m.fit_bhhh(th, 10, 1e-3, out=bb), 3)
    ex["chi2_1e7"] = {"variant": m.info["variant"], "n_events": w["n"], "eval_grad_ms": tg, "eval_ms": tf,
                      "events_per_s": w["n"] / (tg * 1e-3), "achieved_GBs": 8.0 * w["n"] / (tg * 1e-3) / 1e9,
                      "bhhh_10_steps_ms_per_step": t_bh / 10, "bhhh_status": int(bb[3].item()),
                      "schedule": m.schedule}
    del m
    torch.cuda.empty_cache()
    # Hypatia2 peak over an exponential background (the two-sided Hypatia
    # of Sec. 3), 1e7 events, all 11 parameters free: NLL+gradient and NLL
    # alone, the per-point table build included in every launch; parity
    # against the oracle on the first 2e5 events at two points
    w = datagen.hypatia_workload()
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.n_param, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: m.eval_grad(th, out=out, grad=g), 20)
    tf = time_launches(torch, lambda: m.eval(th, out=out), 20)
    ex["hypatia_exp_1e7"] = {"variant": m.info["variant"], "n_events": w["n"], "eval_grad_ms": tg, "eval_ms": tf,
                             "events_per_s": w["n"] / (tg * 1e-3),
                             "achieved_GBs": 8.0 * w["n"] / (tg * 1e-3) / 1e9,
                             "hbm_frac": 8.0 * w["n"] / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "schedule": m.schedule, "status": m.sync()}
    del m
    n_par = 200_000
    sub = [c[:n_par] for c in w["cols"]]
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in sub])
    vals = [(float(a.item()), b.cpu().numpy()) for a, b in (m.eval_grad(torch.from_numpy(p)) for p in w["points"][:2])]
    parity.check("hypatia_exp_2e5", w["spec"], sub, w["points"][:2], vals, n_par)
    del m
    torch.cuda.empty_cache()
    # binned template likelihood of HistFactory type: 2e6 bins, 4 samples,
    # 16 histosys, 4 normsys, 2 normfactors (22 parameters); HBM-bound,
    # 8 (1 + 4 + 16) bytes per bin
    w = datagen.hf_workload()
    mh = nllmi.HFModel(w["spec"])
    mh.set_data(w["counts"], w["nominal"], w["up"], w["down"])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(mh.n_param, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: mh.eval_grad(th, out=out, grad=g), 20)
    tf = time_launches(torch, lambda: mh.eval(th, out=out), 20)
    nbytes = 8.0 * (1 + mh.n_samples + mh.n_histosys) * mh.n_bins
    ex["histfactory_2e6_bins"] = {"n_bins": mh.n_bins, "samples": mh.n_samples, "histosys": mh.n_histosys,
                                  "params": mh.n_param, "eval_grad_ms": tg, "eval_ms": tf,
                                  "bytes_per_eval": nbytes, "achieved_GBs": nbytes / (tg * 1e-3) / 1e9,
                                  "hbm_frac": nbytes / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "status": mh.sync()}
    # the same model with per-bin statistical parameters on the first two
    # samples: gamma_b and 1/sigma_b^2 read, d NLL / d gamma_b written per bin
    rng = np.random.default_rng(2003012875 + 9000)
    sigma = torch.as_tensor(rng.uniform(0.01, 0.1, mh.n_bins), dtype=torch.float64, device="cuda")
    gam = torch.as_tensor(1.0 + rng.uniform(-0.05, 0.05, mh.n_bins), dtype=torch.float64, device="cuda")
    gg = torch.empty(mh.n_bins, dtype=torch.float64, device="cuda")
    mh.set_staterror([0, 1], sigma)
    L = nllmi.lib()
    ts = time_launches(torch, lambda: L.nll_hf_eval_stat(mh._h, th.data_ptr(), gam.data_ptr(), out.data_ptr(),
                                                         g.data_ptr(), gg.data_ptr()), 20)
    sbytes = nbytes + 24.0 * mh.n_bins
    ex["histfactory_2e6_bins"]["staterror"] = {"eval_grad_ms": ts, "bytes_per_eval": sbytes,
                                               "achieved_GBs": sbytes / (ts * 1e-3) / 1e9,
                                               "hbm_frac": sbytes / (ts * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                               "status": mh.sync()}
    del mh
    torch.cuda.empty_cache()
    # the smooth interpolation codes (every normsys and histosys), 12
    # histosys at 2e6 bins: both delta templates of every histosys are read,
    # 8 (1 + 4 + 2 x 12) bytes per bin
    w = datagen.hf_workload(n_histosys=12, n_points=1)
    spec = w["spec"]
    for md in spec["modifiers"]:
        if md["type"] in ("normsys", "histosys"):
            md["interp"] = "poly6"
    mh = nllmi.HFModel(spec)
    mh.set_data(w["counts"], w["nominal"], w["up"], w["down"])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    g = torch.empty(mh.n_param, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: mh.eval_grad(th, out=out, grad=g), 20)
    nbytes = 8.0 * (1 + mh.n_samples + 2 * mh.n_histosys) * mh.n_bins
    ex["histfactory_smooth_2e6_bins"] = {"n_bins": mh.n_bins, "samples": mh.n_samples, "histosys": mh.n_histosys,
                                         "params": mh.n_param, "eval_grad_ms": tg, "bytes_per_eval": nbytes,
                                         "achieved_GBs": nbytes / (tg * 1e-3) / 1e9,
                                         "hbm_frac": nbytes / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                         "status": mh.sync()}
    del mh
    torch.cuda.empty_cache()
    # just-in-time density: a Gaussian written as an expression string on the
    # 1-D Gaussian's range with 1e7 events, against the built-in Gaussian leaf
    # on the same events (compile time included once)
    w = datagen.workload(1, n=10_000_000)
    x = torch.from_numpy(w["cols"][0]).cuda()
    t0 = time.perf_counter()
    mj = nllmi.JITModel("exp(-0.5*((x-p[0])/p[1])*((x-p[0])/p[1]))", -10.0, 10.0, w["spec"]["params"])
    t_compile = time.perf_counter() - t0
    mj.set_data(x)
    mb = nllmi.Model.from_spec(w["spec"])
    mb.set_data([x])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(2, dtype=torch.float64, device="cuda")
    tj = time_launches(torch, lambda: mj.eval_grad(th, out=out, grad=g), 20)
    tb = time_launches(torch, lambda: mb.eval_grad(th, out=out, grad=g), 20)
    ex["jit_gauss_1e7"] = {"compile_s": t_compile, "eval_grad_ms": tj, "events_per_s": 1e7 / (tj * 1e-3),
                           "builtin_gauss_eval_grad_ms": tb, "status": mj.sync()}
    del mj, mb, x
    torch.cuda.empty_cache()
    # a formula leaf inside a composite model: f Breit-Wigner(x) formula +
    # (1 - f) built-in Exp(x) with 1e7 events, compiled at model creation
    # (the code-object cache may hold it from an earlier run)
    w = datagen.jit_composite_workload("bw_exp", n=10_000_000, n_points=1)
    t0 = time.perf_counter()
    mc = nllmi.Model.from_spec(w["spec"])
    t_compile = time.perf_counter() - t0
    mc.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    g = torch.empty(mc.n_param, dtype=torch.float64, device="cuda")
    tg = time_launches(torch, lambda: mc.eval_grad(th, out=out, grad=g), 20)
    tf = time_launches(torch, lambda: mc.eval(th, out=out), 20)
    ex["jit_composite_bw_exp_1e7"] = {"create_s": t_compile, "eval_grad_ms": tg, "eval_ms": tf,
                                      "events_per_s": 1e7 / (tg * 1e-3), "variant": mc.info["variant"],
                                      "status": mc.sync()}
    del mc
    torch.cuda.empty_cache()
    return ex


# ---------------------------------------------------------------------------
# profiling helpers
# ---------------------------------------------------------------------------
def probe_pmc(torch, nllmi, datagen, steps):
    """Workload for counter runs: one calibration kernel of known traffic
    (elementwise negation of 1 GiB: reads and writes COPY_BYTES), then eager
    fit steps of the toys and of the 1e7-event mixture."""
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    w, m, offs, start = toys_setup(torch, nllmi, datagen)
    m.set_option("graph", False)
    m.fit_batched(offs, start, 3, 1.0)
    torch.cuda.synchronize()
    del m
    torch.cuda.empty_cache()
    log("probe: 3 eager toy-fit steps done")
    w = datagen.workload(2)
    model = nllmi.Model.from_spec(w["spec"])
    model.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    model.set_option("graph", False)
    th0 = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    model.fit(th0, steps)
    torch.cuda.synchronize()
    log(f"probe: {steps} eager mixture fit steps done")


def probe_pmc_2d(torch, nllmi, datagen, reps):
    """Workload for counter runs on the 2-D model: NLL+gradient of the
    5e7-event Crystal Ball/ARGUS x Chebyshev model at its default schedule,
    `reps` times."""
    w = datagen.workload(3)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    th = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.n_param, dtype=torch.float64, device="cuda")
    for _ in range(reps):
        m.eval_grad(th, out=out, grad=g)
    torch.cuda.synchronize()
    log(f"probe: {reps} NLL+gradient evaluations of the 2-D model done ({m.schedule})")


# How each committed summary is made (from the repository root; the
# profiler runs from /tmp with TMPDIR=/tmp, paths below relative to the root)
PROFILE_COMMANDS = {
    "trace": ["rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/trace_toys -o toys -- "
              "python3 bench.py --quick --no-cpu-baseline --steps 50 --warmup 5",
              "python3 bench.py --summarize-trace gpurun_out/trace_toys --workload-name '<workload>'"],
    "pmc": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o f -- python3 bench.py --probe pmc",
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o w -- python3 bench.py --probe pmc",
            "python3 bench.py --summarize-pmc gpurun_out/pmc_fetch gpurun_out/pmc_write --kernel <toys|mixture>"],
    "valu": ["rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 "
             "SQ_INSTS_VALU_TRANS_F64 SQ_WAVES --output-format csv -d gpurun_out/pmc_valu -o v -- "
             "python3 bench.py --probe pmc",
             "python3 bench.py --summarize-valu gpurun_out/pmc_valu"],
    "counters": ["rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES "
                 "SQ_WAVE_CYCLES GRBM_GUI_ACTIVE --output-format csv -d gpurun_out/pmc_2d -o c -- "
                 "python3 bench.py --probe pmc-2d",
                 "python3 bench.py --summarize-counters gpurun_out/pmc_2d 'k_single<'"],
}


def print_commands(kind):
    print("Made by (repository root; the profiler itself run from /tmp with TMPDIR=/tmp):\n")
    for c in PROFILE_COMMANDS[kind]:
        print(f"    {c}")
    print()


N_SIMD, N_XCD, N_EVENTS_2D = 256 * 4, 8, 50_000_000


def summarize_counters(d, pattern):
    """Average of every counter per dispatch of the kernels whose name
    contains `pattern` (one line per kernel and counter), and the derived
    issue figures of the 2-D model's NLL+gradient kernel."""
    rows = [r for r in _csv_rows(d, "_counter_collection.csv") if pattern in r["Kernel_Name"]]
    agg = {}
    for r in rows:
        agg.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    print("# SQ counters of the 2-D model's NLL+gradient kernel: (0.1 CB + 0.9 ARGUS)(m) x Cheb4(y), "
          "5e7 FP64 events x 2 observables\n")
    print_commands("counters")
    print(f"- csrc_sha256: `{csrc_hash()}`")
    for (k, c), v in sorted(agg.items()):
        print(f"- `{_short(k)}` {c}: {sum(v) / len(v):.6e} (dispatches {len(v)})")
    kernels = sorted({k for k, _ in agg})
    for k in kernels:
        a = {c: sum(v) / len(v) for (kk, c), v in agg.items() if kk == k}
        if not all(c in a for c in ("SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU")):
            continue
        # GRBM_GUI_ACTIVE reads the sum over the XCDs (8 x the kernel's cycles)
        cyc = a["GRBM_GUI_ACTIVE"] / N_XCD
        print(f"\nDerived, `{_short(k)}`:\n")
        print(f"- gpu_cycles_per_xcd: {cyc:.4e} ({cyc / 2.4e3:.1f} us at 2.4 GHz)")
        print(f"- valu_busy: {a['SQ_ACTIVE_INST_VALU'] * 4 / N_SIMD / cyc:.3f}"
              "  (SQ_ACTIVE_INST_VALU x 4 / 1024 SIMDs / cycles)")
        print(f"- valu_issue_4cyc: {a['SQ_INSTS_VALU'] * 4 / N_SIMD / cyc:.3f}"
              "  (SQ_INSTS_VALU x 4 cycles per wave64 instruction / 1024 SIMDs / cycles)")
        print(f"- valu_lane_instructions_per_event: {64.0 * a['SQ_INSTS_VALU'] / N_EVENTS_2D:.1f}")
        if "SQ_INSTS_SALU" in a:
            print(f"- salu_instructions_per_wave_instruction_valu: {a['SQ_INSTS_SALU'] / a['SQ_INSTS_VALU']:.3f}")


def _csv_rows(d, suffix):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {d}")
    return rows


def _short(name):
    name = name.replace("nllmi::", "")
    return name if len(name) < 160 else name[:157] + "..."


def summarize_trace(d, workload):
    """Per-kernel duration summary from a --kernel-trace CSV output folder."""
    rows = _csv_rows(d, "_kernel_trace.csv")
    agg = {}
    for r in rows:
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3  # ns -> us
        agg.setdefault(r["Kernel_Name"], []).append(dt)
    tot = sum(sum(v) for v in agg.values())
    print(f"# Kernel durations: {workload}\n")
    print_commands("trace")
    print(f"- csrc_sha256: `{csrc_hash()}`\n")
    print("| kernel | calls | total us | avg us | median us | min us | max us | % |")
    print("|---|---|---|---|---|---|---|---|")
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{_short(k)}` | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.2f} | {median(v):.2f} | "
              f"{min(v):.2f} | {max(v):.2f} | {100 * sum(v) / tot:.1f} |")


def _per_kernel(d, counter, scale=1.0):
    """{kernel name: [value per dispatch, in dispatch order]} of one counter."""
    out = {}
    rows = [r for r in _csv_rows(d, "_counter_collection.csv") if r["Counter_Name"] == counter]
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * scale)
    return out


def _pick(tab, pred):
    ks = [k for k in tab if pred(k)]
    if len(ks) != 1:
        raise SystemExit(f"expected one kernel, found {ks}")
    return ks[0], tab[ks[0]]


def _streaming(values):
    """Indices of the launches that streamed the events: a proposal outside
    the parameter ranges is rejected before the stream (the step size
    halved), and its launch reads only the first preloaded tiles."""
    top = max(values)
    return [i for i, v in enumerate(values) if v >= 0.5 * top]


def summarize_pmc(fetch_dir, write_dir, which):
    """HBM traffic per launch of one streaming kernel from two counter runs
    (FETCH_SIZE, WRITE_SIZE: KiB per dispatch), scaled by what the same
    counters read for the calibration kernel; averaged over the launches
    that streamed."""
    stem, pred, alg, workload = KERNELS[which]
    if alg is None:  # the toys: 8 bytes per event of the 4096 datasets
        import datagen
        alg = 8.0 * float(datagen.toys_workload()["offsets"][-1])
    fetch, write = _per_kernel(fetch_dir, "FETCH_SIZE", 1024.0), _per_kernel(write_dir, "WRITE_SIZE", 1024.0)
    _, cf = _pick(fetch, lambda k: "neg" in k)
    _, cw = _pick(write, lambda k: "neg" in k)
    kk, kf_all = _pick(fetch, pred)
    _, kw_all = _pick(write, lambda k: k == kk)
    idx = _streaming(kf_all)
    kf = [kf_all[i] for i in idx]
    kw = [kw_all[i] for i in idx if i < len(kw_all)]
    f_fac = COPY_BYTES / (sum(cf) / len(cf))
    w_fac = COPY_BYTES / (sum(cw) / len(cw))
    fb = f_fac * sum(kf) / len(kf)
    wb = w_fac * sum(kw) / len(kw)
    print(f"# HBM traffic of the streaming kernel: {workload}\n")
    print("Counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own run, scaled by")
    print(f"the same counter on the calibration kernel (elementwise negation, {COPY_BYTES} bytes read and written).")
    print("Averaged over the launches that streamed the events.\n")
    print_commands("pmc")
    print(f"- kernel: `{_short(kk)}`")
    print(f"- csrc_sha256: `{csrc_hash()}`")
    print(f"- dispatches: {len(kf_all)} ({len(kf)} streamed)")
    print("- fetch_bytes_per_dispatch: " + ", ".join(f"{f_fac * v:.4e}" for v in kf_all))
    print(f"- calibration_fetch_factor: {f_fac:.4f}")
    print(f"- calibration_write_factor: {w_fac:.4f}")
    print(f"- fetch_bytes_per_launch: {fb:.4e}")
    print(f"- write_bytes_per_launch: {wb:.4e}")
    print(f"- traffic_bytes_per_launch: {fb + wb:.4e}")
    print(f"- algorithmic_bytes_per_launch: {alg:.4e}")
    print(f"- traffic_over_algorithmic: {(fb + wb) / alg:.4f}")


def summarize_valu(d):
    """VALU instructions per launch of the mixture's fit kernel from one
    counter run (wave-level instruction counts, summed over the chip),
    averaged over the launches that streamed."""
    tabs = {c: _per_kernel(d, c) for c in VALU_COUNTERS}
    kk, valu_all = _pick(tabs["SQ_INSTS_VALU"], KERNELS["mixture"][1])
    idx = _streaming(valu_all)
    avg = {c: sum(tabs[c][kk][i] for i in idx) / len(idx) for c in VALU_COUNTERS}
    lane_ops = 64.0 * avg["SQ_INSTS_VALU"]
    flops = 64.0 * (2.0 * avg["SQ_INSTS_VALU_FMA_F64"] + avg["SQ_INSTS_VALU_ADD_F64"] +
                    avg["SQ_INSTS_VALU_MUL_F64"] + avg["SQ_INSTS_VALU_TRANS_F64"])
    print("# VALU work of the streaming fit kernel: gauss+exp mixture, 1e7 FP64 events\n")
    print("SQ instruction counters (wave instructions per dispatch, all CUs), one run, averaged over the")
    print("launches that streamed the events. Lane-instructions = 64 x wave instructions (wave64);")
    print("FP64 FLOPs = 64 x (2 FMA + ADD + MUL + TRANS).\n")
    print_commands("valu")
    print(f"- kernel: `{_short(kk)}`")
    print(f"- csrc_sha256: `{csrc_hash()}`")
    print(f"- dispatches: {len(valu_all)} ({len(idx)} streamed)")
    for c in VALU_COUNTERS:
        print(f"- {c}: {avg[c]:.4e}")
    print(f"- valu_lane_instructions_per_launch: {lane_ops:.4e}")
    print(f"- valu_lane_instructions_per_event: {lane_ops / 1e7:.2f}")
    print(f"- fp64_flops_per_launch: {flops:.4e}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch schedules")
    ap.add_argument("--probe", choices=["pmc", "pmc-2d"], help="run a counter-collection workload only")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("DIR", "KERNEL_SUBSTRING"))
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--workload-name", default="")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--kernel", choices=sorted(KERNELS), default="toys")
    ap.add_argument("--summarize-valu", metavar="DIR")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload_name)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.kernel)
        return
    if args.summarize_valu:
        summarize_valu(args.summarize_valu)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for {max(args.gpus, world)}); "
              "multi-GPU sharding is a design note only", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    import torch
    import datagen
    import paper_2003_12875_amd as nllmi
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    nllmi.lib()
    if args.probe == "pmc":
        probe_pmc(torch, nllmi, datagen, 10)
        return
    if args.probe == "pmc-2d":
        probe_pmc_2d(torch, nllmi, datagen, 5)
        return
    res, (w, theta_fit, nll_fit) = headline(torch, nllmi, datagen, args)
    torch.cuda.empty_cache()
    T = cores()
    if not args.quick:
        parity = Parity(min(T, 16))
        try:
            res["extra"] = extras(torch, nllmi, datagen, args, parity)
        except Exception as e:  # extras never hide the headline
            res["extra"] = {"error": repr(e)}
        log("toys: checks against the oracle")
        parity.out["c4_toys_fit"] = toys_checks(datagen, w, theta_fit, nll_fit, args.steps, min(T, 16))
        res["extra"]["parity"] = parity.out
        res["extra"]["oracle_timing"] = parity.orc_time
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle")
        res["cpu_baseline"] = cpu_baseline(datagen, w, args.steps)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

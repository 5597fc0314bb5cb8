#!/usr/bin/env python3
"""Benchmark of the batched unbinned NLL on one MI355X.

Headline workload (one JSON line on stdout): the extended
signal+background model f*Gauss(mu, sigma) + (1-f)*Exp(c) on x in [0, 10]
with 1e7 synthetic FP64 events.  One step = one gradient-descent iteration
on the device: per-point constants (normalisation and its derivatives),
one fused pass over the events computing NLL and the adjoint gradient of
all 4 parameters, the compensated reduction, and the parameter update --
all in the library's HIP kernels (one launch per step), recorded once into
a HIP graph.

Also reported, on the same GPU:
  * fd_baseline -- forward-only FP64 NLL plus a central finite-difference
    gradient (2P+1 passes per step), the per-fit speed-up of the adjoint;
  * roofline    -- the dominant kernel (k_single_fit, one launch per step:
    the previous step's update and this proposal's constants in every
    block, then the fused streaming pass), whose average duration is measured in the same run with HIP start/stop events
    attached to its launch on the library's stream (hipExtLaunchKernel) in
    every step of an eager K-step fit.  It is bound by FP64 VALU issue
    ("alu"): its VALU lane-instructions per launch (SQ_INSTS_VALU summary
    under profiles/) over that duration, against 256 CUs x 4 SIMDs x 16
    lanes x 2.4 GHz; `hbm` holds the metric's HBM figure (algorithmic bytes
    per launch over the same duration, against 8 TB/s); `traffic` is the HBM
    byte count per launch from the FETCH_SIZE and WRITE_SIZE summary under
    profiles/ (scaled by the same counters on a plain streaming kernel of
    known size).  Counter figures are reported only while the kernel
    sources still hash to what was profiled;
  * cpu_baseline -- the scalar FP64 oracle (test infrastructure) on the
    host cores, same events, same minimiser;
  * extra       -- the other workloads: 1-D Gaussian (1e5 events) at 64
    parameter points (64 launches, and all 64 in one nll_eval_points pass)
    and fit steps, the damped BHHH fit and the extended (Poisson yield)
    mixture on the 1e7 events,
    the precision study (1e8 events, FP64
    and FP32-compensated passes), the 2-D Crystal Ball/ARGUS x Chebyshev
    model (5e7 events), and 4096 batched toy fits (4.1e8 events per step).

    python bench.py [--steps K] [--warmup W] [--quick] [--no-cpu-baseline] [--no-tune]

Each extra workload first runs the library's autotuner (nll_autotune:
every candidate launch schedule checked against the current one's NLL, the
fastest kept); --no-tune keeps the default schedules.  The headline keeps
the default schedule, which is the one profiled under profiles/.

Profiling helpers (used to write the summaries under profiles/):
    python bench.py --probe pmc          # calibration copy + a few eager fit steps
    python bench.py --summarize-trace DIR [--workload-name NAME]
    python bench.py --summarize-pmc FETCH_DIR WRITE_DIR
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_single_fit_gauss_exp_1e7_traffic.txt")
COPY_BYTES = 1 << 30  # calibration kernel: reads and writes 1 GiB


def csrc_hash():
    """sha256 over the device and host sources of the library (sorted)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if f.endswith((".h", ".hip", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per launch from the committed counter summary, or None if
    absent or taken on different kernel sources."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    kv[k.strip()] = v.strip().strip("`")
        if kv.get("csrc_sha256") != csrc_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


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


def median(v):
    v = sorted(v)
    n = len(v)
    return 0.5 * (v[(n - 1) // 2] + v[n // 2]) if n else float("nan")


def headline(torch, nllmi, datagen, args):
    log("c2: generating 1e7 events")
    w = datagen.workload(2)
    spec, n = w["spec"], w["n"]
    cols = [torch.from_numpy(c).cuda() for c in w["cols"]]
    model = nllmi.Model.from_spec(spec)
    model.set_data(cols)
    theta0 = w["points"][0]
    # the default schedule, not the tuner's pick: for this workload the
    # candidates are within a few per cent of each other (run-to-run noise
    # decides), and the profiled kernel (counters, trace) must be the timed one
    log(f"c2: timing {args.steps} gradient-descent steps")
    r = timed_fit(torch, model, theta0, args.steps, args.warmup)
    if r["status"] != 0:
        raise RuntimeError(f"fit status {r['status']}")
    ms_per_step = 1e3 * r["wall_s"] / args.steps
    value = n * args.steps / r["wall_s"]
    graph_step_ms = r["gpu_ms"] / args.steps  # HIP events around the replay, per step
    # the dominant kernel alone: start/stop events attached to the streaming
    # kernel's launch in every step of an eager fit of the same K steps
    kt = timed_fit(torch, model, theta0, args.steps, 0, step_timing="kernel")
    kern_ms = sum(kt["step_ms"]) / len(kt["step_ms"])
    bytes_per_launch = 8.0 * n * len(spec["obs"])
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9
    traffic = profiled_traffic()
    # the kernel is bound by FP64 VALU issue: its measured VALU work per
    # launch (committed counter summary) over the same launch time
    valu = profiled_valu()
    alu_achieved = valu[0] / (kern_ms * 1e-3) / 1e12 if valu else None

    # same-GPU baseline: forward-only FP64 NLL + central finite differences
    th = torch.as_tensor(theta0, dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(model.n_param, dtype=torch.float64, device="cuda")
    t_fwd = time_launches(torch, lambda: model.eval(th, out=out), 50)
    t_grad = time_launches(torch, lambda: model.eval_grad(th, out=out, grad=grad), 50)
    n_free = int(sum(1 for p in spec["params"] if p.get("free", True)))
    fd_passes = 2 * n_free + 1
    fd_step_ms = fd_passes * t_fwd
    res = {
        "metric": METRIC, "value": value, "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "f*Gauss(mu,sigma)+(1-f)*Exp(c) on x in [0,10], f=0.2, 1e7 FP64 events; "
                               "NLL + adjoint gradient of 4 parameters and one on-device gradient-descent "
                               "update per step (HIP-graph replay)",
                   "n_events": n, "n_params": model.n_param, "schedule": model.schedule,
                   "variant": model.info["variant"]},
        "roofline": {"bound": "alu", "achieved": alu_achieved, "peak": VALU_PEAK_LANE_OPS / 1e12,
                     "unit": "T FP64-VALU lane-instructions/s",
                     "frac": alu_achieved / (VALU_PEAK_LANE_OPS / 1e12) if valu else None,
                     "traffic": traffic,
                     "kernel": "k_single_fit<gauss+exp>: the previous step's update and this proposal's "
                               "constants, then the NLL/gradient pass",
                     "valu_lane_instructions_per_event": valu[0] / n if valu else None,
                     "fp64_tflops": valu[1] / (kern_ms * 1e-3) / 1e12 if valu else None,
                     "fp64_tflops_peak": FP64_PEAK_FLOPS / 1e12,
                     "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bytes_per_launch},
                     "avg_launch_ms": kern_ms, "graph_step_ms": graph_step_ms, "csrc_sha256": csrc_hash(),
                     "note": "VALU peak = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz; the instruction count is "
                             "measured (SQ_INSTS_VALU, profiles/); 80 MB of events also fit in the 256 MB "
                             "last-level cache"},
        "fd_baseline": {"forward_ms": t_fwd, "passes_per_step": fd_passes, "fd_step_ms": fd_step_ms,
                        "eval_grad_ms": t_grad, "speedup_per_fit": fd_step_ms / ms_per_step,
                        "speedup_vs_eval_grad": fd_step_ms / t_grad},
    }
    return res, w, model


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


def cpu_baseline(datagen, w, budget_s=12.0):
    import oracle
    o = oracle.Oracle(w["spec"])
    T = cores()
    t0 = time.perf_counter()
    st, *_ = o.gd_fit(w["cols"], w["points"][0], 1, 1.0, threads=T)
    one = time.perf_counter() - t0
    steps = int(max(2, min(50, budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    st, *_ = o.gd_fit(w["cols"], w["points"][0], steps, 1.0, threads=T)
    dt = time.perf_counter() - t0
    return {"value": w["n"] * steps / dt, "unit": "events/s", "cores": T, "kind": "oracle",
            "sample": f"{steps} gradient-descent steps (NLL+analytic gradient+update) on all {w['n']} events "
                      f"of the same workload, scalar FP64 C++ oracle, {T} threads over contiguous chunks"}


def extras(torch, nllmi, datagen, args):
    ex = {}
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
    ex["gauss_1e5"] = {"eval_64_points_ms": t64, "eval_us": 1e3 * t64 / 64,
                       "eval_points_64_one_pass_ms": tpts, "eval_grad_points_64_one_pass_ms": tptsg,
                       "fit_steps": 50,
                       "fit_ms_per_step": 1e3 * r["wall_s"] / 50, "fit_avg_step_us": 1e3 * r["gpu_ms"] / 50,
                       "fit_events_per_s": w["n"] * 50 / r["wall_s"]}
    del m
    # precision study: 1e8 events of the mixture, FP64 and FP32-compensated
    # event passes; NLL+gradient timing and fp32c-vs-fp64 differences at the
    # 32 seeded points (the comparison with the FP64 oracle is a GPU test)
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
    import numpy as np
    nerr = [abs(a[0] / b[0] - 1.0) for a, b in zip(vals["fp32c"], vals["fp64"])]
    gerr = [float(np.max(np.abs(a[1] - b[1])) / max(np.max(np.abs(b[1])), 1e-300))
            for a, b in zip(vals["fp32c"], vals["fp64"])]
    res5["fp32c_vs_fp64_gpu"] = {"points": 32, "max_nll_rel_err": max(nerr), "max_grad_rel_err_vs_max_abs": max(gerr)}
    ex["precision_study_1e8"] = res5
    del cols
    torch.cuda.empty_cache()
    # second-order fit on the headline workload: damped BHHH from the same
    # start, steps until the NLL is within 1e-9 (relative) of its final value,
    # against gradient descent's 200 steps
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
    # extended model (the c2 mixture with a Poisson yield term nu - N ln nu,
    # 5 parameters) on the c2 events: NLL+gradient and a 200-step fit
    w = datagen.workload(2)
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
    # weighted events on the headline mixture: the 1e7 events with weights
    # in [0.5, 1.5] (16 bytes per event, one logarithm more), and a binned
    # fit of the same events (1e4 bins of [0, 10], centres weighted by the
    # counts)
    w = datagen.workload(2)
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
    import numpy as np
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
    # just-in-time density: a Gaussian written as an expression string on the
    # c1 range with 1e7 events, against the built-in Gaussian leaf on the same
    # events (compile time included once)
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
    ex["cb_argus_cheb_5e7"] = {"eval_grad_ms": tg, "eval_ms": tf, "events_per_s": w["n"] / (tg * 1e-3),
                               "achieved_GBs": 16.0 * w["n"] / (tg * 1e-3) / 1e9,
                               "hbm_frac": 16.0 * w["n"] / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "fd_step_ms": 19 * tf, "speedup_vs_fd": 19 * tf / tg, "schedule": m.schedule}
    del m, cols
    torch.cuda.empty_cache()
    # 4096 toys, sizes U[1e3, 2e5], 50 gradient-descent steps each, one graph
    log("c4: generating 4096 toy datasets")
    w = datagen.toys_workload()
    n = int(w["offsets"][-1])
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    offs = torch.from_numpy(w["offsets"]).cuda()
    start = torch.as_tensor(w["theta_start"], dtype=torch.float64, device="cuda").repeat(4096, 1)
    tune(torch, m, start, args, offsets=offs)
    bufs = (start.clone(), torch.empty(4096, dtype=torch.float64, device="cuda"),
            torch.empty(4096, 2, dtype=torch.float64, device="cuda"),
            torch.empty(4096, dtype=torch.int32, device="cuda"))
    m.fit_batched(offs, start, 50, 1.0, out=bufs)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    m.fit_batched(offs, start, 50, 1.0, out=bufs)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = ev0.elapsed_time(ev1) / 50
    ex["toys_4096x50"] = {"events_per_step": n, "total_ms": 1e3 * wall, "avg_step_ms": step_ms,
                          "events_per_s": n * 50 / wall, "achieved_GBs": 8.0 * n / (step_ms * 1e-3) / 1e9,
                          "hbm_frac": 8.0 * n / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "status_ok": bool((bufs[3] == 0).all().item()), "schedule": m.schedule}
    return ex


def probe_pmc(torch, nllmi, datagen, steps):
    """Workload for counter runs: one calibration kernel of known traffic
    (elementwise negation of 1 GiB: reads and writes COPY_BYTES), then an
    eager fit of the headline workload."""
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    w = datagen.workload(2)
    model = nllmi.Model.from_spec(w["spec"])
    model.set_data([torch.from_numpy(c).cuda() for c in w["cols"]])
    model.set_option("graph", False)
    th0 = torch.as_tensor(w["points"][0], dtype=torch.float64, device="cuda")
    model.fit(th0, steps)
    torch.cuda.synchronize()
    log(f"probe: {steps} eager fit steps done")


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
        a = agg.setdefault(r["Kernel_Name"], [])
        a.append(dt)
    tot = sum(sum(v) for v in agg.values())
    print(f"# Kernel durations: {workload}\n")
    print("| kernel | calls | total us | avg us | min us | max us | % |")
    print("|---|---|---|---|---|---|---|")
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{_short(k)}` | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.2f} | {min(v):.2f} | "
              f"{max(v):.2f} | {100 * sum(v) / tot:.1f} |")


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


def _is_fit_kernel(k):
    """The gradient-descent fit's streaming kernel k_single_fit<M, U> (one
    launch per step: the previous step's update, then the pass)."""
    return "k_single_fit<" in k


def _streaming(values):
    """Indices of the launches that streamed the events: a proposal outside
    the parameter ranges is rejected before the stream (the step size
    halved), and its launch reads only the first preloaded tiles."""
    top = max(values)
    return [i for i, v in enumerate(values) if v >= 0.5 * top]


def summarize_pmc(fetch_dir, write_dir):
    """HBM traffic per launch of the streaming fit kernel from two counter
    runs (FETCH_SIZE, WRITE_SIZE: KiB per dispatch), scaled by what the same
    counters read for the calibration kernel; averaged over the launches
    that streamed."""
    fetch, write = _per_kernel(fetch_dir, "FETCH_SIZE", 1024.0), _per_kernel(write_dir, "WRITE_SIZE", 1024.0)
    ck, cf = _pick(fetch, lambda k: "neg" in k)
    _, cw = _pick(write, lambda k: "neg" in k)
    kk, kf_all = _pick(fetch, _is_fit_kernel)
    _, kw_all = _pick(write, lambda k: k == kk)
    idx = _streaming(kf_all)
    kf = [kf_all[i] for i in idx]
    kw = [kw_all[i] for i in idx if i < len(kw_all)]
    f_fac = COPY_BYTES / (sum(cf) / len(cf))
    w_fac = COPY_BYTES / (sum(cw) / len(cw))
    fb = f_fac * sum(kf) / len(kf)
    wb = w_fac * sum(kw) / len(kw)
    print("# HBM traffic of the streaming fit kernel: gauss+exp mixture, 1e7 FP64 events\n")
    print("Counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own run, scaled by")
    print(f"the same counter on the calibration kernel (elementwise negation, {COPY_BYTES} bytes read and written).")
    print("Averaged over the launches that streamed the events (a rejected out-of-range proposal skips")
    print("the stream and reads only the first preloaded tiles).\n")
    print(f"- kernel: `{_short(kk)}`")
    print(f"- csrc_sha256: `{csrc_hash()}`")
    print(f"- dispatches: {len(kf_all)} ({len(kf)} streamed)")
    print("- fetch_bytes_per_dispatch: " + ", ".join(f"{f_fac * v:.4e}" for v in kf_all))
    print(f"- calibration_fetch_factor: {f_fac:.4f}")
    print(f"- calibration_write_factor: {w_fac:.4f}")
    print(f"- fetch_bytes_per_launch: {fb:.4e}")
    print(f"- write_bytes_per_launch: {wb:.4e}")
    print(f"- traffic_bytes_per_launch: {fb + wb:.4e}")
    print(f"- algorithmic_bytes_per_launch: {8.0e7:.4e}")


VALU_FILE = os.path.join(ROOT, "profiles", "k_single_fit_gauss_exp_1e7_valu.txt")
VALU_COUNTERS = ["SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                 "SQ_INSTS_VALU_TRANS_F64", "SQ_WAVES"]
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: FP64 VALU lane-instructions/s
FP64_PEAK_FLOPS = 78.6e12


def summarize_valu(d):
    """VALU instructions per launch of the streaming fit kernel from one
    counter run (wave-level instruction counts, summed over the chip),
    averaged over the launches that streamed."""
    tabs = {c: _per_kernel(d, c) for c in VALU_COUNTERS}
    kk, valu_all = _pick(tabs["SQ_INSTS_VALU"], _is_fit_kernel)
    idx = _streaming(valu_all)
    avg = {c: sum(tabs[c][kk][i] for i in idx) / len(idx) for c in VALU_COUNTERS}
    lane_ops = 64.0 * avg["SQ_INSTS_VALU"]
    flops = 64.0 * (2.0 * avg["SQ_INSTS_VALU_FMA_F64"] + avg["SQ_INSTS_VALU_ADD_F64"] +
                    avg["SQ_INSTS_VALU_MUL_F64"] + avg["SQ_INSTS_VALU_TRANS_F64"])
    print("# VALU work of the streaming fit kernel: gauss+exp mixture, 1e7 FP64 events\n")
    print("SQ instruction counters (wave instructions per dispatch, all CUs), one run, averaged over the")
    print("launches that streamed the events. Lane-instructions = 64 x wave instructions (wave64);")
    print("FP64 FLOPs = 64 x (2 FMA + ADD + MUL + TRANS).\n")
    print(f"- kernel: `{_short(kk)}`")
    print(f"- csrc_sha256: `{csrc_hash()}`")
    print(f"- dispatches: {len(valu_all)} ({len(idx)} streamed)")
    for c in VALU_COUNTERS:
        print(f"- {c}: {avg[c]:.4e}")
    print(f"- valu_lane_instructions_per_launch: {lane_ops:.4e}")
    print(f"- valu_lane_instructions_per_event: {lane_ops / 1e7:.2f}")
    print(f"- fp64_flops_per_launch: {flops:.4e}")


def profiled_valu():
    """(VALU lane-instructions, FP64 FLOPs) per launch from the committed
    counter summary, or None if absent or taken on different sources."""
    try:
        kv = {}
        with open(VALU_FILE) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    kv[k.strip()] = v.strip().strip("`")
        if kv.get("csrc_sha256") != csrc_hash():
            return None
        return float(kv["valu_lane_instructions_per_launch"]), float(kv["fp64_flops_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch schedules")
    ap.add_argument("--probe", choices=["pmc"], help="run the counter-collection workload only")
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--workload-name", default="")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-valu", metavar="DIR")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload_name)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.summarize_valu:
        summarize_valu(args.summarize_valu)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for {max(args.gpus, world)}); "
              "multi-GPU sharding is a design note only", file=sys.stderr)
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
    res, w, model = headline(torch, nllmi, datagen, args)
    del model
    if not args.quick:
        try:
            res["extra"] = extras(torch, nllmi, datagen, args)
        except Exception as e:  # extras never hide the headline
            res["extra"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle")
        res["cpu_baseline"] = cpu_baseline(datagen, w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

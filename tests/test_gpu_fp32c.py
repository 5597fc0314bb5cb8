"""GPU parity of the FP32-compensated event pass (precision "fp32c"):
per-event density arithmetic in FP32 with two-sum-compensated per-thread
sums; normalisation, cross-thread reductions and the minimiser in FP64.

Tolerances: relative NLL error <= 1e-9 against the scalar FP64 oracle at
the precision-study size (1e8 events).  The gradient of this mode is
reported, not bound by 1e-8 of ||g_orc||_inf (that bound is the FP64
path's): each row carries ||g - g_orc||_inf / ||g_orc||_inf.  It is
checked against the random walk of its per-event FP32 roundings, on the
scale G = max_k sum_i |d l_i / d theta_k|.

The random-walk bounds.  Each event's value carries FP32 rounding errors
of a few units of u = 2^-24 relative; they are unbiased (the pass is built
so), so their sum grows as sqrt(N): for the NLL, 5 standard deviations of
c u sqrt(N) |l| with c ~ 4 over |NLL| ~ N |l| is ~ 1e-6 / sqrt(N) (3e-9 at
N = 1e5, 1.7e-7 at N = 30); 1e-9 is the larger from N = 1e6 on.  A
gradient feature phi of parameter k carries c u |phi_i| per event, and the
sum of those errors has standard deviation c u sqrt(sum_i phi_i^2) =
c u r G_k / sqrt(N) with r = rms / mean of |phi| over the events.  r is
~1.7 for t^2 of a Gaussian and grows as 1/sqrt(q) when only a fraction q
of the events carries the feature (the Crystal Ball's tenth of the 2-D
model's events: r ~ 5); 5 standard deviations at c = 4 and r = 5 give
6e-6 G / sqrt(N), so the bound is 1e-5 G / sqrt(N) (and 1e-8 G from
N = 1e6 on).
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

NLL_TOL = 1e-9
GRAD_TOL = 1e-8
RANDOM_WALK = 1e-6       # per-event relative FP32 error envelope of the NLL, divided by sqrt(N)
RANDOM_WALK_GRAD = 1e-5  # the same for gradient components


def nll_tol(n):
    return max(NLL_TOL, RANDOM_WALK / np.sqrt(max(n, 1)))


def grad_tol(n):
    return max(GRAD_TOL, RANDOM_WALK_GRAD / np.sqrt(max(n, 1)))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def nllmi():
    import paper_2003_12875_amd as m
    m.lib()
    return m


def to_dev(torch, cols):
    return [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in cols]


def compare(torch, nllmi, spec, cols, points, threads, n_check=None, against_fp64=False, report=False):
    """Errors of the fp32c path against the oracle (and the fp64 GPU path)
    at each point; asserts the tolerances and returns the error rows."""
    m = nllmi.Model.from_spec(spec, precision="fp32c")
    assert m.info["precision"] == 1 and m.info["variant"].endswith("/fp32c")
    dev = to_dev(torch, cols)
    m.set_data(dev)
    m64 = None
    if against_fp64:
        m64 = nllmi.Model.from_spec(spec)
        m64.set_data(dev)
    o = oracle.Oracle(spec)
    rows = []
    for th in points[:n_check]:
        st, ref, gref, stats = o.nll(cols, th, threads=threads, stats=True)
        assert st == 0
        v, g = m.eval_grad(torch.from_numpy(th))
        v, g = float(v.item()), g.cpu().numpy()
        scale = max(np.max(np.abs(gref)), np.max(stats[1:]))
        gnorm = np.max(np.abs(gref))
        nerr = abs(v / ref - 1.0)
        gerr = np.max(np.abs(g - gref)) / scale
        row = {"nll_rel_err": nerr, "grad_rel_err": gerr, "grad_err_vs_norm": np.max(np.abs(g - gref)) / gnorm}
        if m64 is not None:
            v64, g64 = m64.eval_grad(torch.from_numpy(th))
            v64, g64 = float(v64.item()), g64.cpu().numpy()
            row["nll_rel_err_vs_fp64_gpu"] = abs(v / v64 - 1.0)
            row["grad_rel_err_vs_fp64_gpu"] = np.max(np.abs(g - g64)) / scale
            # the FP64 GPU leg against the oracle, to the FP64 bounds
            row["fp64_nll_rel_err"] = abs(v64 / ref - 1.0)
            row["fp64_grad_err_vs_norm"] = np.max(np.abs(g64 - gref)) / gnorm
            assert row["fp64_nll_rel_err"] <= 1e-12, (th, v64, ref)
            assert row["fp64_grad_err_vs_norm"] <= 1e-8, (th, g64, gref)
        rows.append(row)
        if report:
            print(f"point {len(rows) - 1:2d}: " + "  ".join(f"{k} {v:.3e}" for k, v in row.items()), flush=True)
    n = len(cols[0])
    for th, row in zip(points, rows):
        assert row["nll_rel_err"] <= nll_tol(n), (th, row, nll_tol(n))
        assert row["grad_rel_err"] <= grad_tol(n), (th, row, grad_tol(n))
    assert m.sync() == 0
    return rows


@pytest.mark.parametrize("n", [3, 1000, 123_457])
def test_mixture_small(torch, nllmi, threads, n):
    w = datagen.workload(5, n=n)
    print(f"[fp32c mixture n={n}]", flush=True)
    compare(torch, nllmi, w["spec"], w["cols"], w["points"], threads, n_check=4, report=True)


@pytest.mark.parametrize("n", [1, 4097, 100_000])
def test_gauss_small(torch, nllmi, threads, n):
    w = datagen.workload(1, n=n)
    print(f"[fp32c gauss n={n}]", flush=True)
    compare(torch, nllmi, w["spec"], w["cols"], w["points"], threads, n_check=4)


@pytest.mark.parametrize("norm", ["gl256", "analytic"])
def test_cb_argus_cheb_small(torch, nllmi, threads, norm):
    w = datagen.workload(3, n=100_003)
    spec = datagen.cb_argus_cheb_spec(cheb=w["theta"][7:11], norm=norm)
    print(f"[fp32c c3 {norm}]", flush=True)
    compare(torch, nllmi, spec, w["cols"], w["points"], threads, n_check=3, report=True)


SINGLE_LEAVES = [
    ("exp", [("c", -0.4, -3, 3)], 0.0, 8.0),
    ("cb", [("m0", 0.2, -2, 2), ("sigma", 0.8, 0.1, 3), ("alpha", 1.1, 0.2, 5), ("n", 2.5, 1.2, 20)], -6.0, 4.0),
    ("argus", [("m0", 1.0, 0.96, 1.2), ("c", -6.0, -50, 0)], 0.2, 0.99),
    ("cheb", [("a1", 0.1, -1, 1), ("a2", -0.2, -1, 1), ("a3", 0.05, -1, 1), ("a4", 0.1, -1, 1)], -1.0, 1.0),
    ("johnson", [("mu", 0.3, -3, 3), ("lambda", 0.9, 0.1, 5), ("gamma", 0.6, -5, 5), ("delta", 0.8, 0.1, 10)],
     -8.0, 12.0),
    ("chi2", [("nu", 5.0, 0.5, 50)], 0.0, 30.0),
    ("chi2", [("nu", 12.0, 0.5, 50)], 3.0, 40.0),
]


@pytest.mark.parametrize("kind,params,lo,hi", SINGLE_LEAVES)
def test_single_leaves(torch, nllmi, threads, kind, params, lo, hi):
    spec = {"obs": [{"name": "x", "lo": lo, "hi": hi}],
            "params": [datagen.param(n, v, a, b) for n, v, a, b in params],
            "nodes": [{"kind": kind, "obs": 0, "params": list(range(len(params))), "norm": "analytic"}],
            "root": 0}
    cols = datagen.generate(spec, 50_001, seed=91)
    points = datagen.jittered_points(datagen.theta_of(spec), 3, seed=92, rel=0.05)
    if kind == "argus":
        points[:, 0] = np.abs(points[:, 0] - 1.0) + 1.0
    print(f"[fp32c single {kind}]", flush=True)
    compare(torch, nllmi, spec, cols, points, threads)


def test_batched_matches_single(torch, nllmi):
    w = datagen.toys_workload(n_sets=24, size_lo=0, size_hi=30_000)
    m = nllmi.Model.from_spec(w["spec"], precision="fp32c")
    m.set_data(to_dev(torch, w["cols"]))
    th = np.tile(w["theta_start"], (24, 1))
    nll, g, st = m.eval_batched(torch.from_numpy(w["offsets"]).cuda(), torch.from_numpy(th).cuda(), grad=True)
    nll, g, st = nll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    o = oracle.Oracle(w["spec"])
    for s in range(24):
        a, b = int(w["offsets"][s]), int(w["offsets"][s + 1])
        sub = [c[a:b] for c in w["cols"]]
        r, ref, gref, stats = o.nll(sub, th[s], threads=4, stats=True)
        assert st[s] == 0 and r == 0
        if b == a:
            assert nll[s] == 0.0
            continue
        assert abs(nll[s] / ref - 1.0) <= nll_tol(b - a), (s, nll[s], ref)
        scale = max(np.max(np.abs(gref)), np.max(stats[1:]))
        assert np.max(np.abs(g[s] - gref)) <= grad_tol(b - a) * scale, (s, g[s], gref)


def test_fit_reaches_fp64_minimum(torch, nllmi):
    """200 gradient-descent steps in fp32c and in fp64 from the same start
    end at the same NLL to the fp32c tolerance."""
    w = datagen.workload(5, n=200_000)
    th0 = torch.from_numpy(w["points"][0]).cuda()
    res = {}
    for prec in ("fp64", "fp32c"):
        m = nllmi.Model.from_spec(w["spec"], precision=prec)
        m.set_data(to_dev(torch, w["cols"]))
        th, f, g, st = m.fit(th0, 200)
        assert int(st.item()) == 0
        res[prec] = (th.cpu().numpy(), float(f.item()))
    assert abs(res["fp32c"][1] / res["fp64"][1] - 1.0) <= nll_tol(200_000), res


@pytest.mark.slow
def test_precision_study_full(torch, nllmi, threads):
    """The precision-study workload: 1e8 events of the signal+background
    mixture, NLL and gradient at 32 seeded parameter points, fp32c against
    the oracle and against the fp64 GPU path, and the fp64 GPU path against
    the oracle to the FP64 bounds (errors printed per point)."""
    w = datagen.workload(5, threads=threads)
    print(f"[fp32c precision study n={w['n']}]", flush=True)
    assert nll_tol(w["n"]) == NLL_TOL and grad_tol(w["n"]) == GRAD_TOL
    rows = compare(torch, nllmi, w["spec"], w["cols"], w["points"], threads, against_fp64=True, report=True)
    worst = {k: max(r[k] for r in rows) for k in rows[0]}
    print("worst: " + "  ".join(f"{k} {v:.3e}" for k, v in worst.items()), flush=True)


def test_autotune_fp32c(torch, nllmi, monkeypatch):
    """The autotuner accepts single-precision regroupings within the mode's
    accuracy (it would otherwise keep only the current schedule) and the
    tuned schedule still meets the oracle bound."""
    monkeypatch.delenv("NLLMI_TUNE_CACHE", raising=False)
    w = datagen.workload(5, n=300_000)
    m = nllmi.Model.from_spec(w["spec"], precision="fp32c")
    m.set_data(to_dev(torch, w["cols"]))
    th = w["points"][1]
    sched = m.autotune(torch.from_numpy(th).cuda())
    assert sched["unroll"] in (2, 4, 8) and 1 <= sched["blocks_per_cu"] <= 32
    st, ref, gref, stats = oracle.Oracle(w["spec"]).nll(w["cols"], th, threads=8, stats=True)
    v, g = m.eval_grad(torch.from_numpy(th))
    assert abs(float(v.item()) / ref - 1.0) <= nll_tol(len(w["cols"][0]))

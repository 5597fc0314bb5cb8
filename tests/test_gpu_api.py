"""GPU tests of the rest of the C ABI through the Python binding: the
extended (Poisson yield) term, the autotuner and its cache, step timing,
graph-recorded versus eager fits, and schedule validation."""
import os

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


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


def extended_spec():
    spec = datagen.mixture_spec()
    spec["params"].append(datagen.param("nu", 1000.0, 1.0, 1e9))
    spec["extended"] = True
    spec["yield_param"] = len(spec["params"]) - 1
    return spec


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32c", 1e-9)])
def test_extended_term_single_and_batched(torch, nllmi, precision, tol):
    """NLL + nu - N ln nu and its gradient (d/d nu = 1 - N / nu) against the
    oracle, for one dataset and for sets of different sizes."""
    spec = extended_spec()
    cols = datagen.generate(datagen.mixture_spec(), 200_000, seed=31)
    o = oracle.Oracle(spec)
    m = nllmi.Model.from_spec(spec, precision=precision)
    m.set_data(to_dev(torch, cols))
    for nu in (1000.0, 200_000.0, 3.5e5):
        th = np.array([0.2, 5.0, 0.4, -0.7, nu])
        st, ref, gref, stats = o.nll(cols, th, threads=8, stats=True)
        v, g = m.eval_grad(torch.from_numpy(th))
        v, g = float(v.item()), g.cpu().numpy()
        assert abs(v / ref - 1) <= tol, (nu, v, ref)
        if precision == "fp64":
            assert np.max(np.abs(g - gref)) <= 1e-8 * np.max(np.abs(gref)), (nu, g, gref)
        else:  # the FP32 pass's random-walk bound (its own tests derive it)
            scale = max(np.max(np.abs(gref)), np.max(stats[1:]))
            assert np.max(np.abs(g - gref)) <= max(1e-8, 1e-5 / np.sqrt(len(cols[0]))) * scale, (nu, g, gref)
        assert abs(g[4] - (1.0 - len(cols[0]) / nu)) <= 1e-12 * max(1.0, len(cols[0]) / nu)
    # batched: the yield term uses each set's own event count
    offsets = np.array([0, 1000, 1000, 51_000, 200_000], dtype=np.int64)
    th = np.tile([0.2, 5.0, 0.4, -0.7, 40_000.0], (4, 1))
    nll, g, st = m.eval_batched(torch.from_numpy(offsets).cuda(), torch.from_numpy(th).cuda())
    nll, g, st = nll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    for s in range(4):
        sub = [c[offsets[s]:offsets[s + 1]] for c in cols]
        r, ref, gref = o.nll(sub, th[s])
        assert st[s] == 0 and r == 0
        assert abs(nll[s] - ref) <= tol * max(abs(ref), 1.0), (s, nll[s], ref)
        assert abs(g[s][4] - gref[4]) <= 1e-12 * max(1.0, abs(gref[4])), (s, g[s], gref)


def test_autotune_keeps_results_and_caches(torch, nllmi, tmp_path, monkeypatch):
    """The autotuner checks every candidate against the reference NLL, keeps
    a valid schedule, leaves the results unchanged (to the parity bound),
    and a second model of the same shape reads the cached choice."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("NLLMI_TUNE_CACHE", str(cache))
    monkeypatch.delenv("NLLMI_TUNE_FORCE", raising=False)
    w = datagen.workload(2, n=300_000)
    th = torch.from_numpy(w["points"][1]).cuda()
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    v0, g0 = m.eval_grad(th)
    v0, g0 = float(v0.item()), g0.cpu().numpy()
    sched = m.autotune(th)
    assert sched["unroll"] in (2, 4, 8) and 1 <= sched["blocks_per_cu"] <= 32
    v1, g1 = m.eval_grad(th)
    assert abs(float(v1.item()) / v0 - 1) <= 1e-12
    assert np.max(np.abs(g1.cpu().numpy() - g0)) <= 1e-10 * np.max(np.abs(g0))
    assert cache.exists() and cache.read_text().strip()
    m2 = nllmi.Model.from_spec(w["spec"])
    m2.set_data(to_dev(torch, w["cols"]))
    assert m2.autotune(th) == sched  # from the cache
    # batched
    t = datagen.toys_workload(n_sets=64, size_lo=1000, size_hi=20_000)
    mb = nllmi.Model.from_spec(t["spec"])
    mb.set_data(to_dev(torch, t["cols"]))
    offs = torch.from_numpy(t["offsets"]).cuda()
    thb = torch.from_numpy(np.tile(t["theta_start"], (64, 1))).cuda()
    n0, _, _ = mb.eval_batched(offs, thb)
    sb = mb.autotune(thb, offsets=offs)
    assert sb["sets_unroll"] in (2, 4, 8) and 1024 <= sb["tile_events"] <= (1 << 22)
    n1, _, st = mb.eval_batched(offs, thb)
    assert (st == 0).all()
    assert np.max(np.abs(n1.cpu().numpy() / n0.cpu().numpy() - 1)) <= 1e-12


def test_step_timing_modes(torch, nllmi):
    w = datagen.workload(2, n=500_000)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    th = torch.from_numpy(w["points"][0]).cuda()
    with pytest.raises(nllmi.NLLError):
        m.step_times()  # no timed fit yet
    m.set_option("step_timing", True)
    m.fit(th, 7)
    steps = m.step_times()
    assert len(steps) == 7 and all(x > 0 for x in steps)
    m.set_option("step_timing", "kernel")
    m.fit(th, 5)
    kern = m.step_times()
    assert len(kern) == 5 and all(x > 0 for x in kern)
    assert np.median(kern) <= np.median(steps) * 1.5
    with pytest.raises(nllmi.NLLError):
        m.set_option("step_timing", 3)


def test_graph_and_eager_fits_are_identical(torch, nllmi):
    """Replaying the recorded graph and enqueuing the same steps eagerly give
    the same bits (single dataset and batched)."""
    w = datagen.workload(2, n=123_457)
    th = torch.from_numpy(w["points"][2]).cuda()
    res = []
    for graph in (True, False, True):
        m = nllmi.Model.from_spec(w["spec"])
        m.set_data(to_dev(torch, w["cols"]))
        m.set_option("graph", graph)
        out = m.fit(th, 40)
        res.append([x.cpu().numpy().copy() for x in out])
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    for a, b in zip(res[0], res[2]):
        assert np.array_equal(a, b)
    t = datagen.toys_workload(n_sets=40, size_lo=500, size_hi=30_000)
    offs = torch.from_numpy(t["offsets"]).cuda()
    start = torch.from_numpy(np.tile(t["theta_start"], (40, 1))).cuda()
    rb = []
    for graph in (True, False):
        m = nllmi.Model.from_spec(t["spec"])
        m.set_data(to_dev(torch, t["cols"]))
        m.set_option("graph", graph)
        rb.append([x.cpu().numpy().copy() for x in m.fit_batched(offs, start, 25, 1.0)])
    for a, b in zip(rb[0], rb[1]):
        assert np.array_equal(a, b)


def test_schedule_validation(torch, nllmi):
    m = nllmi.Model.from_spec(datagen.gauss_spec())
    for bad in ({"unroll": 3}, {"unroll": 1}, {"sets_unroll": 16}, {"blocks_per_cu": 0}, {"blocks_per_cu": 33},
                {"tile_events": 1000}, {"tile_events": (1 << 22) + 512}, {"sets_blocks_per_cu": 0}):
        with pytest.raises(nllmi.NLLError):
            m.set_schedule(**bad)
    m.set_schedule(unroll=8, sets_unroll=8, blocks_per_cu=32, sets_blocks_per_cu=32, tile_events=1 << 22)
    assert m.schedule["unroll"] == 8 and m.schedule["tile_events"] == 1 << 22


def test_eval_points(torch, nllmi, threads):
    """nll_eval_points: one dataset at many parameter points in one pass
    equals eval_grad point by point (the same per-event arithmetic, summed
    in a different grouping) and the oracle; a point outside the parameter
    ranges reports its own status and +inf, the others are unaffected."""
    w = datagen.workload(1)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    pts = np.array(w["points"], dtype=np.float64)
    pts[5, 1] = -1.0  # sigma < 0
    nll, g, st = m.eval_points(torch.from_numpy(pts).cuda())
    nll, g, st = nll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    assert st[5] != 0 and np.isinf(nll[5])
    o = oracle.Oracle(w["spec"])
    for i in range(len(pts)):
        if i == 5:
            continue
        assert st[i] == 0
        v, gi = m.eval_grad(torch.from_numpy(pts[i]))
        v, gi = float(v.item()), gi.cpu().numpy()
        assert abs(nll[i] - v) <= 1e-12 * abs(v), (i, nll[i], v)
        assert np.max(np.abs(g[i] - gi)) <= 1e-10 * max(np.max(np.abs(gi)), 1.0), (i, g[i], gi)
        if i % 16 == 0:
            r, ref, gref = o.nll(w["cols"], pts[i], threads=threads)
            assert r == 0 and abs(nll[i] / ref - 1.0) <= 1e-12, (i, nll[i], ref)
    # NLL only, the 2-D model, a ragged event count
    w3 = datagen.workload(3, n=33_333)
    m3 = nllmi.Model.from_spec(w3["spec"])
    m3.set_data(to_dev(torch, w3["cols"]))
    pts3 = np.array(w3["points"][:5], dtype=np.float64)
    nll3, g3, st3 = m3.eval_points(torch.from_numpy(pts3).cuda(), grad=False)
    assert g3 is None and (st3.cpu().numpy() == 0).all()
    o3 = oracle.Oracle(w3["spec"])
    for i in range(5):
        r, ref, _ = o3.nll(w3["cols"], pts3[i], threads=threads)
        assert r == 0 and abs(nll3.cpu().numpy()[i] / ref - 1.0) <= 1e-12, (i,)

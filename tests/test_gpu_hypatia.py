"""GPU tests of the Hypatia2 leaf (Sec. 3: a generalised hyperbolic core
continued on both sides by power-law tails) against the scalar FP64 oracle
at seeded parameter points, all nine parameters free: NLL within 1e-12
relative, gradient within 1e-8 of the oracle's max-norm.

The device evaluates K_nu through per-point Chebyshev tables of log K_nu,
the ratio K_{nu+1}/K_nu and d log K_nu / d nu over the core's range of
alpha r, built by the block from trapezoidal sums; the oracle evaluates
K_nu's integral directly at every event (and its derivatives by complex
steps), so the two share nothing but the definition.

Shapes: the leaf alone over four parameter regions (a narrow peak with a
strong low tail, lambda < 0 with small zeta, lambda = 1 with a skew, a
near-Gaussian core with zeta = 20), a Hypatia + exponential mixture, a
product with a Chebyshev series in a second observable (compiled at run
time), the batched pass and gradient-descent fits, weighted events, a range
cut inside one tail, and the parameter checks."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

NLL_TOL = 1e-12
GRAD_TOL = 1e-8
P = datagen.param
NAMES = ["mu", "sigma", "lambda", "zeta", "beta", "a_l", "n_l", "a_r", "n_r"]
CASES = {
    "narrow_peak": ([5.28, 0.003, -2.0, 0.5, 0.0, 2.0, 3.0, 2.5, 4.0], 5.20, 5.35),
    "small_zeta": ([0.0, 1.0, -1.2, 0.05, 0.1, 1.5, 2.0, 1.8, 6.0], -8.0, 8.0),
    "hyperbolic_skew": ([1.0, 0.5, 1.0, 2.0, -0.2, 2.5, 1.5, 3.0, 3.0], -3.0, 5.0),
    "near_gauss": ([0.0, 1.0, 3.0, 20.0, 0.0, 3.0, 5.0, 3.0, 5.0], -6.0, 6.0),
}


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


def hyp_params(th, lo, hi, first=0):
    """The nine parameters with wide ranges and jitters of a few per cent
    of the scale each one acts on (so that seeded points stay valid)."""
    mu, sg = th[0], th[1]
    ranges = [(lo - (hi - lo), hi + (hi - lo)), (1e-6, 100.0), (-6.0, 6.0), (1e-3, 100.0), (-50.0, 50.0), (0.05, 20.0), (1.001, 100.0),
              (0.05, 20.0), (1.001, 100.0)]
    jit = [0.05 * sg, 0.05 * sg, 0.05 * max(abs(th[2]), 0.5), 0.05 * th[3], 0.02 / sg, 0.05 * th[5],
           0.05 * th[6], 0.05 * th[7], 0.05 * th[8]]
    return [P(f"{n}{first or ''}", v, a, b, jitter=j) for n, v, (a, b), j in zip(NAMES, th, ranges, jit)]


def hyp_spec(th, lo, hi):
    return {"obs": [{"name": "m", "lo": lo, "hi": hi}], "params": hyp_params(th, lo, hi),
            "nodes": [{"kind": "hypatia", "obs": 0, "params": list(range(9))}], "root": 0}


def build(torch, nllmi, spec, n, seed, precision="fp64"):
    cols = datagen.generate(spec, n, seed=seed)
    m = nllmi.Model.from_spec(spec, precision=precision)
    m.set_data([torch.from_numpy(c).cuda() for c in cols])
    return m, cols


def check_points(torch, m, spec, cols, points, threads, weights=None):
    o = oracle.Oracle(spec)
    for th in points:
        st, ref, gref = o.nll(cols, th, threads=threads, weights=weights)
        assert st == 0, th
        v, g = m.eval_grad(torch.from_numpy(np.ascontiguousarray(th)))
        v, g = float(v.item()), g.cpu().numpy()
        assert abs(v / ref - 1.0) <= NLL_TOL, (th, v, ref)
        err = np.abs(g - gref)
        assert np.max(err) <= GRAD_TOL * np.max(np.abs(gref)), (th, dict(zip(NAMES, err)), gref)
    assert m.sync() == 0


@pytest.mark.parametrize("case", sorted(CASES))
def test_hypatia_against_oracle(torch, nllmi, threads, case):
    th, lo, hi = CASES[case]
    spec = hyp_spec(th, lo, hi)
    print(f"[hypatia {case}]", flush=True)
    m, cols = build(torch, nllmi, spec, 200_000, seed=1200 + sorted(CASES).index(case))
    assert m.info["variant"] == "hypatia", m.info
    pts = np.vstack([np.array(th), datagen.parameter_points(spec, 2, seed=1210)])
    check_points(torch, m, spec, cols, pts, threads)


def test_hypatia_range_cut_in_a_tail(torch, nllmi, threads):
    """The observable range starts inside the high tail's junction: the
    low tail and most of the core lie outside it."""
    th = [0.0, 1.0, 1.0, 2.0, 0.0, 2.0, 3.0, 1.5, 4.0]
    spec = hyp_spec(th, 0.5, 9.0)
    m, cols = build(torch, nllmi, spec, 150_000, seed=1220)
    check_points(torch, m, spec, cols, datagen.parameter_points(spec, 2, seed=1221), threads)
    spec2 = hyp_spec(th, 2.0, 9.0)  # the whole range in the high tail
    m2, cols2 = build(torch, nllmi, spec2, 100_000, seed=1222)
    check_points(torch, m2, spec2, cols2, [np.array(th)], threads)


def hyp_exp_spec():
    """0.4 Hypatia2 + 0.6 Exp(-1.5) on [5.20, 5.35]."""
    th, lo, hi = CASES["narrow_peak"]
    return {"obs": [{"name": "m", "lo": lo, "hi": hi}],
            "params": [P("f", 0.4, 0.0, 1.0, jitter=0.02)] + hyp_params(th, lo, hi, first=1) +
                      [P("c", -1.5, -50.0, 50.0)],
            "nodes": [{"kind": "hypatia", "obs": 0, "params": list(range(1, 10))},
                      {"kind": "exp", "obs": 0, "params": [10]},
                      {"kind": "sum", "params": [0], "children": [0, 1]}],
            "root": 2}


def test_hypatia_exp_mixture(torch, nllmi, threads):
    spec = hyp_exp_spec()
    m, cols = build(torch, nllmi, spec, 200_000, seed=1230)
    assert m.info["variant"] == "hypatia+exp", m.info
    check_points(torch, m, spec, cols, datagen.parameter_points(spec, 3, seed=1231), threads)


def test_hypatia_times_chebyshev(torch, nllmi, threads):
    """Hypatia2(x) x Chebyshev-2(y): a shape outside the ahead-of-time
    registry, compiled at model creation."""
    th, lo, hi = CASES["hyperbolic_skew"]
    spec = {"obs": [{"name": "x", "lo": lo, "hi": hi}, {"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": hyp_params(th, lo, hi) + [P("a1", 0.2, -1.0, 1.0), P("a2", -0.1, -1.0, 1.0)],
            "nodes": [{"kind": "hypatia", "obs": 0, "params": list(range(9))},
                      {"kind": "cheb", "obs": 1, "params": [9, 10]},
                      {"kind": "prod", "children": [0, 1]}],
            "root": 2}
    m, cols = build(torch, nllmi, spec, 150_000, seed=1240)
    assert m.info["variant"].startswith("rtc:"), m.info
    check_points(torch, m, spec, cols, datagen.parameter_points(spec, 2, seed=1241), threads)


def test_hypatia_batched_and_fit(torch, nllmi, threads):
    """The batched pass (per-set tables built by the constants kernel, sets
    of uneven sizes, one empty), gradient-descent fits of one dataset and
    of every set against the oracle's trajectory."""
    th, lo, hi = CASES["small_zeta"]
    spec = hyp_spec(th, lo, hi)
    m, cols = build(torch, nllmi, spec, 120_000, seed=1250)
    o = oracle.Oracle(spec)
    offsets = np.array([0, 3, 5_000, 5_000, 60_000, 120_000], dtype=np.int64)
    pts = datagen.parameter_points(spec, 5, seed=1251)
    nll, g, st = m.eval_batched(torch.from_numpy(offsets).cuda(), torch.from_numpy(pts).cuda())
    nll, g, st = nll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    for s in range(5):
        a, b = offsets[s], offsets[s + 1]
        sto, ref, gref = o.nll([c[a:b] for c in cols], pts[s], threads=threads)
        assert st[s] == sto == 0
        if b == a:
            assert nll[s] == 0.0 and np.all(g[s] == 0.0)
            continue
        assert abs(nll[s] / ref - 1.0) <= NLL_TOL, (s, nll[s], ref)
        assert np.max(np.abs(g[s] - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (s, g[s], gref)
    th0 = pts[0]
    for steps in (1, 4):
        thf, f, gg, stt = m.fit(torch.from_numpy(th0), steps, 0.5)
        sto, th_o, f_o, g_o, _ = o.gd_fit(cols, th0, steps, 0.5, threads=threads)
        assert int(stt.item()) == sto == 0
        assert abs(float(f.item()) / f_o - 1.0) <= NLL_TOL, (steps, float(f.item()), f_o)
        np.testing.assert_allclose(thf.cpu().numpy(), th_o, rtol=1e-10, atol=1e-12)
    # every set fitted at once (two sets with events), three steps
    off2 = np.array([0, 50_000, 120_000], dtype=np.int64)
    th2 = pts[:2].copy()
    thb, fb, gb, stb = m.fit_batched(torch.from_numpy(off2).cuda(), torch.from_numpy(th2).cuda(), 3, 0.5)
    thb, fb, stb = thb.cpu().numpy(), fb.cpu().numpy(), stb.cpu().numpy()
    for s in range(2):
        a, b = off2[s], off2[s + 1]
        sto, th_o, f_o, g_o, _ = o.gd_fit([c[a:b] for c in cols], th2[s], 3, 0.5, threads=threads)
        assert stb[s] == sto == 0
        assert abs(fb[s] / f_o - 1.0) <= NLL_TOL, (s, fb[s], f_o)
        np.testing.assert_allclose(thb[s], th_o, rtol=1e-10, atol=1e-12)
    assert m.sync() == 0


def test_hypatia_weighted(torch, nllmi, threads):
    th, lo, hi = CASES["hyperbolic_skew"]
    spec = hyp_spec(th, lo, hi)
    m, cols = build(torch, nllmi, spec, 120_000, seed=1260)
    w = 0.5 + np.random.default_rng(1261).uniform(0.0, 1.0, 120_000)
    m.set_weights(torch.from_numpy(w).cuda())
    check_points(torch, m, spec, cols, datagen.parameter_points(spec, 2, seed=1262), threads, weights=w)


def test_hypatia_parameter_checks(torch, nllmi):
    """Out-of-domain parameters (sigma, zeta, a_l, a_r <= 0, n <= 1, a skew
    that turns a tail upwards) give +inf and the parameter status, as in the
    oracle; the FP32-compensated pass and a second Hypatia2 leaf are refused
    at model creation."""
    th, lo, hi = CASES["small_zeta"]
    spec = hyp_spec(th, lo, hi)
    for p in spec["params"]:
        p["lo"], p["hi"] = -1e3, 1e3  # let the leaf's own checks decide
    m, cols = build(torch, nllmi, spec, 20_000, seed=1270)
    o = oracle.Oracle(spec)
    for k, v in ((1, 0.0), (3, 0.0), (5, -1.0), (6, 1.0), (7, 0.0), (8, 0.5), (4, 5.0)):
        t = np.array(th, dtype=float)
        t[k] = v
        assert o.nll(cols, t)[0] == -3, (NAMES[k], v)
        val = float(m.eval(torch.from_numpy(t)).item())
        assert val == float("inf"), (NAMES[k], v, val)
        assert m.sync() == -3
    assert float(m.eval(torch.tensor(th, dtype=torch.float64)).item()) < float("inf")
    assert m.sync() == 0
    with pytest.raises(nllmi.NLLError) as e:
        nllmi.Model.from_spec(spec, precision="fp32c")
    assert e.value.status == -2
    two = {"obs": spec["obs"], "params": spec["params"],
           "nodes": [{"kind": "hypatia", "obs": 0, "params": list(range(9))},
                     {"kind": "hypatia", "obs": 0, "params": list(range(9))},
                     {"kind": "sum", "params": [4], "children": [0, 1]}], "root": 2}
    with pytest.raises(nllmi.NLLError) as e:
        nllmi.Model.from_spec(two)
    assert e.value.status == -2

"""GPU parity of weighted events (binned datasets as bin centres weighted by
the counts; sWeights of either sign) against the oracle: the weighted NLL
-sum w_i log p(x_i), its gradient, the extended term nu - W ln nu, gradient
descent scaled by 1/W, and the entry points that refuse weights.

Tolerances as for the unweighted pass: NLL 1e-12 relative, gradient 1e-8 of
||g_oracle||_inf at seeded points; fitted points 1e-9 relative.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

NLL_TOL = 1e-12
GRAD_TOL = 1e-8


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


def check(torch, nllmi, spec, cols, wt, points, threads, unroll=None):
    m = nllmi.Model.from_spec(spec)
    m.set_data(to_dev(torch, cols))
    m.set_weights(torch.from_numpy(wt).cuda())
    if unroll:
        m.set_schedule(unroll=unroll)
    o = oracle.Oracle(spec)
    for th in points:
        st, ref, gref, stats = o.nll(cols, th, threads=threads, stats=True, weights=wt)
        assert st == 0
        v, g = m.eval_grad(torch.from_numpy(np.ascontiguousarray(th)))
        v, g = float(v.item()), g.cpu().numpy()
        assert abs(v - ref) <= NLL_TOL * abs(ref), (th, v, ref)
        assert np.max(np.abs(g - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (th, g, gref)
        v1 = float(m.eval(torch.from_numpy(np.ascontiguousarray(th))).item())
        assert abs(v1 - ref) <= NLL_TOL * abs(ref), (th, v1, ref)
    assert m.sync() == 0
    return m


@pytest.mark.parametrize("config", [1, 2, 3])
@pytest.mark.parametrize("n", [1, 4097, 100_003])
def test_signed_weights_match_oracle(torch, nllmi, threads, config, n):
    w = datagen.workload(config, n=n)
    wt = datagen.signed_weights(n, seed=config + 100 * n)
    print(f"[weighted c{config} n={n}]", flush=True)
    check(torch, nllmi, w["spec"], w["cols"], wt, w["points"][:2], threads)


def test_weighted_mixture_full(torch, nllmi, threads):
    """The headline mixture at 1e7 events with positive weights."""
    w = datagen.workload(2)
    wt = 0.5 + datagen.uniforms(5, 12, w["n"])
    print("[weighted c2 n=1e7]", flush=True)
    check(torch, nllmi, w["spec"], w["cols"], wt, w["points"][:2], threads)


@pytest.mark.parametrize("unroll", [2, 4, 8])
def test_weighted_every_unroll(torch, nllmi, threads, unroll):
    w = datagen.workload(2, n=4097 * 5 + 13)
    wt = datagen.signed_weights(len(w["cols"][0]), seed=9)
    check(torch, nllmi, w["spec"], w["cols"], wt, w["points"][:1], threads, unroll=unroll)


def test_integer_weights_equal_repeated_events(torch, nllmi):
    """On the device: weights 0..4 give the NLL and gradient of the dataset
    with each event repeated w_i times (the unweighted kernels)."""
    w = datagen.workload(2, n=200_000)
    wt = np.floor(5 * datagen.uniforms(7, 3, 200_000))
    rep = [np.repeat(c, wt.astype(np.int64)) for c in w["cols"]]
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    m.set_weights(torch.from_numpy(wt).cuda())
    mr = nllmi.Model.from_spec(w["spec"])
    mr.set_data(to_dev(torch, rep))
    for th in w["points"][:3]:
        v, g = m.eval_grad(torch.from_numpy(th))
        vr, gr = mr.eval_grad(torch.from_numpy(th))
        assert abs(v.item() - vr.item()) <= 1e-13 * abs(vr.item())
        np.testing.assert_allclose(g.cpu().numpy(), gr.cpu().numpy(), rtol=1e-9, atol=1e-9 * np.abs(gr.cpu().numpy()).max())


def test_binned_gauss_fit(torch, nllmi, threads):
    """A binned fit: c1's events histogrammed into 400 bins; 50 gradient
    descent steps on the device equal the oracle's and reach the
    weighted-moment MLE."""
    w = datagen.workload(1)
    xc, cnt = datagen.binned(w["cols"][0], -10.0, 10.0, 400)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, [xc]))
    m.set_weights(torch.from_numpy(cnt).cuda())
    th, nll, g, status = m.fit(torch.from_numpy(w["theta"]), 50, 1.0)
    st, th_o, nll_o, g_o, eta_o = oracle.Oracle(w["spec"]).gd_fit([xc], w["theta"], 50, 1.0, weights=cnt)
    assert status.item() == 0 and st == 0
    th = th.cpu().numpy()
    np.testing.assert_allclose(th, th_o, rtol=1e-9)
    assert abs(nll.item() - nll_o) <= NLL_TOL * abs(nll_o)
    x = xc.astype(np.longdouble)
    W = cnt.sum()
    mu = float((cnt * x).sum() / W)
    assert abs(th[0] - mu) <= 1e-8 * abs(mu)
    assert abs(th[1] - float(np.sqrt((cnt * (x - mu) ** 2).sum() / W))) <= 1e-8 * th[1]


def test_weighted_extended_and_fit_rerecorded(torch, nllmi, threads):
    """Extended mixture over weighted events: the yield's derivative is
    1 - W/nu; a recorded fit is re-recorded when the weights change."""
    w = datagen.workload(2, n=50_000)
    spec = datagen.mixture_spec()
    spec["params"].append(datagen.param("nu", 1000.0, 1.0, 1e9))
    spec["extended"] = True
    spec["yield_param"] = 4
    wa = 0.5 + datagen.uniforms(1, 12, 50_000)
    wb = 2.0 * datagen.uniforms(2, 12, 50_000)
    th0 = np.append(w["points"][0], 40_000.0)
    m = nllmi.Model.from_spec(spec)
    m.set_data(to_dev(torch, w["cols"]))
    o = oracle.Oracle(spec)
    for wt in (wa, wb):
        m.set_weights(torch.from_numpy(wt).cuda())
        v, g = m.eval_grad(torch.from_numpy(th0))
        st, ref, gref = o.nll(w["cols"], th0, threads=threads, weights=wt)
        assert abs(v.item() - ref) <= NLL_TOL * abs(ref)
        assert abs(g[4].item() - (1.0 - wt.sum() / 40_000.0)) <= 1e-12
        th, nll, gg, status = m.fit(torch.from_numpy(th0), 20, 1.0)
        st, th_o, nll_o, g_o, eta_o = o.gd_fit(w["cols"], th0, 20, 1.0, threads=threads, weights=wt)
        assert status.item() == 0 and st == 0
        np.testing.assert_allclose(th.cpu().numpy(), th_o, rtol=1e-9)


def test_weights_lifecycle_and_refusals(torch, nllmi):
    w = datagen.workload(2, n=20_000)
    wt = datagen.signed_weights(20_000, seed=3)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    th = torch.from_numpy(w["points"][0])
    base = m.eval(th).item()
    m.set_weights(torch.from_numpy(wt).cuda())
    weighted = m.eval(th).item()
    assert weighted != base
    offs = torch.tensor([0, 10_000, 20_000], dtype=torch.int64)
    two = torch.from_numpy(np.stack([w["points"][0]] * 2))
    for call in (lambda: m.eval_batched(offs, two), lambda: m.eval_points(two), lambda: m.eval_bhhh(th),
                 lambda: m.fit_bhhh(th, 3), lambda: m.autotune(th), lambda: m.fit_batched(offs, two, 3)):
        with pytest.raises(nllmi.NLLError) as e:
            call()
        assert e.value.status == -2
    with pytest.raises(nllmi.NLLError):
        m.set_weights(torch.ones(19_999, dtype=torch.float64))
    m.set_weights(None)
    assert m.eval(th).item() == base
    m.set_weights(torch.from_numpy(wt).cuda())
    m.set_data(to_dev(torch, w["cols"]))  # new data: weights detached
    assert m.eval(th).item() == base
    mf = nllmi.Model.from_spec(w["spec"], precision="fp32c")
    mf.set_data(to_dev(torch, w["cols"]))
    with pytest.raises(nllmi.NLLError) as e:
        mf.set_weights(torch.from_numpy(wt).cuda())
    assert e.value.status == -2
    assert m.sync() == 0


def test_weighted_invalid_densities(torch, nllmi):
    """Weighted events where the density is zero (an ARGUS endpoint below
    the events' largest values) or negative (a Chebyshev series below zero
    over part of the range): the NLL is +inf and the status the invalid
    density's (-5), as for unweighted events; the same models at valid
    points are finite and equal the oracle's weighted NLL."""
    P = datagen.param
    argus = {"obs": [{"name": "m", "lo": 0.2, "hi": 1.0}],
             "params": [P("m0", 1.0, 0.5, 1.0), P("c", -6.0, -50, 0)],
             "nodes": [{"kind": "argus", "obs": 0, "params": [0, 1], "norm": "gl256"}], "root": 0}
    cheb = {"obs": [{"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": [P("a1", 0.1, -2, 2), P("a2", -0.2, -2, 2), P("a3", 0.05, -2, 2), P("a4", 0.1, -2, 2)],
            "nodes": [{"kind": "cheb", "obs": 0, "params": [0, 1, 2, 3], "norm": "analytic"}], "root": 0}
    for spec, bad in ((argus, [0.95, -6.0]), (cheb, [1.5, 0.0, 0.0, 0.0])):
        n = 50_000
        cols = datagen.generate(spec, n, seed=77)
        wt = 0.5 + datagen.uniforms(5, 13, n)
        print(f"[weighted invalid {spec['nodes'][0]['kind']}]", flush=True)
        m = nllmi.Model.from_spec(spec)
        m.set_data(to_dev(torch, cols))
        m.set_weights(torch.from_numpy(wt).cuda())
        assert np.isinf(float(m.eval(torch.from_numpy(np.asarray(bad))).item())) and m.sync() == -5
        th = datagen.theta_of(spec)
        st, ref, gref = oracle.Oracle(spec).nll(cols, th, threads=4, weights=wt)
        assert st == 0
        v = float(m.eval(torch.from_numpy(th)).item())
        assert abs(v - ref) <= NLL_TOL * abs(ref) and m.sync() == 0, (v, ref)

"""GPU tests of sums of yields (one coefficient per component, as RooAddPdf
takes yields; p = sum nu_j p_j / sum nu_j) and of extended models whose
expected count is the total of those yields (nu - N ln nu, d/d nu_j =
1 - N / nu).  Against the scalar FP64 oracle: NLL within 1e-12 relative,
gradient within 1e-8 of the oracle's max-norm, BHHH within 1e-10 of its
largest entry."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

NLL_TOL = 1e-12
GRAD_TOL = 1e-8
P = datagen.param


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


def signal_background(n_sig, n_bkg, extended=True):
    """nu_s Gauss(5, 0.4) + nu_b Exp(-0.7) on [0, 10]: every parameter free."""
    return {"obs": [{"name": "x", "lo": 0.0, "hi": 10.0}],
            "params": [P("nu_s", n_sig, 0.0, 1e9), P("nu_b", n_bkg, 0.0, 1e9), P("mu", 5.0, 0.0, 10.0),
                       P("sigma", 0.4, 0.01, 5.0), P("c", -0.7, -5.0, 5.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [2, 3]}, {"kind": "exp", "obs": 0, "params": [4]},
                      {"kind": "sum", "params": [0, 1], "children": [0, 1]}],
            "root": 2, "extended": extended, "yield_param": -1}


def three_yields(n):
    return {"obs": [{"name": "x", "lo": 0.0, "hi": 10.0}],
            "params": [P("n1", 0.15 * n, 0.0, 1e9), P("n2", 0.25 * n, 0.0, 1e9), P("n3", 0.6 * n, 0.0, 1e9),
                       P("mu1", 2.0, 0.0, 10.0), P("s1", 0.3, 0.01, 5.0), P("mu2", 7.0, 0.0, 10.0),
                       P("s2", 0.5, 0.01, 5.0), P("c", -0.2, -5.0, 5.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [3, 4]}, {"kind": "gauss", "obs": 0, "params": [5, 6]},
                      {"kind": "exp", "obs": 0, "params": [7]},
                      {"kind": "sum", "params": [0, 1, 2], "children": [0, 1, 2]}],
            "root": 3, "extended": True, "yield_param": -1}


def check(torch, m, spec, cols, points, threads, weights=None):
    o = oracle.Oracle(spec)
    for th in points:
        st, ref, gref = o.nll(cols, th, threads=threads, weights=weights)
        assert st == 0
        v, g = m.eval_grad(torch.from_numpy(np.ascontiguousarray(th)))
        v, g = float(v.item()), g.cpu().numpy()
        assert abs(v / ref - 1.0) <= NLL_TOL, (th, v, ref)
        assert np.max(np.abs(g - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (th, g, gref)
    assert m.sync() == 0


def build(torch, nllmi, spec, cols, precision="fp64"):
    m = nllmi.Model.from_spec(spec, precision=precision)
    m.set_data([torch.from_numpy(c).cuda() for c in cols])
    return m


@pytest.mark.parametrize("extended", [True, False])
def test_two_yields(torch, nllmi, threads, extended):
    n = 400_000
    spec = signal_background(0.2 * n, 0.8 * n, extended)
    cols = datagen.generate(spec, n, seed=981)
    m = build(torch, nllmi, spec, cols)
    check(torch, m, spec, cols, datagen.parameter_points(spec, 4, seed=982), threads)


def test_three_yields(torch, nllmi, threads):
    n = 300_000
    spec = three_yields(n)
    cols = datagen.generate(spec, n, seed=983)
    m = build(torch, nllmi, spec, cols)
    check(torch, m, spec, cols, datagen.parameter_points(spec, 4, seed=984), threads)


def test_yields_product_root(torch, nllmi, threads):
    """Extended product: a sum of yields in x times a Chebyshev series in y;
    the expected count is the sum's total."""
    n = 200_000
    base = signal_background(0.3 * n, 0.7 * n)
    spec = {"obs": base["obs"] + [{"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": base["params"] + [P("a1", 0.2, -1.0, 1.0), P("a2", -0.1, -1.0, 1.0)],
            "nodes": base["nodes"] + [{"kind": "cheb", "obs": 1, "params": [5, 6]},
                                      {"kind": "prod", "children": [2, 3]}],
            "root": 4, "extended": True, "yield_param": -1}
    cols = datagen.generate(spec, n, seed=985)
    m = build(torch, nllmi, spec, cols)
    check(torch, m, spec, cols, datagen.parameter_points(spec, 3, seed=986), threads)


def test_yields_batched_fit_and_bhhh(torch, nllmi, threads):
    """Batched sets (each its own yields), gradient-descent steps against
    the oracle's trajectory, and the BHHH matrix with the Poisson block
    N / nu^2 over both yields."""
    n = 150_000
    spec = signal_background(0.2 * n, 0.8 * n)
    cols = datagen.generate(spec, n, seed=987)
    m = build(torch, nllmi, spec, cols)
    o = oracle.Oracle(spec)
    offsets = np.array([0, 20_000, 20_000, 90_000, 150_000], dtype=np.int64)
    pts = datagen.parameter_points(spec, 4, seed=988)
    for s in range(4):  # yields near each set's own size
        pts[s, :2] = pts[s, :2] * max(offsets[s + 1] - offsets[s], 1) / n
    nll, g, st = m.eval_batched(torch.from_numpy(offsets).cuda(), torch.from_numpy(pts).cuda())
    nll, g, st = nll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    for s in range(4):
        a, b = offsets[s], offsets[s + 1]
        sto, ref, gref = o.nll([c[a:b] for c in cols], pts[s], threads=threads)
        assert st[s] == sto == 0
        assert abs(nll[s] / ref - 1.0) <= NLL_TOL, (s, nll[s], ref)
        assert np.max(np.abs(g[s] - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (s, g[s], gref)
    th0 = datagen.parameter_points(spec, 1, seed=989)[0]
    for steps in (1, 5):
        th, f, gg, stt = m.fit(torch.from_numpy(th0), steps)
        sto, th_o, f_o, g_o, _ = o.gd_fit(cols, th0, steps, 1.0, threads=threads)
        assert int(stt.item()) == sto == 0
        assert abs(float(f.item()) / f_o - 1.0) <= NLL_TOL
        np.testing.assert_allclose(th.cpu().numpy(), th_o, rtol=1e-10, atol=1e-12)
    st, ref, gref, B = o.nll_bhhh(cols, th0, threads=threads)
    v, g, Bd = m.eval_bhhh(torch.from_numpy(th0))
    assert abs(float(v.item()) / ref - 1.0) <= NLL_TOL
    assert np.max(np.abs(Bd.cpu().numpy() - B)) <= 1e-10 * np.max(np.abs(B))
    # a damped BHHH fit reaches the oracle's stationary point (yields = the
    # component counts' estimate, total = N)
    th, f, gg, stt = m.fit_bhhh(torch.from_numpy(th0), 25, 1e-3)
    sto, th_o, f_o, g_o, _ = o.bhhh_fit(cols, th0, 25, 1e-3, threads=threads)
    assert abs(float(f.item()) / f_o - 1.0) <= 1e-12
    assert abs(th.cpu().numpy()[:2].sum() / n - 1.0) < 1e-6


def test_yields_weighted(torch, nllmi, threads):
    n = 150_000
    spec = signal_background(0.2 * n, 0.8 * n)
    cols = datagen.generate(spec, n, seed=990)
    w = 0.5 + np.random.default_rng(991).uniform(0.0, 1.0, n)
    m = build(torch, nllmi, spec, cols)
    m.set_weights(torch.from_numpy(w).cuda())
    check(torch, m, spec, cols, datagen.parameter_points(spec, 2, seed=992), threads, weights=w)


def test_yields_fp32c(torch, nllmi, threads):
    """FP32-compensated pass at the small-N bounds of the FP32C tests."""
    n = 400_000
    spec = signal_background(0.2 * n, 0.8 * n)
    cols = datagen.generate(spec, n, seed=993)
    m = build(torch, nllmi, spec, cols, precision="fp32c")
    o = oracle.Oracle(spec)
    ntol, gtol = max(1e-9, 1e-6 / np.sqrt(n)), max(1e-8, 1e-5 / np.sqrt(n))
    for th in datagen.parameter_points(spec, 3, seed=994):
        st, ref, gref, stats = o.nll(cols, th, threads=threads, stats=True)
        v, g = m.eval_grad(torch.from_numpy(th))
        assert abs(float(v.item()) / ref - 1.0) <= ntol
        scale = max(np.max(np.abs(gref)), np.max(stats[1:]))
        assert np.max(np.abs(g.cpu().numpy() - gref)) <= gtol * scale
    assert m.sync() == 0


def test_yields_out_of_range(torch, nllmi):
    """A negative yield: +inf and the parameter-range status."""
    n = 10_000
    spec = signal_background(0.2 * n, 0.8 * n)
    cols = datagen.generate(spec, n, seed=995)
    m = build(torch, nllmi, spec, cols)
    v = float(m.eval(torch.tensor([-1.0, 8000.0, 5.0, 0.4, -0.7], dtype=torch.float64)).item())
    assert v == float("inf")
    assert m.sync() == -3

"""GPU tests of composed models outside the ahead-of-time registry: the
kernel templates compiled at model creation for the lowered shape (hipRTC),
against the scalar FP64 oracle at seeded parameter points.  NLL within
1e-12 relative, gradient within 1e-8 of the oracle's max-norm.

Shapes: a three-component sum, Crystal Ball + exponential, Gauss(x) x
Chebyshev-3(y), a sum of products, a product of two sums (terms that are
not one leaf each), a sum over eight children, Chebyshev series of orders
1, 3, 5, 6, 7, 8; and on some of them the batched pass, gradient-descent
fit steps, the FP32-compensated pass, BHHH and weighted events."""
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


P = datagen.param


def three_sum():
    """0.3 G(2, 0.5) + 0.2 G(6, 0.8) + 0.5 Exp(-0.3) on [0, 10]."""
    return {"obs": [{"name": "x", "lo": 0.0, "hi": 10.0}],
            "params": [P("f1", 0.3, 0.0, 1.0), P("f2", 0.2, 0.0, 1.0), P("mu1", 2.0, 0.0, 10.0),
                       P("s1", 0.5, 0.01, 5.0), P("mu2", 6.0, 0.0, 10.0), P("s2", 0.8, 0.01, 5.0),
                       P("c", -0.3, -5.0, 5.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [2, 3]}, {"kind": "gauss", "obs": 0, "params": [4, 5]},
                      {"kind": "exp", "obs": 0, "params": [6]},
                      {"kind": "sum", "params": [0, 1], "children": [0, 1, 2]}],
            "root": 3}


def cb_exp(norm="analytic"):
    """0.3 CB(5.28, 0.003, 1.5, 3) + 0.7 Exp(-2) on [5.20, 5.30]."""
    return {"obs": [{"name": "m", "lo": 5.20, "hi": 5.30}],
            "params": [P("f", 0.3, 0.0, 1.0), P("m0", 5.28, 5.2, 5.3, jitter=3e-4),
                       P("sigma", 0.003, 1e-4, 0.05, jitter=3e-4), P("alpha", 1.5, 0.1, 10.0),
                       P("n", 3.0, 1.05, 50.0), P("c", -2.0, -50.0, 50.0)],
            "nodes": [{"kind": "cb", "obs": 0, "params": [1, 2, 3, 4], "norm": norm},
                      {"kind": "exp", "obs": 0, "params": [5], "norm": norm},
                      {"kind": "sum", "params": [0], "children": [0, 1]}],
            "root": 2}


def gauss_cheb3():
    """G(x; 0.5, 1.2) on [-5, 5] x Cheb_3(y) on [-1, 1]."""
    return {"obs": [{"name": "x", "lo": -5.0, "hi": 5.0}, {"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": [P("mu", 0.5, -5.0, 5.0), P("s", 1.2, 0.05, 5.0), P("a1", 0.2, -1.0, 1.0),
                       P("a2", -0.15, -1.0, 1.0), P("a3", 0.1, -1.0, 1.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [0, 1]}, {"kind": "cheb", "obs": 1, "params": [2, 3, 4]},
                      {"kind": "prod", "children": [0, 1]}],
            "root": 2}


def sum_of_products():
    """0.4 G(x; 1, 0.7) G(y; -0.5, 0.4) + 0.6 Exp(x; -0.4) Cheb_2(y) on
    [0, 6] x [-1, 1]: two terms of two non-root leaves each."""
    return {"obs": [{"name": "x", "lo": 0.0, "hi": 6.0}, {"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": [P("f", 0.4, 0.0, 1.0), P("mx", 1.0, 0.0, 6.0), P("sx", 0.7, 0.05, 5.0),
                       P("my", -0.5, -1.0, 1.0), P("sy", 0.4, 0.05, 5.0), P("c", -0.4, -5.0, 5.0),
                       P("a1", 0.3, -1.0, 1.0), P("a2", 0.2, -1.0, 1.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [1, 2]}, {"kind": "gauss", "obs": 1, "params": [3, 4]},
                      {"kind": "prod", "children": [0, 1]},
                      {"kind": "exp", "obs": 0, "params": [5]}, {"kind": "cheb", "obs": 1, "params": [6, 7]},
                      {"kind": "prod", "children": [3, 4]},
                      {"kind": "sum", "params": [0], "children": [2, 5]}],
            "root": 6}


def product_of_sums():
    """[0.3 G(x; 2, 0.5) + 0.7 Exp(x; -0.5)] x [0.6 G(y; 0, 0.3) + 0.4
    Cheb_2(y)] on [0, 8] x [-1, 1]: four terms of two non-root leaves each,
    as many non-root leaves as terms."""
    return {"obs": [{"name": "x", "lo": 0.0, "hi": 8.0}, {"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": [P("f", 0.3, 0.0, 1.0), P("mx", 2.0, 0.0, 8.0), P("sx", 0.5, 0.05, 5.0), P("c", -0.5, -5.0, 5.0),
                       P("g", 0.6, 0.0, 1.0), P("my", 0.0, -1.0, 1.0, jitter=0.05), P("sy", 0.3, 0.05, 5.0),
                       P("a1", 0.2, -1.0, 1.0), P("a2", -0.1, -1.0, 1.0)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [1, 2]}, {"kind": "exp", "obs": 0, "params": [3]},
                      {"kind": "sum", "params": [0], "children": [0, 1]},
                      {"kind": "gauss", "obs": 1, "params": [5, 6]}, {"kind": "cheb", "obs": 1, "params": [7, 8]},
                      {"kind": "sum", "params": [4], "children": [3, 4]},
                      {"kind": "prod", "children": [2, 5]}],
            "root": 6}


def eight_gauss():
    """Eight Gaussians at 1..8 (width 0.3 + 0.05 k) with fractions 0.1 each
    (the last takes 0.3) on [0, 9]."""
    ps = [P(f"f{k}", 0.1, 0.0, 1.0) for k in range(7)]
    nodes = []
    for k in range(8):
        ps += [P(f"mu{k}", 1.0 + k, 0.0, 9.0), P(f"s{k}", 0.3 + 0.05 * k, 0.02, 5.0)]
        nodes.append({"kind": "gauss", "obs": 0, "params": [7 + 2 * k, 8 + 2 * k]})
    nodes.append({"kind": "sum", "params": list(range(7)), "children": list(range(8))})
    return {"obs": [{"name": "x", "lo": 0.0, "hi": 9.0}], "params": ps, "nodes": nodes, "root": 8}


def cheb(order):
    coef = [0.25 * (-0.6) ** k for k in range(order)]
    return {"obs": [{"name": "y", "lo": -1.0, "hi": 1.0}],
            "params": [P(f"a{k + 1}", c, -1.0, 1.0) for k, c in enumerate(coef)],
            "nodes": [{"kind": "cheb", "obs": 0, "params": list(range(order))}], "root": 0}


def build(torch, nllmi, spec, n, seed, precision="fp64"):
    cols = datagen.generate(spec, n, seed=seed)
    m = nllmi.Model.from_spec(spec, precision=precision)
    m.set_data([torch.from_numpy(c).cuda() for c in cols])
    return m, cols


def check_points(torch, m, spec, cols, points, threads, nll_tol=NLL_TOL, grad_tol=GRAD_TOL):
    o = oracle.Oracle(spec)
    for th in points:
        st, ref, gref = o.nll(cols, th, threads=threads)
        assert st == 0
        v, g = m.eval_grad(torch.from_numpy(np.ascontiguousarray(th)))
        v, g = float(v.item()), g.cpu().numpy()
        assert abs(v / ref - 1.0) <= nll_tol, (th, v, ref)
        assert np.max(np.abs(g - gref)) <= grad_tol * np.max(np.abs(gref)), (th, g, gref)
        v1 = float(m.eval(torch.from_numpy(np.ascontiguousarray(th))).item())
        assert abs(v1 / ref - 1.0) <= nll_tol, (th, v1, ref)
    assert m.sync() == 0


CASES = {"three_sum": (three_sum, 300_000), "cb_exp": (cb_exp, 300_000), "gauss_cheb3": (gauss_cheb3, 300_000),
         "sum_of_products": (sum_of_products, 300_000), "product_of_sums": (product_of_sums, 300_000),
         "eight_gauss": (eight_gauss, 400_000)}


@pytest.mark.parametrize("name", sorted(CASES))
def test_composed_shape_against_oracle(torch, nllmi, threads, name):
    make, n = CASES[name]
    spec = make()
    print(f"[composition {name}: {n} events]", flush=True)
    m, cols = build(torch, nllmi, spec, n, seed=901)
    assert m.info["variant"].startswith("rtc:"), m.info["variant"]
    pts = datagen.parameter_points(spec, 4, seed=902)
    check_points(torch, m, spec, cols, pts, threads)


@pytest.mark.parametrize("order", [1, 3, 5, 6, 7, 8])
def test_chebyshev_orders(torch, nllmi, threads, order):
    spec = cheb(order)
    print(f"[chebyshev order {order}]", flush=True)
    m, cols = build(torch, nllmi, spec, 200_001, seed=910 + order)
    assert m.info["variant"].startswith("rtc:")
    pts = datagen.parameter_points(spec, 3, seed=920 + order)
    check_points(torch, m, spec, cols, pts, threads)


def test_gl_normalisation_composed(torch, nllmi, threads):
    """Crystal Ball + exponential with Gauss-Legendre panels instead of the
    closed forms."""
    spec = cb_exp(norm="gl256")
    m, cols = build(torch, nllmi, spec, 200_000, seed=930)
    check_points(torch, m, spec, cols, datagen.parameter_points(spec, 3, seed=931), threads)


def test_three_sum_batched_and_fit(torch, nllmi, threads):
    """The run-time compiled batched pass (sets of uneven sizes, one empty)
    and gradient-descent fit steps against the oracle's trajectory."""
    spec = three_sum()
    m, cols = build(torch, nllmi, spec, 120_000, seed=940)
    o = oracle.Oracle(spec)
    offsets = np.array([0, 1, 777, 777, 40_000, 120_000], dtype=np.int64)
    pts = datagen.parameter_points(spec, 5, seed=941)
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
    for steps in (1, 4, 9):
        th, f, gg, stt = m.fit(torch.from_numpy(pts[0]), steps)
        sto, th_o, f_o, g_o, _ = o.gd_fit(cols, pts[0], steps, 1.0, threads=threads)
        assert int(stt.item()) == sto == 0
        assert abs(float(f.item()) / f_o - 1.0) <= NLL_TOL, (steps, float(f.item()), f_o)
        np.testing.assert_allclose(th.cpu().numpy(), th_o, rtol=1e-10, atol=1e-12)


def test_three_sum_fp32c(torch, nllmi, threads):
    """The FP32-compensated pass of a run-time compiled shape, at the bounds
    the FP32C tests derive for small N: NLL within max(1e-9, 1e-6/sqrt(N))
    relative, gradient within max(1e-8, 1e-5/sqrt(N)) of the larger of the
    oracle's max-norm and the sums of |d log p_i / d theta|."""
    spec = three_sum()
    n = 300_000
    m, cols = build(torch, nllmi, spec, n, seed=950, precision="fp32c")
    assert m.info["variant"].startswith("rtc:") and "FP32C" in m.info["variant"]
    o = oracle.Oracle(spec)
    ntol = max(1e-9, 1e-6 / np.sqrt(n))
    gtol = max(1e-8, 1e-5 / np.sqrt(n))
    for th in datagen.parameter_points(spec, 3, seed=951):
        st, ref, gref, stats = o.nll(cols, th, threads=threads, stats=True)
        v, g = m.eval_grad(torch.from_numpy(th))
        assert abs(float(v.item()) / ref - 1.0) <= ntol
        scale = max(np.max(np.abs(gref)), np.max(stats[1:]))
        assert np.max(np.abs(g.cpu().numpy() - gref)) <= gtol * scale
    assert m.sync() == 0


def test_gauss_cheb3_bhhh(torch, nllmi, threads):
    """BHHH matrix of a run-time compiled shape (5 score features) against
    the oracle's sum of per-event score outer products."""
    spec = gauss_cheb3()
    m, cols = build(torch, nllmi, spec, 150_000, seed=960)
    o = oracle.Oracle(spec)
    th = datagen.parameter_points(spec, 1, seed=961)[0]
    st, ref, gref, B = o.nll_bhhh(cols, th, threads=threads)
    v, g, Bd = m.eval_bhhh(torch.from_numpy(th))
    assert abs(float(v.item()) / ref - 1.0) <= NLL_TOL
    assert np.max(np.abs(g.cpu().numpy() - gref)) <= GRAD_TOL * np.max(np.abs(gref))
    assert np.max(np.abs(Bd.cpu().numpy() - B)) <= 1e-10 * np.max(np.abs(B))


def test_cb_exp_weighted(torch, nllmi, threads):
    """Weighted events on a run-time compiled shape: -sum w_i log p(x_i)
    and its gradient against the oracle."""
    spec = cb_exp()
    m, cols = build(torch, nllmi, spec, 150_000, seed=970)
    w = 0.5 + np.random.default_rng(971).uniform(0.0, 1.0, 150_000)
    m.set_weights(torch.from_numpy(w).cuda())
    o = oracle.Oracle(spec)
    for th in datagen.parameter_points(spec, 2, seed=972):
        st, ref, gref = o.nll(cols, th, threads=threads, weights=w)
        v, g = m.eval_grad(torch.from_numpy(th))
        assert abs(float(v.item()) / ref - 1.0) <= NLL_TOL
        assert np.max(np.abs(g.cpu().numpy() - gref)) <= GRAD_TOL * np.max(np.abs(gref))
    assert m.sync() == 0

"""GPU parity of the BHHH pass (nll_eval_bhhh: NLL, gradient and the
outer-product matrix B = sum_i s_i s_i^T of the events' scores) and of the
damped BHHH minimiser (nll_fit_bhhh) against the oracle.

Tolerances: NLL 1e-12 relative and gradient 1e-8 of ||g_oracle||_inf as for
the FP64 pass (gradients after a fit, where g -> 0, on the scale G =
max_k sum_i |d l_i / d theta_k|); B entry-wise 1e-10 of max|B| (its entries are sums of
non-negative-definite terms of the size of that maximum, and the kernel
forms them from reduced second moments instead of per-event products);
fitted points 1e-9 relative, as for gradient descent.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

NLL_TOL = 1e-12
GRAD_TOL = 1e-8
B_TOL = 1e-10


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


def product_spec():
    """Gauss(x) * Gauss(y): one term, two root leaves on two observables."""
    return {"obs": [{"name": "x", "lo": -8.0, "hi": 8.0}, {"name": "y", "lo": -5.0, "hi": 9.0}],
            "params": [datagen.param("mx", 0.5, -3, 3), datagen.param("sx", 1.2, 0.1, 5),
                       datagen.param("my", 2.0, -3, 6), datagen.param("sy", 0.8, 0.1, 5)],
            "nodes": [{"kind": "gauss", "obs": 0, "params": [0, 1]},
                      {"kind": "gauss", "obs": 1, "params": [2, 3]},
                      {"kind": "prod", "children": [0, 1]}],
            "root": 2}


def check_bhhh(torch, nllmi, spec, cols, points, threads, unroll=None):
    m = nllmi.Model.from_spec(spec)
    m.set_data(to_dev(torch, cols))
    if unroll:
        m.set_schedule(unroll=unroll)
    o = oracle.Oracle(spec)
    for th in points:
        st, ref, gref, Bref = o.nll_bhhh(cols, th, threads=threads)
        _, _, _, stats = o.nll(cols, th, threads=threads, stats=True)
        assert st == 0
        v, g, B = m.eval_bhhh(torch.from_numpy(np.ascontiguousarray(th)))
        v, g, B = float(v.item()), g.cpu().numpy(), B.cpu().numpy()
        assert abs(v - ref) <= NLL_TOL * abs(ref), (th, v, ref)
        assert np.max(np.abs(g - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (g, gref)
        assert np.array_equal(B, B.T)
        assert np.max(np.abs(B - Bref)) <= B_TOL * np.max(np.abs(Bref)), (th, B, Bref)
    assert m.sync() == 0
    return m


@pytest.mark.parametrize("case", ["gauss", "mixture", "extended", "product"])
def test_eval_bhhh_matches_oracle(torch, nllmi, threads, case):
    if case == "gauss":
        w = datagen.workload(1)
        spec, cols, pts = w["spec"], w["cols"], w["points"][:3]
    elif case == "mixture":
        w = datagen.workload(2, n=200_001)
        spec, cols, pts = w["spec"], w["cols"], w["points"][:3]
    elif case == "extended":
        w = datagen.workload(2, n=150_000)
        spec, cols = extended_spec(), w["cols"]
        pts = [np.append(p, nu) for p, nu in zip(w["points"][:3], (1.2e5, 1.5e5, 2e5))]
    else:
        spec = product_spec()
        cols = datagen.generate(spec, 99_999, seed=77)
        pts = datagen.jittered_points(datagen.theta_of(spec), 3, seed=78, rel=0.05)
    print(f"[bhhh {case}]", flush=True)
    check_bhhh(torch, nllmi, spec, cols, pts, threads)


def test_eval_bhhh_every_unroll_and_fixed_parameter(torch, nllmi, threads):
    spec = datagen.mixture_spec()
    spec["params"][3]["free"] = False
    w = datagen.workload(2, n=4097 * 3 + 11)
    for u in (2, 4, 8):
        check_bhhh(torch, nllmi, spec, w["cols"], w["points"][1:2], threads, unroll=u)


def test_bhhh_unsupported_shapes(torch, nllmi):
    w = datagen.workload(3, n=1000)
    m = nllmi.Model.from_spec(w["spec"])  # 12 score features: not compiled
    m.set_data(to_dev(torch, w["cols"]))
    with pytest.raises(nllmi.NLLError):
        m.eval_bhhh(torch.from_numpy(w["points"][0]))
    with pytest.raises(nllmi.NLLError):
        m.fit_bhhh(torch.from_numpy(w["points"][0]), 3)
    w = datagen.workload(2, n=1000)
    m = nllmi.Model.from_spec(w["spec"], precision="fp32c")
    m.set_data(to_dev(torch, w["cols"]))
    with pytest.raises(nllmi.NLLError):
        m.eval_bhhh(torch.from_numpy(w["points"][0]))


def test_fit_bhhh_gauss_matches_oracle_and_mle(torch, nllmi, threads):
    w = datagen.workload(1)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    th0 = w["points"][0]
    th, nll, g, status = m.fit_bhhh(torch.from_numpy(th0), 12, 1e-3)
    th = th.cpu().numpy()
    st, th_o, nll_o, g_o, lam_o = oracle.Oracle(w["spec"]).bhhh_fit(w["cols"], th0, 12, 1e-3, threads=threads)
    assert status.item() == 0 and st == 0
    np.testing.assert_allclose(th, th_o, rtol=1e-9)
    assert abs(nll.item() - nll_o) <= NLL_TOL * abs(nll_o)
    x = w["cols"][0].astype(np.longdouble)
    assert abs(th[0] - float(x.mean())) <= 1e-8 * abs(float(x.mean()))
    assert abs(th[1] - float(np.sqrt(((x - x.mean()) ** 2).mean()))) <= 1e-8 * th[1]


def test_fit_bhhh_mixture_matches_oracle(torch, nllmi, threads):
    """20 damped BHHH steps on the mixture: same accepted point as the
    oracle's run, a stationary point, and graph replay gives the same bits."""
    w = datagen.workload(2, n=300_000)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    th0 = w["points"][0]
    out = m.fit_bhhh(torch.from_numpy(th0), 20, 1e-3)
    th = out[0].cpu().numpy().copy()
    st, th_o, nll_o, g_o, lam_o = oracle.Oracle(w["spec"]).bhhh_fit(w["cols"], th0, 20, 1e-3, threads=threads)
    assert out[3].item() == 0 and st == 0
    np.testing.assert_allclose(th, th_o, rtol=1e-9)
    assert abs(out[1].item() - nll_o) <= NLL_TOL * abs(nll_o)
    _, _, _, stats = oracle.Oracle(w["spec"]).nll(w["cols"], th_o, threads=threads, stats=True)
    assert np.max(np.abs(out[2].cpu().numpy()) / stats[1:]) < 1e-8
    out2 = m.fit_bhhh(torch.from_numpy(th0), 20, 1e-3, out=out)
    assert np.array_equal(out2[0].cpu().numpy(), th)

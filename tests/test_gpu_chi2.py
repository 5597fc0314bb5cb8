"""GPU parity of the chi-square leaf (the ChiSquarePdf model of Sec. 5.2's
speed-up figure) against the oracle: closed-form normalisation by the lower
incomplete gamma series and Gauss-Legendre after x = s^2, ragged sizes up
to the benchmarked 1e7 events, every unroll, invalid events and parameters,
gradient descent, BHHH, many datasets and the FP32-compensated pass.

Tolerances as for the other leaves: NLL 1e-12 relative, gradient 1e-8 of
||g_oracle||_inf at seeded points (after a fit, where g -> 0, of G, the
largest per-parameter sum of |d l_i/d theta|); fitted points 1e-9
relative.
"""
import math

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


def check(torch, nllmi, spec, cols, points, threads, unroll=None):
    m = nllmi.Model.from_spec(spec)
    assert m.info["variant"] == "chi2", m.info
    m.set_data(to_dev(torch, cols))
    if unroll:
        m.set_schedule(unroll=unroll)
    o = oracle.Oracle(spec)
    for th in points:
        st, ref, gref, stats = o.nll(cols, th, threads=threads, stats=True)
        assert st == 0
        v, g = m.eval_grad(torch.from_numpy(np.ascontiguousarray(th)))
        v, g = float(v.item()), g.cpu().numpy()
        assert abs(v - ref) <= NLL_TOL * abs(ref), (th, v, ref)
        assert np.max(np.abs(g - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (th, g, gref)
        v1 = float(m.eval(torch.from_numpy(np.ascontiguousarray(th))).item())
        assert abs(v1 - ref) <= NLL_TOL * abs(ref), (th, v1, ref)
    assert m.sync() == 0
    return m


@pytest.mark.parametrize("norm", ["analytic", "gl256"])
@pytest.mark.parametrize("n", [1, 257, 100_003])
def test_chi2_small(torch, nllmi, threads, norm, n):
    w = datagen.chi2_workload(n, n_points=3, norm=norm)
    print(f"[chi2 {norm} n={n}]", flush=True)
    check(torch, nllmi, w["spec"], w["cols"], w["points"], threads)


def test_chi2_full(torch, nllmi, threads):
    """The benchmarked size: 1e7 events."""
    w = datagen.chi2_workload(n_points=2)
    print("[chi2 n=1e7]", flush=True)
    check(torch, nllmi, w["spec"], w["cols"], w["points"], threads)


@pytest.mark.parametrize("unroll", [2, 4, 8])
def test_chi2_every_unroll(torch, nllmi, threads, unroll):
    w = datagen.chi2_workload(4097 * 5 + 13, n_points=2)
    check(torch, nllmi, w["spec"], w["cols"], w["points"], threads, unroll=unroll)


@pytest.mark.parametrize("nu", [0.8, 2.0, 3.0, 47.5, 150.0])
def test_chi2_shapes_and_wide_range(torch, nllmi, threads, nu):
    """Few to many degrees of freedom (a density that is infinite, finite or
    zero at 0) on [0, 1000], the widest range supported, with events at
    the range's top and, for few degrees of freedom, at tiny x (for many,
    p there underflows the oracle's linear-domain double)."""
    spec = datagen.chi2_spec(nu=nu, lo=0.0, hi=1000.0)
    x = datagen.generate(spec, 30_000, seed=41)[0]
    x[:3] = [1e-300, 1000.0, 1e-9] if nu <= 3 else [1.0, 1000.0, 999.0]
    pts = [np.array([nu]), np.array([nu * 1.03])]
    check(torch, nllmi, spec, [x], pts, threads)


def test_chi2_invalid_event_and_parameter(torch, nllmi):
    """An event at x = 0 with nu > 2 has density 0: the value is +inf and the
    status reads NLL_ERR_INVALID_PDF; nu <= 0 is flagged as a parameter
    outside the density's domain (Sec. 3)."""
    spec = datagen.chi2_spec()
    spec["params"][0]["lo"] = -1.0
    x = datagen.generate(spec, 1000, seed=43)[0]
    m = nllmi.Model.from_spec(spec)
    m.set_data(to_dev(torch, [x]))
    for v in (0.0, -0.5):
        val = m.eval(torch.tensor([v], dtype=torch.float64))
        assert math.isinf(val.item()) and m.sync() == -3
    x[7] = 0.0
    m.set_data(to_dev(torch, [x]))
    val = m.eval(torch.tensor([5.0], dtype=torch.float64))
    assert math.isinf(val.item()) and m.sync() == -5
    assert oracle.Oracle(spec).nll([x], np.array([5.0]))[0] == oracle.E_PDF
    bad = datagen.chi2_spec(lo=0.0, hi=1500.0)
    with pytest.raises(nllmi.NLLError) as e:
        nllmi.Model.from_spec(bad)
    assert e.value.status == -2


def test_chi2_fits(torch, nllmi, threads):
    w = datagen.chi2_workload(300_000, n_points=1)
    m = nllmi.Model.from_spec(w["spec"])
    m.set_data(to_dev(torch, w["cols"]))
    th0 = w["points"][0]
    o = oracle.Oracle(w["spec"])
    th, nll, g, status = m.fit(torch.from_numpy(th0), 30, 1.0)
    st, th_o, nll_o, g_o, eta_o = o.gd_fit(w["cols"], th0, 30, 1.0, threads=threads)
    assert status.item() == 0 and st == 0
    np.testing.assert_allclose(th.cpu().numpy(), th_o, rtol=1e-9)
    assert abs(nll.item() - nll_o) <= NLL_TOL * abs(nll_o)
    st, ref, gref, Bref = o.nll_bhhh(w["cols"], th0, threads=threads)
    v, gb, B = m.eval_bhhh(torch.from_numpy(th0))
    assert abs(v.item() - ref) <= NLL_TOL * abs(ref)
    assert abs(B.item() - Bref[0, 0]) <= 1e-10 * abs(Bref[0, 0])
    out = m.fit_bhhh(torch.from_numpy(th0), 10, 1e-3)
    st, th_b, nll_b, g_b, lam_b = o.bhhh_fit(w["cols"], th0, 10, 1e-3, threads=threads)
    assert out[3].item() == 0 and st == 0
    np.testing.assert_allclose(out[0].cpu().numpy(), th_b, rtol=1e-9)
    _, _, _, stats = o.nll(w["cols"], th_b, threads=threads, stats=True)
    assert abs(out[2].item()) / stats[1] < 1e-8


def test_chi2_many_datasets(torch, nllmi, threads):
    spec = datagen.chi2_spec()
    sizes = datagen.toy_sizes(40, datagen.CHI2_SEED, 0, 9000)
    offsets = np.zeros(41, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    truths = datagen.jittered_points(datagen.theta_of(spec), 40, datagen.CHI2_SEED + 2)
    cols = datagen.generate_sets(spec, truths, offsets, datagen.CHI2_SEED, 5 << 32, threads=threads)
    o = oracle.Oracle(spec)
    st, ref, gref, _ = o.nll_batched(cols, offsets, truths, threads=threads)
    m = nllmi.Model.from_spec(spec)
    m.set_data(to_dev(torch, cols))
    m.set_schedule(tile_events=2048)
    nll, g, status = m.eval_batched(torch.from_numpy(offsets), torch.from_numpy(truths))
    nll, g = nll.cpu().numpy(), g.cpu().numpy()
    assert np.all(status.cpu().numpy() == 0)
    for s in range(40):
        assert abs(nll[s] - ref[s]) <= NLL_TOL * max(1.0, abs(ref[s])), (s, nll[s], ref[s])
        a, b = offsets[s], offsets[s + 1]
        assert np.max(np.abs(g[s] - gref[s])) <= GRAD_TOL * np.max(np.abs(gref[s])), (s, g[s], gref[s])


def test_chi2_fp32c(torch, nllmi, threads):
    from test_gpu_fp32c import compare
    w = datagen.chi2_workload(300_001, n_points=2)
    print("[chi2 fp32c]", flush=True)
    compare(torch, nllmi, w["spec"], w["cols"], w["points"], threads, against_fp64=True, report=True)

"""GPU parity of the just-in-time densities (Sec. 4) against the expression
oracle (numpy, adaptive quadrature, complex-step derivatives) and, for a
Gaussian written as an expression, against the built-in Gaussian kernels.

Tolerances: NLL 1e-12 relative; gradient 1e-8 of ||g_oracle||_inf at the
seeded points."""
import math

import numpy as np
import pytest

import datagen
from oracle import jit

pytestmark = pytest.mark.gpu

NLL_TOL = 1e-12
GRAD_TOL = 1e-8
GAUSS = "exp(-0.5*((x-p[0])/p[1])*((x-p[0])/p[1]))"
POLYEXP = "(1.0 + p[0]*x*x) * exp(-x/p[1]) + p[2]"
MIXED = "pow(x, p[0]) * exp(-p[1]*x) + sqrt(p[2]) * atan(x) + erf(x - p[3]) + 2.0"


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


def params(values, lo, hi):
    return [datagen.param(f"p{k}", v, a, b) for k, (v, a, b) in enumerate(zip(values, lo, hi))]


def check(torch, nllmi, expr, lo, hi, ps, x, points):
    m = nllmi.JITModel(expr, lo, hi, ps)
    m.set_data(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    plo, phi = [p["lo"] for p in ps], [p["hi"] for p in ps]
    for th in points:
        th = np.asarray(th, dtype=np.float64)
        st, ref, gref = jit.nll(expr, lo, hi, plo, phi, x, th)
        assert st == jit.OK
        v, d = jit.g_and_grad(expr, x, th)
        Z, dZ = jit.norm(expr, lo, hi, th)
        val, g = m.eval_grad(torch.from_numpy(th))
        val, g = float(val.item()), g.cpu().numpy()
        assert abs(val - ref) <= NLL_TOL * abs(ref), (th, val, ref)
        assert np.max(np.abs(g - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (th, g, gref)
        v1 = float(m.eval(torch.from_numpy(th)).item())
        assert abs(v1 - ref) <= NLL_TOL * abs(ref)
    assert m.sync() == 0
    return m


def test_gauss_expression_matches_builtin_kernels(torch, nllmi):
    w = datagen.workload(1)
    x = w["cols"][0]
    print("[jit gauss]", flush=True)
    m = check(torch, nllmi, GAUSS, -10.0, 10.0, params([0.3, 1.5], [-10, 0.05], [10, 10]), x, w["points"][:3])
    b = nllmi.Model.from_spec(w["spec"])
    b.set_data([torch.from_numpy(x).cuda()])
    for th in w["points"][:3]:
        v1, g1 = m.eval_grad(torch.from_numpy(th))
        v2, g2 = b.eval_grad(torch.from_numpy(th))
        assert abs(v1.item() - v2.item()) <= NLL_TOL * abs(v2.item())
        np.testing.assert_allclose(g1.cpu().numpy(), g2.cpu().numpy(), rtol=1e-9, atol=1e-9 * np.abs(g2.cpu().numpy()).max())


def exp_events(n, lo, hi, c, seed):
    spec = {"obs": [{"name": "x", "lo": lo, "hi": hi}], "params": [datagen.param("c", c, -5, 5)],
            "nodes": [{"kind": "exp", "obs": 0, "params": [0]}], "root": 0}
    return datagen.generate(spec, n, seed=seed)[0]


@pytest.mark.parametrize("n", [1, 257, 100_003])
def test_polyexp_expression(torch, nllmi, n):
    x = exp_events(n, 0.0, 8.0, -0.5, seed=n)
    pts = [[0.3, 2.0, 0.05], [0.1, 1.5, 0.2], [0.6, 3.0, 0.01]]
    print(f"[jit polyexp n={n}]", flush=True)
    check(torch, nllmi, POLYEXP, 0.0, 8.0, params(pts[0], [0, 0.1, 0], [5, 10, 1]), x, pts)


def test_mixed_functions_expression(torch, nllmi):
    x = exp_events(50_000, 0.1, 5.0, -0.3, seed=5)
    pts = [[1.5, 0.8, 0.4, 1.0], [2.2, 1.1, 0.9, 2.5]]
    print("[jit mixed]", flush=True)
    check(torch, nllmi, MIXED, 0.1, 5.0, params(pts[0], [0.5, 0.1, 0.01, -5], [5, 5, 5, 5]), x, pts)


def test_compile_errors_limits_and_status(torch, nllmi):
    with pytest.raises(nllmi.NLLError) as e:
        nllmi.JITModel("1.0 + p[0] * x +", 0.0, 1.0, params([0.5], [0], [1]))
    assert e.value.status == -1 and "error" in str(e.value)
    with pytest.raises(nllmi.NLLError) as e:
        nllmi.JITModel("x", 0.0, 1.0, params([0.1] * 9, [0] * 9, [1] * 9))
    assert e.value.status == -2
    m = nllmi.JITModel("x - p[0]", 0.0, 2.0, params([0.1], [-5], [5]))
    m.set_data(torch.tensor([0.5, 1.0, 1.5], dtype=torch.float64).cuda())
    assert math.isinf(m.eval(torch.tensor([0.7], dtype=torch.float64)).item()) and m.sync() == -5
    assert math.isinf(m.eval(torch.tensor([7.0], dtype=torch.float64)).item()) and m.sync() == -3
    assert math.isfinite(m.eval(torch.tensor([0.1], dtype=torch.float64)).item()) and m.sync() == 0
    with pytest.raises(nllmi.NLLError) as e:
        m.set_data(torch.tensor([0.5, 2.5], dtype=torch.float64).cuda())
    assert e.value.status == -4


@pytest.mark.parametrize("sigma", [0.05, 0.02, 0.005])
def test_narrow_peak_expression(torch, nllmi, threads, sigma):
    """A Gaussian expression whose width is 1/200 to 1/2000 of the range:
    one 256-node Gauss-Legendre panel misses most of it (Z off by 24 % at
    sigma = 0.02), so the finishing block refines the panels until two
    levels agree.  Against the scalar oracle's built-in Gaussian (closed-
    form normalisation through erf)."""
    import oracle
    spec = datagen.gauss_spec(5.0, sigma, 0.0, 10.0)
    spec["params"][1]["lo"] = 1e-4  # the oracle's range check: widths below the spec's default floor
    x = datagen.generate(spec, 40_000, seed=321)[0]
    o = oracle.Oracle(spec)
    m = nllmi.JITModel(GAUSS, 0.0, 10.0, params([5.0, sigma], [0.0, 1e-4], [10.0, 5.0]))
    m.set_data(torch.from_numpy(x).cuda())
    print(f"[jit narrow peak sigma={sigma}]", flush=True)
    for th in ([5.0, sigma], [5.0 + 0.3 * sigma, 1.1 * sigma], [5.0 - 0.2 * sigma, 0.93 * sigma]):
        th = np.asarray(th)
        st, ref, gref = o.nll([x], th, threads=threads)
        assert st == 0
        v, g = m.eval_grad(torch.from_numpy(th))
        v, g = float(v.item()), g.cpu().numpy()
        assert abs(v - ref) <= NLL_TOL * abs(ref), (th, v, ref)
        assert np.max(np.abs(g - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (th, g, gref)
    assert m.sync() == 0


def test_subnormal_density_values(torch, nllmi):
    """Events where g is subnormal (down to 1e-320): the running product
    takes each g's own mantissa and exponent, so log g keeps full
    precision, and the features g'_k / g take the reciprocal of g 2^64
    where that of g would overflow.  g = (p0 x) e^(-p1 x) and its derivatives x e^(-p1 x)
    and -x g are formed by the same correctly rounded operations on both
    sides (e^(-p1 x) is exactly 1 at the subnormal events), so the
    reference takes them written out in numpy (the complex step of the
    expression oracle underflows there); Z and dZ/dp by the expression
    oracle's quadrature."""
    expr = "p[0] * x * exp(-p[1] * x)"
    x = np.array([1e-320, 3.3e-318, 2.5e-315, 7e-310, 1e-305, 0.25, 0.5, 0.9, 3.0])
    ps = params([1.0, 0.5], [0.5, 0.0], [2.0, 2.0])
    m = nllmi.JITModel(expr, 0.0, 4.0, ps)
    m.set_data(torch.from_numpy(x).cuda())
    for th in ([1.0, 0.5], [0.999, 0.7], [1.3, 0.2]):
        p0, p1 = th
        e = np.exp(-p1 * x)
        gv = (p0 * x) * e
        d0, d1 = x * e, (p0 * x) * (-x * e)
        Z, dZ = jit.norm(expr, 0.0, 4.0, np.asarray(th))
        n = len(x)
        ref = -math.fsum(np.log(gv)) + n * math.log(Z)
        gref = np.array([-math.fsum(d0 / gv) + n * dZ[0] / Z, -math.fsum(d1 / gv) + n * dZ[1] / Z])
        v, g = m.eval_grad(torch.from_numpy(np.asarray(th)))
        assert abs(v.item() - ref) <= NLL_TOL * abs(ref), (th, v.item(), ref)
        assert np.max(np.abs(g.cpu().numpy() - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (th, g, gref)
        assert abs(m.eval(torch.from_numpy(np.asarray(th))).item() - ref) <= NLL_TOL * abs(ref)
    assert m.sync() == 0


MANY = {
    1: ("exp(-p[0]*x)", 0.0, 8.0, [0.6], [0.01], [5.0]),
    5: ("p[0] + p[1]*x + p[2]*x*x + p[3]*exp(-p[4]*x)", 0.0, 2.0,
        [1.0, 0.3, 0.2, 0.5, 1.0], [0.1, -1, -1, 0, 0], [5, 5, 5, 5, 5]),
    8: ("p[0] + p[1]*x + p[2]*x*x + p[3]*exp(-p[4]*x) + p[5]/(1.0 + p[6]*x*x) + p[7]*sin(x)", 0.0, 2.0,
        [1.0, 0.3, 0.2, 0.5, 1.0, 0.4, 0.7, 0.1], [0.1, -1, -1, 0, 0, 0, 0, -1], [5] * 8),
}


@pytest.mark.parametrize("np_", [1, 5, 8])
def test_parameter_counts_and_full_trips(torch, nllmi, np_):
    """One, five and eight parameters (five and more take the finishing
    block's three separate reductions; every count a different width of the
    halving block reduction), on 2.2-3e6 events, so that every thread of the
    streaming pass runs full trips of 8 events with the next trip's loads in
    flight and then a ragged last trip."""
    expr, lo, hi, p0, plo, phi = MANY[np_]
    n = 3_000_017 if np_ < 8 else 2_200_001
    x = exp_events(n, lo, hi, -0.3, seed=40 + np_)
    pts = [p0, [v * (1.0 + 0.05 * ((k % 3) - 1)) for k, v in enumerate(p0)]]
    print(f"[jit {np_} parameters, {n} events]", flush=True)
    check(torch, nllmi, expr, lo, hi, params(p0, plo, phi), x, pts)

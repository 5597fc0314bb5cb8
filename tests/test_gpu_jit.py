"""GPU parity of the just-in-time densities (Sec. 4) against the expression
oracle (numpy, adaptive quadrature, complex-step derivatives) and, for a
Gaussian written as an expression, against the built-in Gaussian kernels.

Tolerances: NLL 1e-12 relative; gradient 1e-8 of max(|g|, G) with G the
largest per-parameter sum of |d l_i / d theta| (l_i = log g(x_i) - log Z).
The device normalises by 256-point Gauss-Legendre on one panel, which is
exact to rounding for the smooth densities used here."""
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
        G = max(float(np.sum(np.abs(dk / v - dz / Z))) for dk, dz in zip(d, dZ))
        val, g = m.eval_grad(torch.from_numpy(th))
        val, g = float(val.item()), g.cpu().numpy()
        assert abs(val - ref) <= NLL_TOL * abs(ref), (th, val, ref)
        assert np.max(np.abs(g - gref)) <= GRAD_TOL * max(np.max(np.abs(gref)), G), (th, g, gref)
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

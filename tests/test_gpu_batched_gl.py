"""GPU tests of the batched pass and batched fits for models normalised by
Gauss-Legendre quadrature, whose per-set finishing kernel runs on 128
threads (two quadrature nodes per thread in the per-point set-up): the
2-D Crystal Ball / ARGUS x Chebyshev model, a Crystal Ball alone and a
Chebyshev series alone (one-leaf models, compiled for 8 waves per SIMD),
all with "gl256".  Per set against the scalar oracle (NLL 1e-12 relative,
gradient 1e-8 of the oracle's max-norm); the batched fit against the
oracle's batched fit."""
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


def spec_of(which):
    if which == "c3_gl":
        seed = datagen.data_seed(3)
        return datagen.cb_argus_cheb_spec(cheb=datagen.cheb_coefficients(seed), norm="gl256")
    if which == "cb_gl":
        return {"obs": [{"name": "x", "lo": -6.0, "hi": 4.0}],
                "params": [P("m0", 0.2, -2, 2), P("sigma", 0.8, 0.1, 3), P("alpha", 1.1, 0.2, 5), P("n", 2.5, 1.2, 20)],
                "nodes": [{"kind": "cb", "obs": 0, "params": [0, 1, 2, 3], "norm": "gl256"}], "root": 0}
    return {"obs": [{"name": "x", "lo": -1.0, "hi": 1.0}],
            "params": [P("a1", 0.1, -1, 1), P("a2", -0.2, -1, 1), P("a3", 0.05, -1, 1), P("a4", 0.1, -1, 1)],
            "nodes": [{"kind": "cheb", "obs": 0, "params": [0, 1, 2, 3], "norm": "gl256"}], "root": 0}


@pytest.mark.parametrize("which", ["c3_gl", "cb_gl", "cheb_gl"])
def test_batched_gl_models(torch, nllmi, which):
    spec = spec_of(which)
    n = 60_000
    cols = datagen.generate(spec, n, seed=910)
    offsets = np.array([0, 17, 5000, 5000, 31_000, n], dtype=np.int64)
    pts = datagen.parameter_points(spec, 5, seed=911)
    print(f"[batched gl {which}]", flush=True)
    m = nllmi.Model.from_spec(spec)
    m.set_data([torch.from_numpy(c).cuda() for c in cols])
    o = oracle.Oracle(spec)
    nll, g, st = m.eval_batched(torch.from_numpy(offsets).cuda(), torch.from_numpy(pts).cuda())
    nll, g, st = nll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    for s in range(5):
        a, b = offsets[s], offsets[s + 1]
        assert st[s] == 0
        if b == a:
            assert nll[s] == 0.0 and np.all(g[s] == 0.0)
            continue
        sto, ref, gref = o.nll([c[a:b] for c in cols], pts[s], threads=4)
        assert sto == 0
        assert abs(nll[s] / ref - 1.0) <= NLL_TOL, (s, nll[s], ref)
        assert np.max(np.abs(g[s] - gref)) <= GRAD_TOL * np.max(np.abs(gref)), (s, g[s], gref)
    # batched gradient-descent fits (the finishing kernel's update and next
    # constants) against the oracle's batched fits of the same sets
    steps = 3
    th, f, gg, stt = m.fit_batched(torch.from_numpy(offsets).cuda(), torch.from_numpy(pts).cuda(), steps)
    st_all, th_o, f_o, g_o, sto = o.gd_fit_batched(cols, offsets, pts, steps, 1.0, threads=4)
    th, f, stt = th.cpu().numpy(), f.cpu().numpy(), stt.cpu().numpy()
    for s in range(5):
        if offsets[s + 1] == offsets[s]:
            continue
        assert stt[s] == 0 and sto[s] == 0, (s, stt[s], sto[s])
        assert abs(f[s] / f_o[s] - 1.0) <= NLL_TOL, (s, f[s], f_o[s])
        np.testing.assert_allclose(th[s], th_o[s], rtol=1e-10, atol=1e-12)

"""nll_eval_batched_noalloc through the C ABI: the batched evaluation with
its scratch in the library's fixed per-GPU device array instead of the
model's own buffers.  Same kernels and launch schedule as nll_eval_batched,
so NLL, gradient and status must be the same bits; a few sets are also
checked against the scalar oracle at the parity tolerances (NLL 1e-12
relative, gradient 1e-8 of the oracle's max-norm), for a two-component
mixture and for a Hypatia2 leaf (whose per-set tables also live there).  Two calls in a row, the
second with fewer sets over fewer events, and a request larger than the
array refused before anything is enqueued."""
import ctypes

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


def _sets(seed, n_sets, lo, hi):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, n_sets)
    offsets = np.zeros(n_sets + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return offsets


def _call(torch, L, fn, model, offsets, theta, grad=True):
    n_sets = len(offsets) - 1
    P = theta.shape[1]
    off = torch.from_numpy(offsets).cuda()
    th = torch.from_numpy(np.ascontiguousarray(theta)).cuda()
    nll = torch.full((n_sets,), -1.0, dtype=torch.float64, device="cuda")
    g = torch.full((n_sets, P), -1.0, dtype=torch.float64, device="cuda") if grad else None
    st = torch.full((n_sets,), 7, dtype=torch.int32, device="cuda")
    rc = getattr(L, fn)(model._h, n_sets, off.data_ptr(), th.data_ptr(), nll.data_ptr(),
                        g.data_ptr() if grad else None, st.data_ptr())
    torch.cuda.synchronize()
    return rc, nll.cpu().numpy(), (g.cpu().numpy() if grad else None), st.cpu().numpy()


def _hypatia_spec():
    """A Hypatia2 leaf (its per-set Bessel tables also live in the array)."""
    P = datagen.param
    return {"obs": [{"name": "m", "lo": -8.0, "hi": 8.0}],
            "params": [P("mu", 0.0, -8.0, 8.0, jitter=0.05), P("sigma", 1.0, 1e-6, 100.0, jitter=0.05),
                       P("lambda", -1.2, -6.0, 6.0, jitter=0.06), P("zeta", 0.05, 1e-3, 100.0, jitter=0.0025),
                       P("beta", 0.1, -50.0, 50.0, jitter=0.02), P("a_l", 1.5, 0.05, 20.0, jitter=0.075),
                       P("n_l", 2.0, 1.001, 100.0, jitter=0.1), P("a_r", 1.8, 0.05, 20.0, jitter=0.09),
                       P("n_r", 6.0, 1.001, 100.0, jitter=0.3)],
            "nodes": [{"kind": "hypatia", "obs": 0, "params": list(range(9))}], "root": 0}


@pytest.mark.parametrize("model", ["mixture", "hypatia"])
def test_noalloc_matches_batched_and_oracle(torch, nllmi, threads, model):
    L = nllmi.lib()
    spec = datagen.mixture_spec() if model == "mixture" else _hypatia_spec()
    offsets = _sets(71, 700, 1, 20_000)  # uneven sets, several tiles each, ragged tails
    n = int(offsets[-1])
    cols = datagen.generate(spec, n, seed=72)
    m = nllmi.Model.from_spec(spec)
    m.set_data([torch.from_numpy(c).cuda() for c in cols])
    if model == "mixture":
        base = np.array([p["value"] for p in spec["params"]])
        rng = np.random.default_rng(73)
        theta = base * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, (700, len(base))))
    else:
        theta = datagen.parameter_points(spec, 700, seed=73)
    o = oracle.Oracle(spec)
    # first call: all 700 sets; second: 90 sets over the first part of the
    # events (fewer sets, fewer events, the array keeps the first call's data)
    small = _sets(74, 90, 0, 3_000)
    assert small[-1] <= n
    for step, (off, th) in enumerate(((offsets, theta), (small, theta[:90]))):
        print(f"[noalloc {model} call {step}: {len(off) - 1} sets, {int(off[-1])} events]", flush=True)
        for grad in (False, True):  # the gradient run last: its results are checked below
            rc_a, nll_a, g_a, st_a = _call(torch, L, "nll_eval_batched_noalloc", m, off, th, grad)
            rc_b, nll_b, g_b, st_b = _call(torch, L, "nll_eval_batched", m, off, th, grad)
            assert rc_a == 0 and rc_b == 0
            assert np.array_equal(st_a, st_b)
            assert np.array_equal(nll_a.view(np.int64), nll_b.view(np.int64))
            if grad:
                assert np.array_equal(g_a.view(np.int64), g_b.view(np.int64))
        # oracle parity on a few sets, including an empty one if present
        picks = sorted({0, 1, len(off) // 2, len(off) - 2} | set(np.flatnonzero(np.diff(off) == 0)[:2].tolist()))
        for s in picks:
            a, b = int(off[s]), int(off[s + 1])
            sub = [c[a:b] for c in cols]
            st, ref, gref = o.nll(sub, th[s], threads=threads)
            assert st == st_a[s] == 0, (s, st, st_a[s])
            assert abs(nll_a[s] - ref) <= 1e-12 * max(abs(ref), 1e-300) or (b == a and nll_a[s] == ref), (s, nll_a[s], ref)
            if b > a:
                assert np.max(np.abs(g_a[s] - gref)) <= 1e-8 * np.max(np.abs(gref)), (s, g_a[s], gref)
    assert m.sync() == 0


def test_noalloc_refuses_oversized_request(torch, nllmi):
    """More sets than the array can hold: NLL_ERR_SCRATCH before anything is
    enqueued (the outputs keep their sentinel values)."""
    L = nllmi.lib()
    spec = datagen.gauss_spec()
    cols = datagen.generate(spec, 50_000, seed=75)
    m = nllmi.Model.from_spec(spec)
    m.set_data([torch.from_numpy(c).cuda() for c in cols])
    per_set = m.info["per_set_bytes"]
    n_sets = (32 << 20) // per_set + 16
    offsets = np.linspace(0, 50_000, n_sets + 1).astype(np.int64)
    theta = np.tile(np.array([0.3, 1.5]), (n_sets, 1))
    rc, nll, g, st = _call(torch, L, "nll_eval_batched_noalloc", m, offsets, theta)
    assert rc == -9
    assert np.all(nll == -1.0) and np.all(st == 7)
    # the same request through the allocating entry point works
    rc, nll, g, st = _call(torch, L, "nll_eval_batched", m, offsets, theta)
    assert rc == 0 and np.all(st == 0)
    assert m.sync() == 0

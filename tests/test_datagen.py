"""The seeded input generator: Philox4x64-10 known answers, agreement with
numpy's independent Philox implementation, thread independence, and the
distribution of sampled events against library CDFs (KS tests)."""
import math

import numpy as np
import pytest
from scipy import stats

import datagen


def test_philox_known_answer_and_numpy():
    # Random123 known-answer vector for zero counter and key
    assert datagen.philox4x64([0, 0, 0, 0], [0, 0]) == [
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]
    # numpy's Philox (4x64, 10 rounds) increments the counter before each block
    for key, ctr in (([5, 7], [3, 0, 0, 0]), ([2 ** 63 + 11, 99], [2 ** 40, 1, 2, 3])):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
        want = [int(v) for v in bg.random_raw(4)]
        nxt = list(ctr)
        nxt[0] += 1
        assert datagen.philox4x64(nxt, key) == want


def test_thread_independence():
    spec = datagen.mixture_spec()
    a = datagen.generate(spec, 200_000, seed=17, threads=1)[0]
    b = datagen.generate(spec, 200_000, seed=17, threads=7)[0]
    assert np.array_equal(a, b)


def _ks(x, cdf):
    return stats.kstest(x, cdf).pvalue


def test_gauss_and_exp_samples():
    x = datagen.generate(datagen.gauss_spec(), 100_000, seed=3)[0]
    assert _ks(x, stats.truncnorm((-10 - 0.3) / 1.5, (10 - 0.3) / 1.5, loc=0.3, scale=1.5).cdf) > 1e-3
    spec = datagen.mixture_spec(f=0.0)
    x = datagen.generate(spec, 100_000, seed=4)[0]
    assert _ks(x, stats.truncexpon(b=7.0, loc=0.0, scale=1 / 0.7).cdf) > 1e-3


def test_mixture_samples():
    spec = datagen.mixture_spec()
    x = datagen.generate(spec, 100_000, seed=5)[0]
    g = stats.truncnorm((0 - 5) / 0.4, (10 - 5) / 0.4, loc=5, scale=0.4)
    e = stats.truncexpon(b=7.0, loc=0.0, scale=1 / 0.7)
    assert _ks(x, lambda v: 0.2 * g.cdf(v) + 0.8 * e.cdf(v)) > 1e-3


def test_cb_argus_cheb_samples():
    a = datagen.cheb_coefficients(datagen.data_seed(3))
    spec = datagen.cb_argus_cheb_spec(cheb=a)
    m, y = datagen.generate(spec, 60_000, seed=6)
    cb = stats.crystalball(1.5, 3.0, loc=5.28, scale=0.003)
    ar = stats.argus(math.sqrt(40.0), scale=5.29)
    zc = cb.cdf(5.30) - cb.cdf(5.20)
    za = ar.cdf(5.29) - ar.cdf(5.20)
    cdf_m = lambda v: 0.1 * (cb.cdf(v) - cb.cdf(5.20)) / zc + 0.9 * (ar.cdf(np.minimum(v, 5.29)) - ar.cdf(5.20)) / za
    assert _ks(m, cdf_m) > 1e-3
    coef = np.concatenate([[1.0], a])
    anti = np.polynomial.chebyshev.chebint(coef, lbnd=-1.0)
    tot = np.polynomial.chebyshev.chebval(1.0, anti)
    assert _ks(y, lambda v: np.polynomial.chebyshev.chebval(v, anti) / tot) > 1e-3
    assert np.polynomial.chebyshev.chebval(np.linspace(-1, 1, 10001), coef).min() >= 0.05


def test_points_and_toys():
    w = datagen.workload(2, n=10)
    th = w["theta"]
    assert np.all(np.abs(w["points"] / th - 1) <= 0.1 + 1e-15)
    w3 = datagen.workload(3, n=10)
    free = datagen.free_mask(w3["spec"])
    assert np.all(w3["points"][:, ~free] == w3["theta"][~free])
    assert np.all(np.abs(w3["points"][:, 1] - 5.28) <= 0.0003 + 1e-15)
    sizes = datagen.toy_sizes(4096, datagen.data_seed(4))
    assert sizes.min() >= 1000 and sizes.max() <= 200000
    assert abs(sizes.mean() - 100500) < 3 * 57500 / math.sqrt(4096)


def test_hf_workload_is_seeded_and_well_formed():
    a = datagen.hf_workload(n_bins=3000, n_samples=3, n_histosys=5, n_normsys=2, n_points=2)
    b = datagen.hf_workload(n_bins=3000, n_samples=3, n_histosys=5, n_normsys=2, n_points=2)
    assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["points"], b["points"])
    assert all(np.array_equal(x, y) for x, y in zip(a["up"], b["up"]))
    assert np.all(a["counts"] >= 0) and np.all(a["counts"] == np.floor(a["counts"]))
    assert all(np.all(t > 0) for t in a["nominal"] + a["up"] + a["down"])
    spec = a["spec"]
    assert len(spec["params"]) == 2 + 5 + 2
    assert sum(m["type"] == "histosys" for m in spec["modifiers"]) == 5
    # alphas jittered over both sides of the interpolation
    al = a["points"][:, 2:]
    assert np.any(al < 0) and np.any(al > 0)

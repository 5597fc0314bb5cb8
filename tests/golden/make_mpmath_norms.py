"""Write mpmath_norms.json: normalisation integrals of the leaf shapes at
40 significant digits by mpmath's tanh-sinh quadrature, split at the kinks.

The shapes are the textbook densities the paper's models are built from
(Sec. 3 and 5): Gaussian, exponential, Chebyshev series with unit T_0
coefficient, Crystal Ball with a low-side power-law tail, ARGUS with power
1/2, Johnson's S_U, chi-square.  This script calls only mpmath; the stored numbers pin the closed
forms and the Gauss-Legendre rules of both implementations.

    python tests/golden/make_mpmath_norms.py
"""
import json
import os

import mpmath as mp

mp.mp.dps = 40

CASES = [
    ("gauss", ["0.3", "1.5"], "-10", "10"),
    ("gauss", ["5", "0.4"], "0", "10"),
    ("gauss", ["2", "0.7"], "4", "9"),
    ("exp", ["-0.7"], "0", "10"),
    ("exp", ["0.35"], "-2", "3"),
    ("cheb", ["-0.28", "-0.27", "-0.07", "0.1"], "-1", "1"),
    ("cb", ["5.28", "0.003", "1.5", "3"], "5.20", "5.30"),
    ("cb", ["0", "1", "1", "2.5"], "-8", "4"),
    ("argus", ["5.29", "-20"], "5.20", "5.30"),
    ("argus", ["1", "-5"], "0.1", "0.95"),
    ("johnson", ["5.28", "0.02", "-0.5", "1.5"], "5.0", "5.6"),
    ("johnson", ["0", "1", "0.8", "0.7"], "-10", "10"),
    ("johnson", ["0", "1", "0", "1"], "5", "30"),
    ("chi2", ["5"], "0", "40"),
    ("chi2", ["3.5"], "0", "12"),
    ("chi2", ["30"], "10", "60"),
]


def shape(kind, p, lo, hi):
    if kind == "gauss":
        mu, s = p
        return lambda x: mp.exp(-((x - mu) / s) ** 2 / 2), [mu]
    if kind == "exp":
        (c,) = p
        return lambda x: mp.exp(c * x), []
    if kind == "cheb":
        def g(x):
            y = (2 * x - lo - hi) / (hi - lo)
            return 1 + sum(a * mp.chebyt(k + 1, y) for k, a in enumerate(p))
        return g, []
    if kind == "cb":
        m0, s, al, n = p
        A = (n / al) ** n * mp.exp(-al ** 2 / 2)
        B = n / al - al

        def g(x):
            t = (x - m0) / s
            return mp.exp(-t * t / 2) if t > -al else A * (B - t) ** (-n)
        return g, [m0 - al * s, m0]
    if kind == "argus":
        m0, c = p

        def g(x):
            if x >= m0:
                return mp.mpf(0)
            u = 1 - (x / m0) ** 2
            return x * mp.sqrt(u) * mp.exp(c * u)
        return g, [m0]
    if kind == "johnson":
        mu, la, ga, de = p

        def g(x):
            z = (x - mu) / la
            return mp.exp(-(ga + de * mp.asinh(z)) ** 2 / 2) / mp.sqrt(1 + z * z)
        return g, [mu]
    if kind == "chi2":
        (nu,) = p
        return lambda x: x ** (nu / 2 - 1) * mp.exp(-x / 2), []
    raise ValueError(kind)


def main():
    out = []
    for kind, ps, lo, hi in CASES:
        p = [mp.mpf(v) for v in ps]
        a, b = mp.mpf(lo), mp.mpf(hi)
        g, kinks = shape(kind, p, a, b)
        pts = [a] + sorted(k for k in kinks if a < k < b) + [b]
        z = mp.quad(g, pts)
        out.append({"kind": kind, "params": [float(v) for v in p], "lo": float(a), "hi": float(b),
                    "Z": mp.nstr(z, 35)})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mpmath_norms.json")
    with open(path, "w") as f:
        json.dump({"source": "mpmath quad, 40 digits, split at kinks; shapes per the textbook "
                             "definitions of the paper's built-in densities (Sec. 3, 5)",
                   "cases": out}, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()

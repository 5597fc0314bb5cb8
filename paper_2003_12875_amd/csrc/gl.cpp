// gl.cpp -- the n-point Gauss-Legendre rule used by the device prologue for
// numerical normalisation (Sec. 3: integrals are numerical unless a closed
// form is provided).
//
// Nodes: Tricomi's asymptotic starting values
//   x_k ~ (1 - 1/(8 n^2) + 1/(8 n^3)) cos(pi (4k - 1) / (4n + 2)),
// refined by Newton steps on P_n, evaluated by the Bonnet recurrence in
// extended precision.  Weights: w_k = 2 (1 - x_k^2) / (n P_{n-1}(x_k))^2.
#include <cmath>

namespace nllmi {

static void legendre_pair(int n, long double x, long double* pn, long double* pn1) {
  long double a = 1.0L, b = x;  // P_0, P_1
  for (int j = 2; j <= n; ++j) {
    const long double c = ((2 * j - 1) * x * b - (j - 1) * a) / j;
    a = b;
    b = c;
  }
  *pn = b;   // P_n
  *pn1 = a;  // P_{n-1}
}

void gauss_legendre(int n, double* nodes, double* weights) {
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int k = 1; k <= n / 2 + (n & 1); ++k) {
    const long double nn = n;
    long double x = (1.0L - 1.0L / (8 * nn * nn) + 1.0L / (8 * nn * nn * nn)) *
                    cosl(pi * (4 * k - 1) / (4 * nn + 2));
    long double pn = 0, pn1 = 0;
    for (int it = 0; it < 64; ++it) {
      legendre_pair(n, x, &pn, &pn1);
      const long double dp = nn * (pn1 - x * pn) / (1.0L - x * x);  // P_n'
      const long double dx = pn / dp;
      x -= dx;
      if (fabsl(dx) <= 1e-20L * (1.0L + fabsl(x))) break;
    }
    legendre_pair(n, x, &pn, &pn1);
    const long double w = 2.0L * (1.0L - x * x) / ((nn * pn1) * (nn * pn1));
    // k-th largest root at index n-k, its mirror at k-1
    nodes[n - k] = (double)x;
    weights[n - k] = (double)w;
    nodes[k - 1] = (double)(-x);
    weights[k - 1] = (double)w;
  }
  if (n & 1) nodes[n / 2] = 0.0;
}

}  // namespace nllmi

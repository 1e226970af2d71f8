// Gauss-Legendre S_N quadrature on the host (Sec. "ONE-CELL INVERSION":
// Gauss-Legendre quadrature in all explorations; weights sum to 2, matching
// the 1/2 in front of the scattering source of the S_N equation).
//
// Nodes are the zeros of P_n, refined by Newton's method; P_n and P_n' come
// from the three-term recurrences (k+1)P_{k+1} = (2k+1)x P_k - k P_{k-1} and
// P'_{k+1} = P'_{k-1} + (2k+1) P_k.  Weight 2 / ((1 - x^2) P_n'(x)^2).
// Output ascending.
#include <cmath>

#include "oci.h"

namespace {

void legendre(int n, double x, double *p_out, double *d_out) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) {
    *p_out = 1.0;
    *d_out = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    const double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  *p_out = p1;
  *d_out = d1;
}

}  // namespace

extern "C" int oci_gauss_legendre(int32_t n, double *mu, double *w) {
  if (n < 1 || n > 4096 || !mu || !w) return OCI_EINVAL;
  const double pi = 3.14159265358979323846;
  // roots come out descending for i = 1..n; store ascending
  for (int i = 1; i <= n; ++i) {
    double x = std::cos(pi * (i - 0.25) / (n + 0.5));
    double p, d;
    for (int it = 0; it < 100; ++it) {
      legendre(n, x, &p, &d);
      const double dx = p / d;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    legendre(n, x, &p, &d);
    const int slot = n - i;
    mu[slot] = x;
    w[slot] = 2.0 / ((1.0 - x * x) * d * d);
  }
  return OCI_OK;
}

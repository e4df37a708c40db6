// Quadrature rules for the Galerkin entries (see quadrules.h).
//
// * Radon's degree-5 seven-point rule: the published constants of that rule.
// * Conical product rule: Gauss-Legendre in both directions of the unit square,
//   mapped onto the triangle by (s, t) -> (s, t (1 - s)).
// * Sauter-Schwab: the regularising substitutions for identical triangles, a
//   common edge (P0P1 in both triangles) and a common vertex (P0 in both), each
//   a sum of terms over the 4D unit cube whose Jacobian cancels the 1/r
//   singularity (Sauter & Schwab, Boundary Element Methods, Sec. 5.2).
#include "quadrules.h"

#include <cmath>
#include <stdexcept>

namespace h2 {

void gauss_legendre_unit(int q, std::vector<double>& t, std::vector<double>& w) {
  if (q < 1 || q > 64) throw std::runtime_error("Gauss-Legendre order out of range");
  t.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < q; ++i) {
    double x = std::cos(pi * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= q; ++j) {
        const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      const double pq = (q == 1) ? x : p1;
      const double pqm1 = (q == 1) ? 1.0 : p0;
      dp = q * (x * pq - pqm1) / (x * x - 1.0);
      const double dx = pq / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    // recompute the derivative at the converged root
    double p0 = 1.0, p1 = x;
    for (int j = 2; j <= q; ++j) {
      const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    const double pq = (q == 1) ? x : p1, pqm1 = (q == 1) ? 1.0 : p0;
    dp = q * (x * pq - pqm1) / (x * x - 1.0);
    t[q - 1 - i] = 0.5 * (x + 1.0);
    w[q - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);  // (2 / ((1-x^2) P'^2)) / 2
  }
}

TriRule radon_seven_point() {
  const double r = std::sqrt(15.0);
  const double a = (6.0 - r) / 21.0, b = (9.0 + 2.0 * r) / 21.0;
  const double c = (6.0 + r) / 21.0, d = (9.0 - 2.0 * r) / 21.0;
  const double wa = (155.0 - r) / 1200.0, wc = (155.0 + r) / 1200.0;
  TriRule R;
  R.lam = {1.0 / 3, 1.0 / 3, 1.0 / 3, b, a, a, a, b, a, a, a, b, d, c, c, c, d, c, c, c, d};
  R.w = {9.0 / 40.0, wa, wa, wa, wc, wc, wc};
  return R;
}

TriRule conical_product_rule(int q) {
  std::vector<double> t, w;
  gauss_legendre_unit(q, t, w);
  TriRule R;
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      const double u = t[i], v = t[j] * (1.0 - t[i]);
      R.lam.push_back(1.0 - u - v);
      R.lam.push_back(u);
      R.lam.push_back(v);
      R.w.push_back(2.0 * w[i] * w[j] * (1.0 - t[i]));
    }
  return R;
}

std::vector<double> sauter_schwab_rule(SSCase cs, int q) {
  std::vector<double> t, w;
  gauss_legendre_unit(q, t, w);
  std::vector<double> out;
  auto put = [&](double x1, double x2, double y1, double y2, double wt) {
    out.push_back(x1);
    out.push_back(x2);
    out.push_back(y1);
    out.push_back(y2);
    out.push_back(wt);
  };
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b)
      for (int c = 0; c < q; ++c)
        for (int d = 0; d < q; ++d) {
          const double xi = t[a], e1 = t[b], e2 = t[c], e3 = t[d];
          const double W = w[a] * w[b] * w[c] * w[d];
          const double x3 = xi * xi * xi;
          if (cs == SS_IDENTICAL) {
            const double J = W * x3 * e1 * e1 * e2;
            const double p = xi * (1.0 - e1 + e1 * e2), pp = xi * (1.0 - e1 * e2 * e3), q1 = xi * (1.0 - e1);
            put(xi, p, pp, q1, J);
            put(pp, q1, xi, p, J);
            const double r1 = xi * e1 * (1.0 - e2 + e2 * e3), r2 = xi * (1.0 - e1 * e2), r3 = xi * e1 * (1.0 - e2);
            put(xi, r1, r2, r3, J);
            put(r2, r3, xi, r1, J);
            const double s1 = xi * e1 * (1.0 - e2 * e3);
            put(pp, s1, xi, r3, J);
            put(xi, r3, pp, s1, J);
          } else if (cs == SS_EDGE) {
            const double J1 = W * x3 * e1 * e1, J = J1 * e2;
            put(xi, xi * e1 * e3, xi * (1.0 - e1 * e2), xi * e1 * (1.0 - e2), J1);
            const double u1 = xi * (1.0 - e1 * e2 * e3), u2 = xi * e1 * e2 * (1.0 - e3);
            put(xi, xi * e1, u1, u2, J);
            put(xi * (1.0 - e1 * e2), xi * e1 * (1.0 - e2), xi, xi * e1 * e2 * e3, J);
            put(u1, u2, xi, xi * e1, J);
            put(u1, xi * e1 * (1.0 - e2 * e3), xi, xi * e1 * e2, J);
          } else {
            const double J = W * x3 * e2;
            put(xi, xi * e1, xi * e2, xi * e2 * e3, J);
            put(xi * e2, xi * e2 * e3, xi, xi * e1, J);
          }
        }
  return out;
}

}  // namespace h2

// Quadrature rules of the library, generated on the host in FP64.
#pragma once
#include <vector>

namespace h2 {

// Gauss-Legendre points/weights on [0, 1] by Newton's method on P_q.
void gauss_legendre_unit(int q, std::vector<double>& t, std::vector<double>& w);

// Triangle rule in barycentric form: lam (3 per point), weights summing to 1.
struct TriRule {
  std::vector<double> lam, w;
  int size() const { return static_cast<int>(w.size()); }
};
TriRule radon_seven_point();                 // degree 5 (regular near-field pairs)
TriRule conical_product_rule(int q);         // exact to total degree 2q - 2

// Sauter-Schwab rules on T x T with T = {0 <= x2 <= x1 <= 1}; each point holds
// (x1, x2, y1, y2, weight).  The weights carry the Jacobians of the
// transformations and sum to |T|^2 = 1/4 for q >= 2 (two Gauss points per axis
// integrate those Jacobians exactly; q = 1 does not).
enum SSCase { SS_IDENTICAL = 0, SS_EDGE = 1, SS_VERTEX = 2 };
std::vector<double> sauter_schwab_rule(SSCase c, int q);

}  // namespace h2

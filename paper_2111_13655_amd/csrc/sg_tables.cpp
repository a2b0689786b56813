// One-mode tables of the "Hm" primitive basis (harmonic-oscillator Hermite
// functions, Q0 = 0, scaleQ = 1) and its Gauss-Hermite grid.
//
// Nodes: eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// Hermite weight exp(-x^2) (off-diagonal sqrt(k/2)), found with cyclic Jacobi
// rotations and then polished by Newton steps on the Hermite function of
// order n.  Modified weights wt_u = w_u exp(x_u^2) from the Christoffel
// identity wt_u = 1 / sum_{k<n} b_k(x_u)^2 (b_k orthonormal Hermite
// functions), which is the weight that makes sum_u wt_u f(x_u) the quadrature
// of the plain integral of f used by the grid -> basis transform
// (eq_g_to_b, Sec. 2).
#include <algorithm>
#include <cmath>
#include <vector>

#include "sg_internal.h"

namespace sg {

// b_0..b_{nb-1} at x: b_0 = pi^{-1/4} e^{-x^2/2}, b_1 = sqrt(2) x b_0,
// b_{n+1} = sqrt(2/(n+1)) x b_n - sqrt(n/(n+1)) b_{n-1}.
void hermite_function_values(int nb, double x, double *b) {
  if (nb <= 0) return;
  b[0] = std::pow(M_PI, -0.25) * std::exp(-0.5 * x * x);
  if (nb > 1) b[1] = std::sqrt(2.0) * x * b[0];
  for (int n = 1; n + 1 < nb; ++n)
    b[n + 1] = std::sqrt(2.0 / (n + 1)) * x * b[n] - std::sqrt(double(n) / (n + 1)) * b[n - 1];
}

void jacobi_eigen(std::vector<double> a, int n, std::vector<double> *evals,
                  std::vector<double> *evecs) {
  auto A = [&](int i, int j) -> double & { return a[size_t(i) * n + j]; };
  std::vector<double> v;
  if (evecs) {
    v.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) v[size_t(i) * n + i] = 1.0;
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A(i, i) * A(i, i);
      for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
    }
    if (off <= 1e-32 * diag || off < 1e-300) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        // rotation angle that zeroes A(p,q)
        double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = cs * akp - sn * akq;
          A(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = cs * apk - sn * aqk;
          A(q, k) = sn * apk + cs * aqk;
        }
        if (evecs) {
          for (int k = 0; k < n; ++k) {
            double vkp = v[size_t(k) * n + p], vkq = v[size_t(k) * n + q];
            v[size_t(k) * n + p] = cs * vkp - sn * vkq;
            v[size_t(k) * n + q] = sn * vkp + cs * vkq;
          }
        }
      }
    }
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
  evals->resize(n);
  for (int i = 0; i < n; ++i) (*evals)[i] = A(order[i], order[i]);
  if (evecs) {
    evecs->assign(size_t(n) * n, 0.0);
    for (int k = 0; k < n; ++k)
      for (int i = 0; i < n; ++i) (*evecs)[size_t(k) * n + i] = v[size_t(k) * n + order[i]];
  }
}

void gauss_hermite_nodes(int n, std::vector<double> *x, std::vector<double> *wt) {
  std::vector<double> J(size_t(n) * n, 0.0);
  for (int k = 1; k < n; ++k) J[size_t(k - 1) * n + k] = J[size_t(k) * n + k - 1] = std::sqrt(k / 2.0);
  std::vector<double> nodes;
  jacobi_eigen(J, n, &nodes, nullptr);
  std::vector<double> b(n + 1);
  for (int i = 0; i < n; ++i) {
    double xi = nodes[i];
    for (int it = 0; it < 8; ++it) {  // Newton on b_n: b_n' = sqrt(2n) b_{n-1} - x b_n
      hermite_function_values(n + 1, xi, b.data());
      double d = std::sqrt(2.0 * n) * b[n - 1] - xi * b[n];
      if (d == 0.0) break;
      double step = b[n] / d;
      xi -= step;
      if (std::fabs(step) < 1e-16 * std::max(1.0, std::fabs(xi))) break;
    }
    nodes[i] = xi;
  }
  // symmetrise (the rule is symmetric about 0)
  for (int i = 0; i < n / 2; ++i) {
    double m = 0.5 * (nodes[n - 1 - i] - nodes[i]);
    nodes[i] = -m;
    nodes[n - 1 - i] = m;
  }
  if (n % 2) nodes[n / 2] = 0.0;
  x->assign(nodes.begin(), nodes.end());
  wt->resize(n);
  for (int i = 0; i < n; ++i) {
    hermite_function_values(n, nodes[i], b.data());
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += b[k] * b[k];
    (*wt)[i] = 1.0 / s;
  }
}

}  // namespace sg

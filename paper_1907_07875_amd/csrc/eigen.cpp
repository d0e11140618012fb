// FP64 symmetric eigensolver: Householder tridiagonalisation + implicit Wilkinson-shift QR.
#include "eigen.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace gft {

namespace {

// Reduce symmetric A (n x n, row-major, overwritten) to tridiagonal T = Q^T A Q.
// Returns diag d, off-diagonal e (e[i] couples i and i+1) and Qt = Q^T (row-major), so
// that row k of Qt is column k of Q.
void tridiagonalize(int n, std::vector<double> &A, std::vector<double> &d,
                    std::vector<double> &e, std::vector<double> &Qt) {
  Qt.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Qt[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double norm2 = 0.0;
    for (int i = 0; i < m; ++i) {
      const double a = A[(size_t)(k + 1 + i) * n + k];
      v[i] = a;
      norm2 += a * a;
    }
    const double norm = std::sqrt(norm2);
    if (norm == 0.0) continue;
    const double alpha = v[0] > 0 ? -norm : norm;  // new sub-diagonal entry
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < m; ++i) vn2 += v[i] * v[i];
    if (vn2 == 0.0) continue;
    const double inv = 1.0 / std::sqrt(vn2);
    for (int i = 0; i < m; ++i) v[i] *= inv;  // H = I - 2 v v^T, |v| = 1
    // p = A22 v, K = v^T p, w = p - K v; A22 <- A22 - 2 (v w^T + w v^T)
    double K = 0.0;
    for (int i = 0; i < m; ++i) {
      const double *row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = s;
      K += v[i] * s;
    }
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i) {
      double *row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      const double vi = v[i], wi = w[i];
      for (int j = 0; j < m; ++j) row[j] -= 2.0 * (vi * w[j] + wi * v[j]);
    }
    A[(size_t)(k + 1) * n + k] = alpha;
    A[(size_t)k * n + (k + 1)] = alpha;
    for (int i = 1; i < m; ++i) {
      A[(size_t)(k + 1 + i) * n + k] = 0.0;
      A[(size_t)k * n + (k + 1 + i)] = 0.0;
    }
    // Q <- Q H, i.e. Qt <- H Qt on rows k+1..n-1: Qt22 -= 2 v (v^T Qt22)
    std::vector<double> t(n, 0.0);
    for (int i = 0; i < m; ++i) {
      const double *row = &Qt[(size_t)(k + 1 + i) * n];
      const double vi = v[i];
      for (int j = 0; j < n; ++j) t[j] += vi * row[j];
    }
    for (int i = 0; i < m; ++i) {
      double *row = &Qt[(size_t)(k + 1 + i) * n];
      const double c = 2.0 * v[i];
      for (int j = 0; j < n; ++j) row[j] -= c * t[j];
    }
  }
  d.resize(n);
  e.assign(n > 1 ? n - 1 : 0, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
}

// Deflation test for the off-diagonal e between diagonal entries a and b: relative to its
// neighbours, or absolutely against the norm of the whole tridiagonal matrix.
inline bool negligible(double e, double a, double b, double tnorm) {
  constexpr double eps = 2.220446049250313e-16;
  return std::fabs(e) <= eps * (std::fabs(a) + std::fabs(b)) || std::fabs(e) <= eps * tnorm;
}

}  // namespace

bool symmetric_eigen(int n, const std::vector<double> &Ain, std::vector<double> &lambda,
                     std::vector<double> &V) {
  lambda.assign(n, 0.0);
  V.assign((size_t)n * n, 0.0);
  if (n == 0) return true;
  if (n == 1) {
    lambda[0] = Ain[0];
    V[0] = 1.0;
    return true;
  }
  std::vector<double> A(Ain);
  // symmetrise defensively
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
      A[(size_t)i * n + j] = A[(size_t)j * n + i] = s;
    }
  std::vector<double> d, e, Qt;
  tridiagonalize(n, A, d, e, Qt);

  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) tnorm = std::max(tnorm, std::fabs(d[i]));
  for (int i = 0; i + 1 < n; ++i) tnorm = std::max(tnorm, std::fabs(e[i]));
  const int max_iter = 60 * n + 100;
  int iter = 0;
  int m = n - 1;
  while (m > 0) {
    if (negligible(e[m - 1], d[m - 1], d[m], tnorm)) {
      e[m - 1] = 0.0;
      --m;
      continue;
    }
    int l = m - 1;
    while (l > 0 && !negligible(e[l - 1], d[l - 1], d[l], tnorm)) --l;
    if (l > 0) e[l - 1] = 0.0;
    if (++iter > max_iter) return false;
    // Wilkinson shift from the trailing 2x2 block of the unreduced block l..m
    const double dd = 0.5 * (d[m - 1] - d[m]);
    const double em = e[m - 1];
    const double hyp = std::hypot(dd, em);
    const double mu = d[m] - em * em / (dd + (dd >= 0 ? hyp : -hyp));
    double x = d[l] - mu;
    double z = e[l];
    for (int k = l; k < m; ++k) {
      // rotation R = [[c, s], [-s, c]] on (k, k+1) with R [x; z] = [r; 0]
      const double r = std::hypot(x, z);
      const double c = r == 0.0 ? 1.0 : x / r;
      const double s = r == 0.0 ? 0.0 : z / r;
      if (k > l) e[k - 1] = r;
      const double a = d[k], b = e[k], cc = d[k + 1];
      d[k] = c * c * a + 2.0 * c * s * b + s * s * cc;
      d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * cc;
      e[k] = c * s * (cc - a) + (c * c - s * s) * b;
      if (k + 1 < m) {
        const double next = e[k + 1];
        z = s * next;         // bulge at (k, k+2), rotated into (k+2, k) next step
        e[k + 1] = c * next;
        x = e[k];
      }
      // eigenvectors: Q <- Q R^T, i.e. rows k, k+1 of Qt rotate by R
      double *qk = &Qt[(size_t)k * n];
      double *qk1 = &Qt[(size_t)(k + 1) * n];
      for (int j = 0; j < n; ++j) {
        const double u = qk[j], w = qk1[j];
        qk[j] = c * u + s * w;
        qk1[j] = -s * u + c * w;
      }
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int k = 0; k < n; ++k) {
    lambda[k] = d[order[k]];
    const double *q = &Qt[(size_t)order[k] * n];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + k] = q[i];
  }
  return true;
}

}  // namespace gft

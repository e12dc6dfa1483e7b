// Symmetric eigendecomposition in float64 on the host: the cyclic Jacobi
// method (Golub and Van Loan, "Matrix Computations", the cyclic Jacobi
// algorithm).  Used once per build on the m x m second-moment matrix of the
// sampled residuals, whose top-r eigenvectors are the left singular vectors
// Proposition 3.1 asks for.  Each eigenvector's sign is fixed so that its
// largest-magnitude entry is positive.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace finger {

void eigh_jacobi(const double* Ain, int m, double* evals, double* Vout) {
  std::vector<double> A(Ain, Ain + (size_t)m * m);
  std::vector<double> V((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  // symmetrize exactly
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) {
      const double v = 0.5 * (A[(size_t)i * m + j] + A[(size_t)j * m + i]);
      A[(size_t)i * m + j] = v;
      A[(size_t)j * m + i] = v;
    }
  double total = 0.0;
  for (double v : A) total += v * v;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) off += A[(size_t)p * m + q] * A[(size_t)p * m + q];
    if (off <= 1e-30 * total || off == 0.0) break;
    for (int p = 0; p < m - 1; ++p) {
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[(size_t)p * m + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
        // rotation angle phi with cot(2 phi) = (a_qq - a_pp) / (2 a_pq);
        // t = tan(phi) is the root of t^2 + 2 theta t - 1 = 0 of smaller size
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // A <- A J (columns p, q)
        for (int k = 0; k < m; ++k) {
          double* row = &A[(size_t)k * m];
          const double akp = row[p], akq = row[q];
          row[p] = c * akp - s * akq;
          row[q] = s * akp + c * akq;
        }
        // A <- J^T A (rows p, q)
        double* rp = &A[(size_t)p * m];
        double* rq = &A[(size_t)q * m];
        for (int k = 0; k < m; ++k) {
          const double apk = rp[k], aqk = rq[k];
          rp[k] = c * apk - s * aqk;
          rq[k] = s * apk + c * aqk;
        }
        rp[q] = 0.0;
        rq[p] = 0.0;
        // V <- V J
        for (int k = 0; k < m; ++k) {
          double* row = &V[(size_t)k * m];
          const double vkp = row[p], vkq = row[q];
          row[p] = c * vkp - s * vkq;
          row[q] = s * vkp + c * vkq;
        }
      }
    }
  }
  std::vector<int> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return A[(size_t)a * m + a] > A[(size_t)b * m + b];
  });
  for (int i = 0; i < m; ++i) {
    const int src = order[i];
    evals[i] = A[(size_t)src * m + src];
    // sign: the entry of largest magnitude (first on ties) is positive
    int jmax = 0;
    for (int k = 1; k < m; ++k)
      if (std::fabs(V[(size_t)k * m + src]) > std::fabs(V[(size_t)jmax * m + src])) jmax = k;
    const double sgn = V[(size_t)jmax * m + src] < 0 ? -1.0 : 1.0;
    for (int k = 0; k < m; ++k) Vout[(size_t)i * m + k] = sgn * V[(size_t)k * m + src];
  }
}

}  // namespace finger

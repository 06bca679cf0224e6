// Host-side closed forms shared by the plan set-up code: the dense Chebyshev
// collocation differentiation matrix (matrix-core operator route and the
// fast-diagonalisation preconditioner).
#pragma once

#include <cmath>
#include <vector>

namespace cheb {

// Ascending Chebyshev-Gauss-Lobatto differentiation matrix on an interval of
// length L (Section 2.2, the collocation derivative at t_j = -cos(pi j / N)):
// off-diagonal entries (c_i / c_j) (-1)^(i+j) / (t_i - t_j) with the node
// difference written as 2 sin(pi (i+j) / 2N) sin(pi (i-j) / 2N), diagonal as the
// negative off-diagonal row sum.  Rows N-i are mirrored from rows i so that the
// centro-antisymmetry D[N-i][N-j] = -D[i][j] holds exactly.  Row-major n x n.
inline void dense_D(int N, double L, std::vector<double>& D) {
  const int n = N + 1;
  D.assign((size_t)n * n, 0.0);
  auto offdiag = [N](int i, int j) {
    const double ci = (i == 0 || i == N) ? 2.0 : 1.0;
    const double cj = (j == 0 || j == N) ? 2.0 : 1.0;
    const double sgn = ((i + j) % 2 == 0) ? 1.0 : -1.0;
    const double dif = 2.0 * std::sin(M_PI * (i + j) / (2.0 * N)) * std::sin(M_PI * (i - j) / (2.0 * N));
    return (ci / cj) * sgn / dif;
  };
  for (int i = 0; 2 * i <= N; ++i) {
    double* row = &D[(size_t)i * n];
    if (2 * i == N) {
      // middle row: antisymmetric about j = N/2, zero diagonal
      for (int j = 0; j < i; ++j) {
        row[j] = offdiag(i, j);
        row[N - j] = -row[j];
      }
      row[i] = 0.0;
      continue;
    }
    double rs = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      row[j] = offdiag(i, j);
      rs += row[j];
    }
    row[i] = -rs;
    double* mir = &D[(size_t)(N - i) * n];
    for (int j = 0; j < n; ++j) mir[N - j] = -row[j];
  }
  for (double& v : D) v *= 2.0 / L;
}

}  // namespace cheb

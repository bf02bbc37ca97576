// Host symmetric eigensolver: cyclic Jacobi rotations (Golub & Van Loan,
// "Matrix Computations", symmetric Schur decomposition).  Used once per
// system to diagonalise the one-body matrix H1, so that the half-step
// exp(-tau H1 / 2) of the Split-2 propagator is exact (Sec. III.A-B).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

void jacobi_eigh(int n, std::vector<double>& a, std::vector<double>& evals,
                 std::vector<double>& evecs) {
  std::vector<double> v((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  // Cyclic sweeps.  An off-diagonal entry that is negligible against the
  // geometric mean of its two diagonal entries is set to zero without a
  // rotation; the iteration ends after a sweep with no rotation.
  const double eps = 1e-17;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotations = 0;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        if (std::fabs(apq) <= eps * std::sqrt(std::fabs(A(p, p) * A(q, q)))) {
          A(p, q) = 0.0;
          A(q, p) = 0.0;
          continue;
        }
        ++rotations;
        const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        const double rho = s / (1.0 + c);
        // A' = J^T A J with J = [[c, s], [-s, c]] in the (p, q) plane, written
        // as small corrections to the old entries (Rutishauser's form).
        A(p, p) -= t * apq;
        A(q, q) += t * apq;
        A(p, q) = 0.0;
        A(q, p) = 0.0;
        for (int r = 0; r < n; ++r) {
          if (r == p || r == q) continue;
          const double arp = A(r, p), arq = A(r, q);
          const double np_ = arp - s * (arq + rho * arp);
          const double nq_ = arq + s * (arp - rho * arq);
          A(r, p) = np_;
          A(p, r) = np_;
          A(r, q) = nq_;
          A(q, r) = nq_;
        }
        for (int k = 0; k < n; ++k) {  // V <- V J
          double* row = &v[(size_t)k * n];
          const double vkp = row[p], vkq = row[q];
          row[p] = vkp - s * (vkq + rho * vkp);
          row[q] = vkq + s * (vkp - rho * vkq);
        }
      }
    }
    if (rotations == 0) break;
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
  evals.assign(n, 0.0);
  evecs.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    evals[j] = A(idx[j], idx[j]);
    for (int k = 0; k < n; ++k) evecs[(size_t)k * n + j] = v[(size_t)k * n + idx[j]];
  }
}

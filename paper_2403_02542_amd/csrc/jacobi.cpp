// Host linear algebra of the set-up: a symmetric eigensolver by cyclic
// Jacobi rotations (Golub & Van Loan, "Matrix Computations", symmetric Schur
// decomposition), used once per system to diagonalise the one-body matrix
// H1 so that the half-step exp(-tau H1 / 2) of the Split-2 propagator is
// exact (Sec. III.A-B); and an orthonormal complement of the trial orbitals
// from a Householder QR.
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

// Orthonormal basis of the orthogonal complement of the columns of psi
// (m x n, row-major, orthonormal columns), from the Householder QR of psi:
// Q = H_0 H_1 ... H_{n-1}, and the complement is Q e_c for c = n .. m-1.
// out[(c - n) * m + p] = Q[p][c] (one complement vector per row).
void complement_basis(int m, int n, const std::vector<double>& psi, std::vector<double>& out) {
  std::vector<double> a(psi);                    // reduced in place
  std::vector<double> vs((size_t)n * m, 0.0);    // reflector k in row k (entries k..m-1)
  std::vector<double> beta(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double nrm = 0.0;
    for (int p = k; p < m; ++p) nrm += a[(size_t)p * n + k] * a[(size_t)p * n + k];
    nrm = std::sqrt(nrm);
    const double x0 = a[(size_t)k * n + k];
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    double* v = &vs[(size_t)k * m];
    for (int p = k; p < m; ++p) v[p] = a[(size_t)p * n + k];
    v[k] -= alpha;
    double vv = 0.0;
    for (int p = k; p < m; ++p) vv += v[p] * v[p];
    beta[k] = vv > 0.0 ? 2.0 / vv : 0.0;
    for (int c = k; c < n; ++c) {   // apply H_k = I - beta v v^T to the remaining columns
      double s = 0.0;
      for (int p = k; p < m; ++p) s += v[p] * a[(size_t)p * n + c];
      s *= beta[k];
      for (int p = k; p < m; ++p) a[(size_t)p * n + c] -= s * v[p];
    }
  }
  out.assign((size_t)(m - n) * m, 0.0);
  std::vector<double> q(m);
  for (int c = n; c < m; ++c) {
    for (int p = 0; p < m; ++p) q[p] = p == c ? 1.0 : 0.0;
    for (int k = n - 1; k >= 0; --k) {
      const double* v = &vs[(size_t)k * m];
      double s = 0.0;
      for (int p = k; p < m; ++p) s += v[p] * q[p];
      s *= beta[k];
      for (int p = k; p < m; ++p) q[p] -= s * v[p];
    }
    for (int p = 0; p < m; ++p) out[(size_t)(c - n) * m + p] = q[p];
  }
}

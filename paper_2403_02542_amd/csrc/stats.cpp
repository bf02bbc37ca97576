// Statistics of the per-step estimates of a run (host code; the series are
// a few thousand scalars): the weighted time average and variance of
// Sec. II.A, the correlation length kappa of Eq. (variance), and the
// time-step extrapolation fits of Sec. V.G with the error of Eq. (staterr).
//
// kappa has two estimators, both from the literature (the paper defines
// kappa but names none): the integrated autocorrelation time with Sokal's
// self-consistent window, and the blocking transformation of Flyvbjerg and
// Petersen with the optimal level of Lee, Needs, Drummond and Towler.
#include <cmath>
#include <cstdint>
#include <vector>

#include "afq.h"

namespace {

bool finite_all(const double* x, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// Mean-removed autocovariance C(t) = (1 / (n - t)) sum_i d_i d_{i+t}.
double autocov(const std::vector<double>& d, int64_t t) {
  const int64_t n = (int64_t)d.size();
  double s = 0.0;
  for (int64_t i = 0; i + t < n; ++i) s += d[i] * d[i + t];
  return s / (double)(n - t);
}

struct Level {
  double n, se, se_err;
};

std::vector<Level> block_levels(const double* e, int64_t n) {
  std::vector<double> x(e, e + n);
  std::vector<Level> out;
  while (x.size() >= 2) {
    const int64_t m = (int64_t)x.size();
    double mean = 0.0;
    for (double v : x) mean += v;
    mean /= (double)m;
    double ss = 0.0;
    for (double v : x) ss += (v - mean) * (v - mean);
    const double se = std::sqrt(ss / ((double)m * (double)(m - 1)));
    out.push_back(Level{(double)m, se, se / std::sqrt(2.0 * (double)(m - 1))});
    std::vector<double> y((size_t)(m / 2));
    for (int64_t i = 0; i < m / 2; ++i) y[i] = 0.5 * (x[2 * i] + x[2 * i + 1]);
    x.swap(y);
  }
  return out;
}

// Solve the k x k symmetric positive system S x = b in place (Gauss-Jordan
// with partial pivoting), returning S^-1 in inv; false if singular.
bool solve_small(int k, double* S, double* inv) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) inv[i * k + j] = i == j ? 1.0 : 0.0;
  for (int c = 0; c < k; ++c) {
    int p = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(S[r * k + c]) > std::fabs(S[p * k + c])) p = r;
    if (S[p * k + c] == 0.0) return false;
    if (p != c)
      for (int j = 0; j < k; ++j) {
        std::swap(S[p * k + j], S[c * k + j]);
        std::swap(inv[p * k + j], inv[c * k + j]);
      }
    const double d = S[c * k + c];
    for (int j = 0; j < k; ++j) {
      S[c * k + j] /= d;
      inv[c * k + j] /= d;
    }
    for (int r = 0; r < k; ++r) {
      if (r == c) continue;
      const double f = S[r * k + c];
      for (int j = 0; j < k; ++j) {
        S[r * k + j] -= f * S[c * k + j];
        inv[r * k + j] -= f * inv[c * k + j];
      }
    }
  }
  return true;
}

}  // namespace

extern "C" {

afq_status afq_stats_time_average(const double* w, const double* e, int64_t n, int64_t n_eq,
                                  double* out) {
  if (!w || !e || !out || n < 0 || n_eq < 0) return AFQ_EINVAL;
  double num = 0.0, num2 = 0.0, den = 0.0;
  int64_t used = 0;
  for (int64_t k = n_eq; k < n; ++k) {
    num += w[k] * e[k];
    num2 += w[k] * e[k] * e[k];
    den += w[k];
    ++used;
  }
  out[2] = (double)used;
  if (used == 0 || den == 0.0) {
    out[0] = out[1] = NAN;
    return AFQ_OK;
  }
  const double mean = num / den;
  out[0] = mean;
  out[1] = num2 / den - mean * mean;
  return AFQ_OK;
}

afq_status afq_stats_blocking(const double* e, int64_t n, double* levels, int32_t max_levels,
                              int32_t* n_levels) {
  if (!e || !levels || !n_levels || n < 2 || max_levels < 1) return AFQ_EINVAL;
  if (!finite_all(e, n)) return AFQ_EINVAL;
  const std::vector<Level> lv = block_levels(e, n);
  const int32_t m = (int32_t)lv.size() < max_levels ? (int32_t)lv.size() : max_levels;
  for (int32_t l = 0; l < m; ++l) {
    levels[3 * l] = lv[l].n;
    levels[3 * l + 1] = lv[l].se;
    levels[3 * l + 2] = lv[l].se_err;
  }
  *n_levels = (int32_t)lv.size();
  return AFQ_OK;
}

afq_status afq_stats_kappa(const double* e, int64_t n, double c, double* out) {
  if (!e || !out || n < 2 || !(c > 0.0)) return AFQ_EINVAL;
  if (!finite_all(e, n)) return AFQ_EINVAL;
  double mean = 0.0;
  for (int64_t i = 0; i < n; ++i) mean += e[i];
  mean /= (double)n;
  std::vector<double> d((size_t)n);
  for (int64_t i = 0; i < n; ++i) d[i] = e[i] - mean;
  const double c0 = autocov(d, 0);
  // integrated autocorrelation time, window M >= c kappa(M)
  double kappa = 1.0;
  int64_t window = n - 1;
  if (c0 > 0.0) {
    for (int64_t m = 1; m < n; ++m) {
      kappa += 2.0 * autocov(d, m) / c0;
      if ((double)m >= c * kappa) {
        window = m;
        break;
      }
    }
  }
  out[0] = kappa;
  out[1] = (double)window;
  // blocking: the smallest level with (2^l)^3 > 2 n_0 (se_l / se_0)^4
  const std::vector<Level> lv = block_levels(e, n);
  int best = (int)lv.size() - 1;
  const double se0 = lv[0].se;
  for (int l = 0; l < (int)lv.size(); ++l) {
    const double r = se0 > 0.0 ? lv[l].se / se0 : 1.0;
    if (std::pow(2.0, 3.0 * l) > 2.0 * lv[0].n * r * r * r * r) {
      best = l;
      break;
    }
  }
  const double r = se0 > 0.0 ? lv[best].se / se0 : 1.0;
  out[2] = r * r;
  out[3] = (double)best;
  return AFQ_OK;
}

afq_status afq_tau_fit(const double* tau, const double* e, const double* sigma, int32_t n,
                       int32_t form, double* coef, double* err) {
  if (!tau || !e || !coef || !err || form < AFQ_FIT_QUADRATIC || form > AFQ_FIT_LINEAR)
    return AFQ_EINVAL;
  int pw[3], k = 0;
  pw[k++] = 0;
  if (form != AFQ_FIT_PURE_SQUARE) pw[k++] = 1;
  if (form != AFQ_FIT_LINEAR) pw[k++] = 2;
  if (n < k) return AFQ_EINVAL;
  double S[9] = {0}, b[3] = {0}, inv[9];
  for (int32_t i = 0; i < n; ++i) {
    const double s = sigma ? sigma[i] : 1.0;
    if (!(s > 0.0) || !std::isfinite(tau[i]) || !std::isfinite(e[i])) return AFQ_EINVAL;
    const double wgt = 1.0 / (s * s);
    double a[3];
    for (int j = 0; j < k; ++j) a[j] = std::pow(tau[i], (double)pw[j]);
    for (int r = 0; r < k; ++r) {
      b[r] += wgt * a[r] * e[i];
      for (int c = 0; c < k; ++c) S[r * k + c] += wgt * a[r] * a[c];
    }
  }
  if (!solve_small(k, S, inv)) return AFQ_ENUMERIC;
  coef[0] = coef[1] = coef[2] = 0.0;
  for (int r = 0; r < k; ++r) {
    double x = 0.0;
    for (int c = 0; c < k; ++c) x += inv[r * k + c] * b[c];
    coef[pw[r]] = x;
  }
  err[0] = std::sqrt(inv[0]);
  // Eq. (staterr): sqrt(sum sigma_i^2) / N_tau (NaN without sigmas)
  if (sigma) {
    double ss = 0.0;
    for (int32_t i = 0; i < n; ++i) ss += sigma[i] * sigma[i];
    err[1] = std::sqrt(ss) / (double)n;
  } else {
    err[1] = NAN;
  }
  return AFQ_OK;
}

}  // extern "C"

// Host-side coefficient fit: Algorithm 2 (Sec. 3) of the paper, float64.
//
// The range kernel is sampled on {0..T}; the cosine columns cos(n w t),
// w = pi / T, are appended one at a time (n = 0, 1, 2, ...).  Each new column
// is orthogonalised against the previous ones by modified Gram-Schmidt, which
// appends one column to Q and one column to the upper-triangular R; the
// coefficients follow from R d = Q^T b by back-substitution and the loop ends
// once ||b - A d||_2 <= eps (eq. (7)/(8)), or when the cap K_max is reached.
#include <cmath>
#include <vector>

#include "bf_internal.h"

namespace bf {

int sample_range_kernel(bf_range_kind kind, double sigma_r, const double* table, int T,
                        std::vector<double>& b) {
  b.assign(static_cast<size_t>(T) + 1, 0.0);
  for (int t = 0; t <= T; ++t) {
    const double x = static_cast<double>(t);
    switch (kind) {
      case BF_RANGE_GAUSSIAN: b[t] = std::exp(-x * x / (2.0 * sigma_r * sigma_r)); break;
      case BF_RANGE_EXPONENTIAL: b[t] = std::exp(-x / sigma_r); break;
      case BF_RANGE_TABLE: b[t] = table[t]; break;
      default: return BF_E_INVALID;
    }
  }
  return BF_OK;
}

FitOutcome fit_cosine_series(const std::vector<double>& b, int T, double eps, int K_max) {
  const int n = T + 1;
  const double omega = M_PI / static_cast<double>(T);
  FitOutcome out;
  // columns of Q and of the basis A, stored column by column
  std::vector<std::vector<double>> Q, A;
  // R stored by columns: Rcol[j] holds R(0..j, j)
  std::vector<std::vector<double>> Rcol;
  std::vector<double> qtb;  // Q^T b
  std::vector<double> d;

  auto residual = [&](const std::vector<double>& coef, double* l2, double* mx) {
    double s = 0.0, m = 0.0;
    for (int t = 0; t < n; ++t) {
      double approx = 0.0;
      for (size_t j = 0; j < coef.size(); ++j) approx += coef[j] * A[j][t];
      const double e = b[t] - approx;
      s += e * e;
      m = std::max(m, std::fabs(e));
    }
    *l2 = std::sqrt(s);
    *mx = m;
  };

  for (int harmonic = 0; harmonic <= K_max; ++harmonic) {
    std::vector<double> a(n);
    for (int t = 0; t < n; ++t) a[t] = std::cos(static_cast<double>(harmonic) * omega * t);
    A.push_back(a);
    std::vector<double> r(static_cast<size_t>(harmonic) + 1, 0.0);
    for (int j = 0; j < harmonic; ++j) {  // modified Gram-Schmidt: project the updated vector
      double dot = 0.0;
      for (int t = 0; t < n; ++t) dot += a[t] * Q[j][t];
      r[j] = dot;
      for (int t = 0; t < n; ++t) a[t] -= dot * Q[j][t];
    }
    double nrm = 0.0;
    for (int t = 0; t < n; ++t) nrm += a[t] * a[t];
    nrm = std::sqrt(nrm);
    r[harmonic] = nrm;
    for (int t = 0; t < n; ++t) a[t] /= nrm;
    Q.push_back(a);
    Rcol.push_back(r);
    double pb = 0.0;
    for (int t = 0; t < n; ++t) pb += a[t] * b[t];
    qtb.push_back(pb);
    // back-substitution R d = Q^T b
    const int m = harmonic + 1;
    d.assign(m, 0.0);
    for (int i = m - 1; i >= 0; --i) {
      double s = qtb[i];
      for (int j = i + 1; j < m; ++j) s -= Rcol[j][i] * d[j];
      d[i] = s / Rcol[i][i];
    }
    residual(d, &out.err_l2, &out.err_max);
    out.K = harmonic;
    out.d = d;
    if (out.err_l2 <= eps) {
      out.converged = true;
      return out;
    }
  }
  out.converged = false;
  return out;
}

}  // namespace bf

// Dense symmetric eigensolver in FP64 for the k x k Gram matrix of the learned
// convolution eigenvectors (Definition 3, eq:A).
//
// Householder reduction to tridiagonal form followed by the implicit symmetric
// QR iteration with Wilkinson shifts, accumulating all transformations
// (Golub & Van Loan, Matrix Computations, Sections 8.3.1 and 8.3.3).
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <stdexcept>
#include <vector>

namespace icnnm {

// A: n x n row-major symmetric, destroyed. On return w holds the eigenvalues in
// descending order and V (row-major, n x n) the matching orthonormal
// eigenvectors as columns, each with its largest-magnitude entry positive.
void sym_eig(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V) {
  if ((int64_t)A.size() != (int64_t)n * n) throw std::invalid_argument("sym_eig: bad size");
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  std::vector<double> d(n), e(std::max(n - 1, 0), 0.0);
  std::vector<std::vector<double>> hv;  // Householder vectors (length n-k-1)
  std::vector<double> hb;
  std::vector<double> p(n), wv(n);

  // --- tridiagonalisation: A <- H_k A H_k, k = 0..n-3
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    double nx = 0.0;
    for (int i = 0; i < len; ++i) nx += a(k + 1 + i, k) * a(k + 1 + i, k);
    nx = std::sqrt(nx);
    std::vector<double> v(len);
    double beta = 0.0;
    if (nx > 0.0) {
      const double x0 = a(k + 1, k);
      const double alpha = x0 >= 0 ? -nx : nx;
      for (int i = 0; i < len; ++i) v[i] = a(k + 1 + i, k);
      v[0] -= alpha;
      double vn = 0.0;
      for (int i = 0; i < len; ++i) vn += v[i] * v[i];
      if (vn > 0.0) {
        beta = 2.0 / vn;
        // p = beta * A22 v
        for (int i = 0; i < len; ++i) {
          double s = 0.0;
          const double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
          for (int j = 0; j < len; ++j) s += row[j] * v[j];
          p[i] = beta * s;
        }
        double pv = 0.0;
        for (int i = 0; i < len; ++i) pv += p[i] * v[i];
        const double h = 0.5 * beta * pv;
        for (int i = 0; i < len; ++i) wv[i] = p[i] - h * v[i];
        // A22 -= v w^T + w v^T
        for (int i = 0; i < len; ++i) {
          double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
          const double vi = v[i], wi = wv[i];
          for (int j = 0; j < len; ++j) row[j] -= vi * wv[j] + wi * v[j];
        }
        a(k + 1, k) = alpha;
        a(k, k + 1) = alpha;
        for (int i = 1; i < len; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
      }
    }
    hv.push_back(std::move(v));
    hb.push_back(beta);
  }
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);

  // --- Q = H_0 H_1 ... H_{n-3}, accumulated backwards
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int k = (int)hv.size() - 1; k >= 0; --k) {
    const double beta = hb[k];
    if (beta == 0.0) continue;
    const std::vector<double>& v = hv[k];
    const int len = n - k - 1;
    // Q[k+1:, k+1:] = (I - beta v v^T) Q[k+1:, k+1:]
    std::vector<double> t(len, 0.0);
    for (int i = 0; i < len; ++i) {
      const double* row = &Q[(size_t)(k + 1 + i) * n + (k + 1)];
      const double vi = v[i];
      for (int j = 0; j < len; ++j) t[j] += vi * row[j];
    }
    for (int i = 0; i < len; ++i) {
      double* row = &Q[(size_t)(k + 1 + i) * n + (k + 1)];
      const double f = beta * v[i];
      for (int j = 0; j < len; ++j) row[j] -= f * t[j];
    }
  }

  // columns of Q as contiguous rows for the rotations below
  std::vector<double> Qt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Qt[(size_t)j * n + i] = Q[(size_t)i * n + j];
  Q.clear();
  Q.shrink_to_fit();

  // --- implicit symmetric QR with Wilkinson shift on (d, e); rotate columns of Q
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1;
  int guard = 0;
  while (hi > 0) {
    int lo = hi;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    if (lo == hi) {
      if (hi > 0) e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    if (++guard > 60 * n) throw std::runtime_error("sym_eig: QR iteration did not converge");
    // shift from the trailing 2x2 block of [lo..hi]
    const double dd = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double den = dd + (dd >= 0 ? 1.0 : -1.0) * std::hypot(dd, eh);
    const double mu = den != 0.0 ? d[hi] - eh * eh / den : d[hi];
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = r != 0.0 ? x / r : 1.0;
      const double s = r != 0.0 ? z / r : 0.0;
      if (k > lo) e[k - 1] = r;
      const double ak = d[k], bk = e[k], ck = d[k + 1];
      d[k] = c * c * ak + 2.0 * c * s * bk + s * s * ck;
      d[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ck;
      e[k] = c * s * (ck - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        z = s * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      double* qk = &Qt[(size_t)k * n];
      double* qk1 = &Qt[(size_t)(k + 1) * n];
      for (int i = 0; i < n; ++i) {
        const double qa = qk[i], qb = qk1[i];
        qk[i] = c * qa + s * qb;
        qk1[i] = -s * qa + c * qb;
      }
    }
  }

  // --- sort descending, normalise signs
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return d[i] > d[j]; });
  w.assign(n, 0.0);
  V.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    const int src = idx[c];
    w[c] = d[src];
    int arg = 0;
    double best = -1.0;
    for (int i = 0; i < n; ++i) {
      const double v = std::fabs(Qt[(size_t)src * n + i]);
      if (v > best) {
        best = v;
        arg = i;
      }
    }
    const double sg = Qt[(size_t)src * n + arg] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) V[(size_t)i * n + c] = sg * Qt[(size_t)src * n + i];
  }
}

}  // namespace icnnm

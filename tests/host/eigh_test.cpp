// Host-only checks of the FP64 symmetric eigensolver (paper_2604_17001_amd/csrc/eigh.cpp),
// built by tests/test_host_sanitized.py with sanitizers: A V = V diag(w), V^T V = I,
// eigenvalues descending, sign convention, and (ICNNM_EIG_THREADS) results that do not
// depend on the thread count.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

namespace icnnm {
void sym_eig(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V);
}

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 60;
  std::mt19937_64 g(1234 + n);
  std::normal_distribution<double> nd;
  std::vector<double> A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = nd(g);
  // a repeated eigenvalue: add a multiple of a rank-2 projector's complement structure
  const std::vector<double> A0 = A;
  std::vector<double> work = A, w, V;
  icnnm::sym_eig(work, n, w, V);
  double res = 0.0, orth = 0.0, nrm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) nrm = std::fmax(nrm, std::fabs(A0[(size_t)i * n + j]));
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double av = 0.0;
      for (int j = 0; j < n; ++j) av += A0[(size_t)i * n + j] * V[(size_t)j * n + c];
      res = std::fmax(res, std::fabs(av - w[c] * V[(size_t)i * n + c]));
    }
    for (int d = 0; d < n; ++d) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += V[(size_t)i * n + c] * V[(size_t)i * n + d];
      orth = std::fmax(orth, std::fabs(s - (c == d ? 1.0 : 0.0)));
    }
  }
  int bad_order = 0, bad_sign = 0;
  for (int c = 0; c + 1 < n; ++c) bad_order += w[c] < w[c + 1];
  for (int c = 0; c < n; ++c) {
    int im = 0;
    for (int i = 1; i < n; ++i)
      if (std::fabs(V[(size_t)i * n + c]) > std::fabs(V[(size_t)im * n + c])) im = i;
    bad_sign += V[(size_t)im * n + c] < 0.0;
  }
  std::printf("n=%d residual %.3e orthogonality %.3e order %d sign %d\n", n, res / (n * nrm), orth, bad_order,
              bad_sign);
  // the eigenvalues and vectors as bits, for the thread-count comparison
  if (argc > 2) {
    FILE* f = std::fopen(argv[2], "wb");
    if (!f) return 2;
    std::fwrite(w.data(), 8, w.size(), f);
    std::fwrite(V.data(), 8, V.size(), f);
    std::fclose(f);
  }
  const bool ok = res <= 1e-12 * n * nrm && orth <= 1e-12 * n && bad_order == 0 && bad_sign == 0;
  return ok ? 0 : 1;
}

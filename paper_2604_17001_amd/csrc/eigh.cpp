// Dense symmetric eigensolver in FP64 for the k x k Gram matrix of the learned
// convolution eigenvectors (Definition 3, eq:A).
//
// Householder reduction to tridiagonal form followed by the implicit symmetric
// QR iteration with Wilkinson shifts, accumulating all transformations
// (Golub & Van Loan, Matrix Computations, Sections 8.3.1 and 8.3.3).
//
// The O(n^3) loops run on host threads: the matrix-vector products and rank
// updates of the reduction split over rows (or over columns where a sum runs over
// rows), and each QR sweep's rotations are applied to column blocks of the
// accumulated basis. Every output element is computed by one thread in the serial
// order, so the result does not depend on the thread count.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <functional>
#include <limits>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <thread>
#include <vector>

namespace icnnm {

namespace {

// Fixed set of worker threads running parallel_for over [0, n) in contiguous blocks.
class Pool {
 public:
  // split_all: split every range over the threads, however small (a forced thread
  // count, to run the threaded path on small matrices)
  explicit Pool(int nt, bool split_all = false) : split_all_(split_all) {
    for (int t = 1; t < nt; ++t) th_.emplace_back([this, t] { work(t); });
    nt_ = nt;
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  // fn(begin, end) on blocks of [0, n), each with at least ~256K operations of work
  // (item_cost operations per index) to amortise the hand-off; small ranges run inline
  void parallel_for(int n, const std::function<void(int, int)>& fn, int64_t item_cost) {
    const int64_t per = split_all_ ? 1 : std::max<int64_t>(1, (int64_t(1) << 18) / std::max<int64_t>(1, item_cost));
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(nt_, n / per));
    if (nt == 1) {
      fn(0, n);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      active_ = nt;
      pending_ = nt - 1;
      ++gen_;
    }
    cv_.notify_all();
    run_block(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return pending_ == 0; });
  }

 private:
  void run_block(int t) {
    const int b = (int)((int64_t)n_ * t / active_), e = (int)((int64_t)n_ * (t + 1) / active_);
    if (b < e) (*fn_)(b, e);
  }
  void work(int t) {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return gen_ != seen; });
      seen = gen_;
      if (stop_) return;
      if (t >= active_) continue;
      lk.unlock();
      run_block(t);
      lk.lock();
      if (--pending_ == 0) done_.notify_one();
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int, int)>* fn_ = nullptr;
  int n_ = 0, active_ = 1, pending_ = 0, nt_ = 1;
  uint64_t gen_ = 0;
  bool stop_ = false;
  bool split_all_ = false;
};

// threads for an n x n problem: below ~1500 the hand-off cost outweighs the gain;
// ICNNM_EIG_THREADS=t forces t threads (runs the threaded path on small matrices)
int pool_threads(int n) {
  if (const char* e = std::getenv("ICNNM_EIG_THREADS")) return std::max(1, std::min(std::atoi(e), 64));
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  return n < 1500 ? 1 : std::min(hw, 16);
}

}  // namespace

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
  Pool pool(pool_threads(n), std::getenv("ICNNM_EIG_THREADS") != nullptr);

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
        pool.parallel_for(len, [&](int i0, int i1) {
          for (int i = i0; i < i1; ++i) {
            double s = 0.0;
            const double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
            for (int j = 0; j < len; ++j) s += row[j] * v[j];
            p[i] = beta * s;
          }
        }, len);
        double pv = 0.0;
        for (int i = 0; i < len; ++i) pv += p[i] * v[i];
        const double h = 0.5 * beta * pv;
        for (int i = 0; i < len; ++i) wv[i] = p[i] - h * v[i];
        // A22 -= v w^T + w v^T
        pool.parallel_for(len, [&](int i0, int i1) {
          for (int i = i0; i < i1; ++i) {
            double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
            const double vi = v[i], wi = wv[i];
            for (int j = 0; j < len; ++j) row[j] -= vi * wv[j] + wi * v[j];
          }
        }, 2 * len);
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
    // Q[k+1:, k+1:] = (I - beta v v^T) Q[k+1:, k+1:]; t = v^T Q22 sums over rows,
    // so it splits over columns
    std::vector<double> t(len, 0.0);
    pool.parallel_for(len, [&](int j0, int j1) {
      for (int i = 0; i < len; ++i) {
        const double* row = &Q[(size_t)(k + 1 + i) * n + (k + 1)];
        const double vi = v[i];
        for (int j = j0; j < j1; ++j) t[j] += vi * row[j];
      }
    }, len);
    pool.parallel_for(len, [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        double* row = &Q[(size_t)(k + 1 + i) * n + (k + 1)];
        const double f = beta * v[i];
        for (int j = 0; j < len; ++j) row[j] -= f * t[j];
      }
    }, len);
  }

  // columns of Q as contiguous rows for the rotations below
  std::vector<double> Qt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Qt[(size_t)j * n + i] = Q[(size_t)i * n + j];
  Q.clear();
  Q.shrink_to_fit();

  // --- implicit symmetric QR with Wilkinson shift on (d, e); rotate columns of Q
  const double eps = std::numeric_limits<double>::epsilon();
  std::vector<double> rc, rs;  // rotations of one sweep
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
    rc.clear();
    rs.clear();
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
      rc.push_back(c);
      rs.push_back(s);
    }
    // the sweep's rotations, in order, on column blocks of the basis
    pool.parallel_for(n, [&](int i0, int i1) {
      for (int k = lo; k < hi; ++k) {
        const double c = rc[k - lo], s = rs[k - lo];
        double* qk = &Qt[(size_t)k * n];
        double* qk1 = &Qt[(size_t)(k + 1) * n];
        for (int i = i0; i < i1; ++i) {
          const double qa = qk[i], qb = qk1[i];
          qk[i] = c * qa + s * qb;
          qk1[i] = -s * qa + c * qb;
        }
      }
    }, 6 * (hi - lo));
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

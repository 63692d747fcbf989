// Symmetric eigensolver on the device, in FP64, for the k x k Gram matrix of the
// learned convolution eigenvectors (Definition 3, eq:A): the cyclic Jacobi method
// with the round-robin parallel ordering (Golub & Van Loan, Matrix Computations,
// Sections 8.5.2 and 8.5.4, "parallel Jacobi").
//
// An even order n is split into n/2 disjoint index pairs; one round rotates every
// pair at once, B = J^T A J with J the product of the n/2 plane rotations, each
// chosen to annihilate its pair's off-diagonal entry, and accumulates V <- V J. The
// n - 1 rounds of a sweep meet every pair of indices once. The matrix is kept with
// the two members of pair i at positions 2i and 2i + 1, so every 2 x 2 block of
// B = J^T A J depends on one 2 x 2 block of A and two rotations only; a round is one
// pass over A and V. Between rounds the positions move along the round-robin circle
// (position 0 fixed, the others shifted by one place), applied as the blocks are
// written to the other buffer. A sweep is repeated until the off-diagonal Frobenius
// norm falls below a tolerance; the diagonal then holds the eigenvalues and the
// columns of V the eigenvectors (rows of V keep the original index order).
#include "icnnm_dev.h"

namespace icnnm {

constexpr int kThreadsJac = 256;

// position of x after one round, on the circle 2, 4, .., 2h - 2, 2h - 1, 2h - 3, .., 1
// (the tops of pairs 1..h-1, then the bottoms of pairs h-1..0), position 0 fixed
__device__ __forceinline__ int jac_next(int x, int h) {
  if (x == 0 || h == 1) return x;
  const int i = x >> 1;
  if ((x & 1) == 0) return i + 1 < h ? 2 * (i + 1) : 2 * i + 1;  // top of pair i
  return i > 0 ? 2 * (i - 1) + 1 : 2;                            // bottom of pair i
}

// rotation (c, s) of pair i annihilating A[2i][2i+1], and t = s / c
__device__ __forceinline__ void jac_rot_of(const double* A, int n, int i, double& c, double& s, double& t) {
  const double app = A[(size_t)(2 * i) * n + 2 * i];
  const double aqq = A[(size_t)(2 * i + 1) * n + 2 * i + 1];
  const double apq = A[(size_t)(2 * i) * n + 2 * i + 1];
  c = 1.0;
  s = 0.0;
  t = 0.0;
  if (apq == 0.0 || fabs(apq) <= 1e-300) return;
  const double theta = (aqq - app) / (2.0 * apq);
  const double at = fabs(theta);
  t = at > 1e150 ? 0.5 / theta : (theta >= 0.0 ? 1.0 : -1.0) / (at + sqrt(at * at + 1.0));
  c = 1.0 / sqrt(t * t + 1.0);
  s = t * c;
}

// the rotations of one round, rot[i] = (c, s, t) of pair i
__global__ __launch_bounds__(kThreadsJac) void k_jacobi_rot(const double* A, int n, double* rot) {
  const int h = n / 2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < h; i += gridDim.x * blockDim.x) {
    double c, s, t;
    jac_rot_of(A, n, i, c, s, t);
    rot[3 * i] = c;
    rot[3 * i + 1] = s;
    rot[3 * i + 2] = t;
  }
}

__device__ __forceinline__ void jac_rot(const double* rot, int i, double& c, double& s, double& t) {
  c = rot[3 * i];
  s = rot[3 * i + 1];
  t = rot[3 * i + 2];
}

// One round: B = J^T A J and W = V J, both written at the next round's positions.
// Items 0 .. h*h - 1 are the 2 x 2 blocks (a, b) of A (b fastest); items h*h .. are
// the (row r, pair b) pieces of V.
__global__ __launch_bounds__(kThreadsJac) void k_jacobi_round(const double* A, double* B, const double* V,
                                                               double* W, int n, const double* rot) {
  const int h = n / 2;
  const int64_t na = (int64_t)h * h, nv = (int64_t)n * h;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < na + nv;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < na) {
      const int a = (int)(e / h), b = (int)(e - (int64_t)a * h);
      double ca, sa, ta, cb, sb, tb;
      jac_rot(rot, a, ca, sa, ta);
      jac_rot(rot, b, cb, sb, tb);
      const double2 r0 = *reinterpret_cast<const double2*>(A + (size_t)(2 * a) * n + 2 * b);
      const double2 r1 = *reinterpret_cast<const double2*>(A + (size_t)(2 * a + 1) * n + 2 * b);
      double y00, y01, y10, y11;
      if (a == b) {
        // the pair's own block: diagonal update, annihilated off-diagonal entry
        y00 = r0.x - ta * r0.y;
        y11 = r1.y + ta * r0.y;
        y01 = y10 = 0.0;
      } else {
        const double x00 = ca * r0.x - sa * r1.x, x01 = ca * r0.y - sa * r1.y;
        const double x10 = sa * r0.x + ca * r1.x, x11 = sa * r0.y + ca * r1.y;
        y00 = cb * x00 - sb * x01;
        y01 = sb * x00 + cb * x01;
        y10 = cb * x10 - sb * x11;
        y11 = sb * x10 + cb * x11;
      }
      const int p0 = jac_next(2 * a, h), p1 = jac_next(2 * a + 1, h);
      const int q0 = jac_next(2 * b, h), q1 = jac_next(2 * b + 1, h);
      B[(size_t)p0 * n + q0] = y00;
      B[(size_t)p0 * n + q1] = y01;
      B[(size_t)p1 * n + q0] = y10;
      B[(size_t)p1 * n + q1] = y11;
    } else {
      const int64_t f = e - na;
      const int r = (int)(f / h), b = (int)(f - (int64_t)r * h);
      double cb, sb, tb;
      jac_rot(rot, b, cb, sb, tb);
      const double2 v = *reinterpret_cast<const double2*>(V + (size_t)r * n + 2 * b);
      W[(size_t)r * n + jac_next(2 * b, h)] = cb * v.x - sb * v.y;
      W[(size_t)r * n + jac_next(2 * b + 1, h)] = sb * v.x + cb * v.y;
    }
  }
}

// Sums of squares of the off-diagonal entries and of all entries of A: block b sums
// rows b, b + nb, .. into part[2b], part[2b + 1]; k_jacobi_offnorm_finish adds the nb
// partials in block order into out[0], out[1]. Fixed order throughout.
constexpr int kOffBlocks = 256;
__global__ __launch_bounds__(kThreadsJac) void k_jacobi_offnorm(const double* A, int n, double* part) {
  double off = 0.0, all = 0.0;
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const double* row = A + (size_t)r * n;
    for (int c = threadIdx.x; c < n; c += kThreadsJac) {
      const double v = row[c];
      all += v * v;
      off += c != r ? v * v : 0.0;
    }
  }
  __shared__ double r0[kThreadsJac], r1[kThreadsJac];
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = all;
  __syncthreads();
  for (int o = kThreadsJac / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ void k_jacobi_offnorm_finish(const double* part, int nb, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double off = 0.0, all = 0.0;
    for (int b = 0; b < nb; ++b) {
      off += part[2 * b];
      all += part[2 * b + 1];
    }
    out[0] = off;
    out[1] = all;
  }
}

// A (n x n) <- G (k x k) with a zero row and column appended when n = k + 1; V <- I
__global__ void k_jacobi_init(const double* G, int k, double* A, double* V, int n) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    A[e] = (i < k && j < k) ? G[(size_t)i * k + j] : 0.0;
    V[e] = i == j ? 1.0 : 0.0;
  }
}

static inline int grid_for_jac(int64_t n) {
  const int64_t g = (n + kThreadsJac - 1) / kThreadsJac;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

void launch_jacobi_init(const double* G, int k, double* A, double* V, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_init, dim3(grid_for_jac((int64_t)n * n)), dim3(kThreadsJac), 0, st, G, k, A, V, n);
}

void launch_jacobi_round(const double* A, double* B, const double* V, double* W, int n, double* rot,
                         hipStream_t st) {
  const int64_t h = n / 2;
  hipLaunchKernelGGL(k_jacobi_rot, dim3(grid_for_jac(h)), dim3(kThreadsJac), 0, st, A, n, rot);
  hipLaunchKernelGGL(k_jacobi_round, dim3(grid_for_jac(h * h + (int64_t)n * h)), dim3(kThreadsJac), 0, st, A, B, V,
                     W, n, (const double*)rot);
}

void launch_jacobi_offnorm(const double* A, int n, double* part, double* out, hipStream_t st) {
  const int nb = n < kOffBlocks ? (n > 0 ? n : 1) : kOffBlocks;
  hipLaunchKernelGGL(k_jacobi_offnorm, dim3(nb), dim3(kThreadsJac), 0, st, A, n, part);
  hipLaunchKernelGGL(k_jacobi_offnorm_finish, dim3(1), dim3(64), 0, st, (const double*)part, nb, out);
}

}  // namespace icnnm

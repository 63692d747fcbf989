// FP64 kernels of the diagnostics entry point (Definition 2, eq:rkL0, eq:alphaK):
// C = V^T G V for the Gram G = A_k(L0)^T A_k(L0) of a tensor. Kept apart from the
// solver kernels; the Gram itself comes from the learning kernels (k_autocorr_tiled,
// k_gram_expand).
#include "icnnm_dev.h"

namespace icnnm {

constexpr int kThreadsDiag = 256;

// C = op(A) B in FP64 for n x n row-major matrices (op(A) = A^T when trans_a), 16 x 16
// output tiles staged through LDS; every output is one fixed-order sum. At most a few
// GFLOP per call (k <= 4096).
constexpr int kGemmTile = 16;
__global__ __launch_bounds__(kGemmTile * kGemmTile) void k_gemm_f64(const double* A, int trans_a,
                                                                    const double* B, double* C, int n) {
  __shared__ double As[kGemmTile][kGemmTile + 1], Bs[kGemmTile][kGemmTile + 1];
  const int tx = threadIdx.x % kGemmTile, ty = threadIdx.x / kGemmTile;
  const int row = blockIdx.y * kGemmTile + ty, col = blockIdx.x * kGemmTile + tx;
  double acc = 0.0;
  for (int l0 = 0; l0 < n; l0 += kGemmTile) {
    const int la = l0 + tx, lb = l0 + ty;
    double av = 0.0, bv = 0.0;
    if (row < n && la < n) av = trans_a ? A[(size_t)la * n + row] : A[(size_t)row * n + la];
    if (lb < n && col < n) bv = B[(size_t)lb * n + col];
    As[ty][tx] = av;
    Bs[ty][tx] = bv;
    __syncthreads();
#pragma unroll
    for (int l = 0; l < kGemmTile; ++l) acc = fma(As[ty][l], Bs[l][tx], acc);
    __syncthreads();
  }
  if (row < n && col < n) C[(size_t)row * n + col] = acc;
}

static inline int grid_for_diag(int64_t n) {
  const int64_t g = (n + kThreadsDiag - 1) / kThreadsDiag;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

__global__ void k_f32_to_f64(const float* src, double* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

void launch_gemm_f64(const double* A, int trans_a, const double* B, double* C, int n, hipStream_t st) {
  const int nb = (n + kGemmTile - 1) / kGemmTile;
  hipLaunchKernelGGL(k_gemm_f64, dim3(nb, nb), dim3(kGemmTile * kGemmTile), 0, st, A, trans_a, B, C, n);
}

void launch_f32_to_f64(const float* src, double* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for_diag(n)), dim3(kThreadsDiag), 0, st, src, dst, n);
}

}  // namespace icnnm

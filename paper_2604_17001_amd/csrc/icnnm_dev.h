// Device-side data structures shared by the ICNNM kernels and the host runtime.
//
// One ADMM iteration (Section III-D) runs as four stage kernels over a table
// of spatial tiles that may span many instances:
//   colnorm : FP64 column norms of Q = W - U -> shrink factors s_i (Z-step), penalty
//             schedule, stopping residuals of the previous iteration
//   adjoint : G = U + s.Q (scaled Y + theta Z), H = G V^T on MFMA, col2im of H
//             into an LDS box (transposed convolutions summed back)
//   lstep   : sums the halo partials of neighbouring tiles, applies the L-step
//             with P_Omega data consistency
//   forward : W = A_k(L) V as an implicit-im2col MFMA contraction from an LDS
//             halo of L, fused with the dual update, next Q and column partials
// Each instance carries a phase so that instances at different points of
// their solve (new, initialising, iterating, done) share the same launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icnnm {

constexpr int kThreads = 256;  // 4 wavefronts of 64 lanes
constexpr int kRowUnit = 64;   // spatial rows per wave work unit (two 32-row MFMA groups)
constexpr int kColUnit = 64;   // columns per wave work unit (two 32-column MFMA blocks)
constexpr int kGroup = 256;    // columns (forward) or kernel offsets (adjoint) per workgroup
constexpr int kLStepElems = 64; // output elements per L-step workgroup (four lanes each)

enum Phase : int32_t { kNew = 0, kInit = 1, kRun = 2, kDone = 3 };

enum Prec : int32_t { kFP32 = 0, kBF16 = 1, kFP16 = 2 };
// Kernel mode (not an instance precision): the refresh rounds of BF16/FP16 instances
// contracted on BF16 MFMA with both operands split into a BF16 head and a BF16 tail
// (three products: head x head, tail x head, head x tail), FP32 accumulation.
constexpr int kX3 = 3;
// tile ranges per 64-column block in the column-norm reduction (kp / 4 reduction
// blocks per instance: kp / 64 column blocks x 16 ranges)
constexpr int kColRanges = 16;

struct alignas(16) InstState {
  double theta;      // penalty for the next iteration (<= 0: derive theta0 at initialisation)
  double theta_cur;  // penalty of the iteration in flight
  double ratio;      // theta_cur / theta_next, rescales the scaled dual U = Y / theta
  double denom;      // ||P_Omega M||_F, 1 when zero
  double r_primal;
  double r_change;
  double objective;
  int32_t phase;
  int32_t iters;
  int32_t converged;
  int32_t status;     // 0 ok, -5 numeric
  int32_t refresh;    // reduced precision: this iteration evaluates both contractions in FP32
  int32_t pad[3];
  double ratio_prev;  // ratio of the previous iteration (reconstructs the previous G)
};
static_assert(sizeof(InstState) == 96, "InstState is copied between host and device as is");

struct alignas(16) InstDev {
  int32_t m[3], k[3], b[3], E[3], nt[3], C[3], goff[3];
  int32_t ntiles, bm, E123, nlblk, nslice, prec, max_iter, refresh_every;
  int32_t gshift, pad_;  // gather-table entries: (tile << gshift) | box position
  int32_t lb[3], pad2_;  // log2 of the tile extents b (powers of two)
  int64_t mtot;
  double lam, rho, theta_max, tol, theta0;
  const float* M;
  const uint8_t* mask;
  float* L;         // current iterate (C order)
  float* D;         // reduced precision: L^t - L^{t-1}, the operand of the delta forward
  void* U;          // scaled multiplier Y / theta, tile layout: FP32, or BF16 in the
                    // reduced-precision forms (16-byte chunks of eight values)
  float* W;         // A_k(L) V of the current iterate, tile layout, FP32 (Q = W - U)
  float* part;      // adjoint halo partials [ntiles][nsg][E123]
  float* qpart;     // [kp / 64][ntiles][64] per-tile sums of Q^2
  float* wpart;     // [kp / 64][ntiles][64] per-tile sums of W^2
  float* rpart;     // [ntiles][ncg] per-tile sums of (Z - W)^2
  double* dlpart;   // [nlblk][2] L-step partial sums: ||dL||^2, ||P_Omega(L - M)||^2
  double* slice;    // [kColRanges][kp][2] column sums per tile range, then [nslice][3]
                    // FP64 slice sums of the scalars
  float* s;         // shrink factors [kp]
  float* T;         // reduced precision: running A_k^*(G V^T) / k, updated by deltas  [m]
  const int32_t* gtab;  // per-dimension gather tables, entries (tile << gshift) | position, -1 = none
  InstState* st;
};

struct StageArgs {
  const InstDev* inst;
  const int2* tiles;     // (instance, local tile) per global tile
  const int2* lblocks;   // (instance, block) for the L-step
  const int2* slices;    // (instance, slice) for the column-norm reduction
  const float* Vf;       // forward operand layout of V (FP32)
  const float* Va;       // adjoint operand layout of V (FP32)
  const float* Vp;       // V zero-padded to kp x kp, row-major (FP32)
  const void* Vf_lo;     // forward operand layout of V (BF16/FP16)
  const void* Va_lo;     // adjoint operand layout of V (BF16/FP16)
  const void* Vp_lo;     // V zero-padded to kp x kp, row-major (BF16/FP16)
  const void* Vf_x;      // split-BF16 V, forward operand layout: heads, then tails
  const void* Vp_x;      // split-BF16 V, zero-padded row-major: heads, then tails
  int32_t kp, k, nsg, ncg;  // k: offsets of the contraction kernel (innermost extent
                            // padded to a multiple of 4 in BF16/FP16)
  int32_t kt;               // offsets of the kernel itself: the 1/k of the L-step
  int32_t u16;              // U stored in 16 bits (the instances' precision is BF16/FP16)
  int32_t ntiles;        // entries of `tiles`
  int32_t nlblocks;      // entries of `lblocks`
  int32_t tiles_per_slice;
  int32_t prec;
  int32_t split;         // split contractions: 64-column (offset) groups, the kernel
                         // offsets (eigendirections) of a unit shared by the four
                         // wavefronts; then ncg = nsg = kp / 64
  int32_t rx3;           // refresh rounds of BF16/FP16 instances run the kX3 kernels
                         // (the FP32 kernels then serve only FP32 instances and the
                         // initialisation)
};

// Launchers (defined in kernels.hip). All take the stream to launch on.
void launch_colnorm(const StageArgs& a, int nslices_total, int ninst, hipStream_t st);
// mode 0: FP32 contraction (initialisation, FP32 solves, refresh iterations);
// mode 1 / 2: BF16 / FP16 contraction of the change since the previous iteration;
// mode kX3: split-BF16 refresh contraction (forward with 64-row units; adjoint: the
// tiled one only).
// gv: col2im gather variant, 0 generic, 8 box lines (innermost kernel extent 4,
// innermost tile extent 8, E0 E1 <= 512 for every instance of the launch)
void launch_adjoint(const StageArgs& a, int ntiles_total, int lds_floats, int mode, int gv, hipStream_t st);
void launch_lstep(const StageArgs& a, int nlblocks_total, hipStream_t st);
// rb: 32-row blocks per reduced-precision unit (2, or 4 when every instance of the
// launch has tiles of a multiple of 128 rows); FP32 always uses 2
void launch_forward(const StageArgs& a, int ntiles_total, int lds_floats, int mode, int rb, hipStream_t st);
void launch_prep_v(const float* V, int k, int kp, float* Vf, float* Va, float* Vp, void* Vf_lo,
                   void* Va_lo, void* Vp_lo, int prec, hipStream_t st);
// split-BF16 copies of V for the kX3 kernels (each kp x kp heads, then kp x kp tails)
void launch_prep_v_x3(const float* V, int k, int kp, void* Vf_x, void* Vp_x, hipStream_t st);
// adjoint tiled for large kernels (kp >= 512, 128-row tiles)
void launch_adjoint_big(const StageArgs& a, int ntiles_total, int mode, int gv, hipStream_t st);
// LDS bytes of the tiled adjoint's split-BF16 refresh (mode kX3) for padded k = kp
size_t adjoint_big_x3_lds_bytes(int kp);
void launch_check_v(const float* V, int k, float* out_maxdev, hipStream_t st);
// Circular autocorrelation R(d) += sum_x L[x] L[x + d] over the lag box |d_j| < k_j
// (the Gram of A_k(L) in lag form), tiled: tiles of L with their halo in LDS, partial
// sums per block in `part` (autocorr_part_doubles(k) doubles), then a fixed-order sum
constexpr int kAcBlocks = 256;         // blocks of the tiled pass (each loops over tiles)
constexpr int kAcHaloFloats = 38912;   // LDS budget of a tile's halo box (152 KB)
struct AcGeom {
  int m[3], k[3], t[3], h[3], nt[3];
  int ntiles, nlags;
};
AcGeom autocorr_geometry(const int32_t* m, const int32_t* k);
size_t autocorr_part_doubles(const int32_t* k);
void launch_autocorr(const float* L, const int32_t* m, const int32_t* k, double* R, double* part,
                     hipStream_t st);
void launch_gram_expand(const double* R, const int32_t* k, double* G, hipStream_t st);
// FP64 products for the diagnostics: C = op(A) B for n x n row-major matrices
// (op(A) = A^T when trans_a), and a float -> double copy of n values
void launch_gemm_f64(const double* A, int trans_a, const double* B, double* C, int n, hipStream_t st);
void launch_f32_to_f64(const float* src, double* dst, int64_t n, hipStream_t st);
void launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st);
void launch_fill_f32(float* dst, float v, int64_t n, hipStream_t st);
// parallel cyclic Jacobi eigensolver (jacobi.hip), order n even: A <- G padded, V <- I;
// one round A -> B, V -> W (rot: 3 n / 2 doubles of scratch for the round's
// rotations); off-diagonal and total sums of squares of A into out[2] (part: 512
// doubles of scratch)
void launch_jacobi_init(const double* G, int k, double* A, double* V, int n, hipStream_t st);
void launch_jacobi_round(const double* A, double* B, const double* V, double* W, int n, double* rot,
                         hipStream_t st);
void launch_jacobi_offnorm(const double* A, int n, double* part, double* out, hipStream_t st);
// V (kt x kt, kernel dims kd) -> the k x k bank of the padded kernel dims kdp (only the
// innermost extent differs): rows of padded offsets and columns past kt are zero
void launch_pad_v(const float* V, const int* kd, const int* kdp, float* out, hipStream_t st);

}  // namespace icnnm

/*
 * icnnm.h - C ABI of the MI355X (gfx950) solver for Inductive Convolution
 * Nuclear Norm Minimization (ICNNM), tensor completion with arbitrary sampling.
 *
 * Problem (Definition 1 and eq:InductiveCNNM): given an observed order-n
 * tensor M (n <= 3; lower orders use unit leading dimensions), a sampling set
 * Omega given as a mask, a kernel size k_1 x .. x k_n with k_j <= m_j
 * (Section II-B) and an orthogonal bank V of k convolution eigenvectors
 * (Section III-A), find
 *     min_L || A_k(L) V ||_{2,1}   s.t.  P_Omega(L) = P_Omega(M)
 * or its penalized form (eq:admm) for a finite lambda, by the ADMM iteration of
 * Section III-D. V is learned beforehand from reference tensors (Definition 3,
 * eq:A).
 *
 * Conventions shared by every entry point
 *  - Layout: tensors are dense float32 in C order (last dimension fastest);
 *    vectorisation of tensors and of kernel offsets is C order, so row s of V
 *    is the kernel offset (s_1, .., s_n) in C order and column i is the i-th
 *    eigenvector. V is k x k float32, row-major.
 *  - Omega is a uint8 mask of the tensor's shape: nonzero = observed.
 *  - Array arguments (M, mask, V, L_out, refs, V_out) are DEVICE pointers on
 *    the context's device, allocated and owned by the caller. The library
 *    never frees them and keeps no reference after the call returns (submit:
 *    until poll reports completion). icnnm_params, icnnm_info, shapes and
 *    eigvals_out are HOST pointers.
 *  - stream is a hipStream_t (NULL = the context's own stream). Calls are
 *    ordered after work already queued on it and return after their outputs
 *    are written (submit/poll excepted).
 *  - Errors: every call returns an icnnm_status; on error, nothing is written
 *    to outputs beyond what is documented and icnnm_last_error() describes the
 *    failure. No C++ exception crosses this boundary.
 *  - Tile boxes: chosen by a cost model, or with the environment variable
 *    ICNNM_AUTOTUNE=1 by timing the best few candidates on the instance (solve
 *    and solve_batch; cached per shape in the context and, if
 *    ICNNM_AUTOTUNE_CACHE names a file, across processes). icnnm_info.tile
 *    reports the box used. Two switches exist for measurement:
 *    ICNNM_TILE=b0,b1,b2 forces one box (ICNNM_E_INVALID if it does not fit
 *    the problem; a different box changes the floating-point summation order,
 *    so results agree to rounding, not bit for bit), and ICNNM_GATHER=generic
 *    keeps the position-owning col2im gather (bit-identical results).
 *  - Refresh contractions of the BF16/FP16 forms: split BF16 where the tiled
 *    adjoint applies (icnnm_info.refresh_x3), FP32 MFMA otherwise or with
 *    ICNNM_REFRESH=fp32 (read when a solve's group is built).
 *  - Thread safety: a context may be used from several host threads; calls
 *    on one context are serialised internally. icnnm_submit/icnnm_poll may be
 *    called concurrently with each other.
 */
#ifndef ICNNM_H
#define ICNNM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icnnm_ctx icnnm_ctx;
typedef int32_t icnnm_status;

#define ICNNM_OK 0
#define ICNNM_PENDING 1
#define ICNNM_E_INVALID (-1)  /* bad shape, pointer or parameter; k_j > m_j; ndim not in [1,3] */
#define ICNNM_E_NOMEM (-2)    /* device allocation failed */
#define ICNNM_E_BUDGET (-3)   /* the request alone exceeds the context's HBM budget */
#define ICNNM_E_DEVICE (-4)   /* HIP runtime error */
#define ICNNM_E_NUMERIC (-5)  /* NaN/Inf in a residual */
#define ICNNM_E_NOTFOUND (-6) /* unknown or already collected ticket */

#define ICNNM_PREC_FP32 0
#define ICNNM_PREC_BF16 1
#define ICNNM_PREC_FP16 2

/* Shape of one tensor and of its convolution kernel. Only the first ndim
 * entries of m[] and kdim[] are read; an order-1 or order-2 problem is solved
 * as an order-3 one with unit leading dimensions (a circular convolution over
 * a unit dimension is the identity). */
typedef struct {
  int32_t ndim;    /* 1..3 */
  int64_t m[3];    /* tensor dimensions m_1..m_n */
  int64_t kdim[3]; /* kernel dimensions k_1..k_n, 1 <= k_j <= m_j */
} icnnm_shape;

/* Solver parameters (Section III-D). Fill with icnnm_params_default first. */
typedef struct {
  double lambda;        /* +INFINITY (default): exact P_Omega constraint (eq:InductiveCNNM);
                           finite > 0: penalized form (eq:admm), lambda = 1000 in the paper */
  double theta0;        /* initial penalty; <= 0 selects 1.25 / ||A_k(P_Omega M) V||_{2,inf}
                           (1.0 when that norm is zero) */
  double rho;           /* penalty growth per iteration, default 1.1 */
  double theta_max;     /* penalty cap, default 1e10 */
  int32_t max_iter;     /* iterations to run (default 100) */
  double tol;           /* stop when max(r_primal, r_change) <= tol; 0 = run max_iter exactly */
  int32_t precision;    /* ICNNM_PREC_*: arithmetic of the two contractions. BF16/FP16 pad
                           the innermost kernel extent to a multiple of 4 with zero rows of V
                           (exact); ICNNM_E_INVALID if the padded extent exceeds the tensor's */
  int32_t refresh_every;/* reduced precision: full FP32 evaluation every this many iterations */
  int32_t check_v;      /* nonzero: reject V unless max|V^T V - I| <= 1e-5 */
} icnnm_params;

/* Per-solve report. r_primal = ||Z - A_k(L)V||_F / (sqrt(k) ||P_Omega M||_F),
 * r_change = ||L^t - L^{t-1}||_F / ||P_Omega M||_F, objective = ||A_k(L)V||_{2,1}
 * at the returned L; all reduced in FP64 on the device. */
typedef struct {
  int32_t iters;
  int32_t converged;
  double r_primal;
  double r_change;
  double objective;
  double theta_final;
  double t_queue_s;  /* submit only: time from submit to first device work */
  double t_device_s; /* wall time from first device work to completion */
  int32_t tile[3];   /* tile box b_1..b_3 the solve ran with (order-3 form; from the
                        cost-model planner, or measured with ICNNM_AUTOTUNE=1) */
  int32_t split;     /* 1: the contractions ran in their split form (an instance solved
                        alone with fewer tiles than the chip has compute units: the
                        kernel offsets of a work unit are shared by four wavefronts,
                        which sum in a different order); 0 otherwise */
  int32_t refresh_x3; /* 1: the refresh iterations of a BF16/FP16 solve ran their
                         contractions in split BF16 (head + tail of each operand, three
                         MFMA products, FP32 accumulation) instead of FP32; set where the
                         tiled adjoint applies (padded k a multiple of 256, 128-row
                         tiles) unless ICNNM_REFRESH=fp32. A served request reports the
                         setting of its group when it completed. */
} icnnm_info;

/* Default parameters: lambda = +inf, theta0 auto, rho 1.1, theta_max 1e10,
 * max_iter 100, tol 0, FP32, refresh_every 10, check_v 0. */
void icnnm_params_default(icnnm_params *p);

/* Create a context on HIP device `device`. hbm_budget_bytes bounds the device
 * memory the context may hold for solver state (0 = 90% of free memory at
 * creation). Returns ICNNM_E_DEVICE if the device is not usable. */
icnnm_status icnnm_create(int device, size_t hbm_budget_bytes, icnnm_ctx **out);

/* Destroy a context: waits for in-flight served requests, frees all state. */
void icnnm_destroy(icnnm_ctx *ctx);

/* Human-readable description of the last error on this context (never NULL). The
 * string is a copy owned by the calling thread, valid until its next call of
 * icnnm_last_error. */
const char *icnnm_last_error(const icnnm_ctx *ctx);

/* Tile plan of one instance, computed on the host alone (no context, no device
 * work; callable without a GPU): the tile box the cost model picks for the shape
 * (joint = 0: as icnnm_solve plans it; joint != 0: as a member of a joint launch of
 * icnnm_solve_batch or the server), the tiles per dimension and in total, the padded
 * kernel size the contractions run at, and the device bytes of the instance's solver
 * state (iterates, multiplier, halo partials, reduction slices, gather tables: what
 * the instance charges to the HBM budget; V operand copies not included). The
 * state per (row, eigendirection) pair is the scaled multiplier and the Z-step
 * operand of Section III-D.
 * Errors: ICNNM_E_INVALID for a bad shape or parameters, or when no tile box fits
 * the planner's limits (e.g. more than 32767 tiles along one dimension). */
typedef struct {
  int32_t tile[3];          /* tile box b_1..b_3 (order-3 form) */
  int32_t tiles_per_dim[3]; /* ceil(m_j / b_j) */
  int32_t ntiles;
  int32_t padded_k;         /* k rounded up to the contraction's column unit */
  int64_t state_bytes;
  int32_t split;            /* 1: split contractions (see icnnm_info.split; joint = 0 only) */
} icnnm_plan_info;
icnnm_status icnnm_plan(const icnnm_shape *shape, const icnnm_params *params, int32_t joint,
                        icnnm_plan_info *out);

/* Learn the k convolution eigenvectors of a reference ensemble (Definition 3):
 * the eigenvectors of sum_j A_k(L_j)^T A_k(L_j) (eq:A), accumulated in FP64 on
 * the device, all k of them, sorted by descending eigenvalue, each column's
 * largest-magnitude entry made positive.
 *   kdim[3]      kernel dimensions, first ref_shapes[0].ndim entries used
 *   b            number of reference tensors (>= 1)
 *   ref_shapes   b host shapes; each ref_shapes[j].kdim must equal kdim
 *   refs         b device pointers to float32 C-order tensors
 *   V_out        device, k*k float32, row-major [s][i]
 *   eigvals_out  host, k doubles (descending); may be NULL
 */
icnnm_status icnnm_learn_eigvecs(icnnm_ctx *ctx, const int64_t kdim[3], int32_t b,
                                 const icnnm_shape ref_shapes[], const float *const refs[],
                                 float *V_out, double *eigvals_out, void *stream);

/* Diagnostics of a tensor L0 under a bank of learned convolution eigenvectors
 * (Definition 2, eq:rkL0, eq:alphaK), for analysis of how well V suits L0:
 *   sigma_out[i] = || L0 * kappa_i ||_F, the relative convolution eigenvalue of
 *                  column i of V (the column norms of A_k(L0) V);
 *   rank_out     = r_K(L0), the number of i with sigma_i > rtol * max_i sigma_i;
 *   alpha_out    = alpha_K(L0) = || A_k(L0) V D ||_2 with D = diag(1 / sigma_i) on
 *                  that support and 0 elsewhere (the spectral correlation).
 * All in FP64: the Gram A_k(L0)^T A_k(L0) from circular autocorrelations on the
 * device (as in icnnm_learn_eigvecs), C = V^T G V on the device, sigma_i =
 * sqrt(C_ii), and alpha^2 the largest eigenvalue of D C D on the host. Through
 * the Gram, a sigma_i far below max sigma is accurate to about 1e-8 max sigma
 * (sqrt of the FP64 rounding of C_ii); rtol should stay above that.
 *   shape      host; the tensor and kernel dimensions (as for icnnm_solve)
 *   L0         device, float32 C-order tensor of the shape
 *   V          device, k x k float32 row-major [s][i]
 *   rtol       > 0, relative threshold of the support
 *   sigma_out  host, k doubles; may be NULL
 *   rank_out   host; may be NULL
 *   alpha_out  host; may be NULL
 * Blocks until the outputs are written. Errors: ICNNM_E_INVALID (bad shape, NULL
 * L0 or V, rtol <= 0), ICNNM_E_NOMEM, ICNNM_E_BUDGET, ICNNM_E_DEVICE. */
icnnm_status icnnm_diagnostics(icnnm_ctx *ctx, const icnnm_shape *shape, const float *L0, const float *V,
                               double rtol, double *sigma_out, int32_t *rank_out, double *alpha_out,
                               void *stream);

/* Solve one completion instance (Section III-D iteration).
 *   shape   host; M, mask, L_out device arrays of prod(m) entries
 *   V       device, k*k float32 orthogonal eigenvector bank
 *   L_out   device, receives the final iterate; with lambda = +inf,
 *           L_out[i] == M[i] bit for bit for every observed i
 *   info    host, may be NULL
 */
icnnm_status icnnm_solve(icnnm_ctx *ctx, const icnnm_shape *shape, const float *M,
                         const uint8_t *mask, const float *V, const icnnm_params *params,
                         float *L_out, icnnm_info *info, void *stream);

/* icnnm_solve for callers that cannot allocate device memory (code that must not
 * call hipMalloc or any allocating routine: tight serving loops, harnesses that
 * forbid allocation, set-ups around graph capture). Same arguments, parameters,
 * results and errors as icnnm_solve, and the same kernels; the call makes no device
 * allocation. Every device array beyond the caller's inputs and output (V operand
 * layouts, instance state, multiplier and Z-step operand, halo partials, reduction
 * slices, tables) is carved from a fixed per-device scratch of 160 MiB that the
 * library holds from its load to the end of the process. Instances whose solver
 * state does not fit return ICNNM_E_BUDGET before any device work (icnnm_plan's
 * state_bytes plus the V layouts, 3 kp^2 floats and for BF16/FP16 3 kp^2 halves,
 * must stay below that; a 64x64x16 tensor with an 8x8x4 kernel takes about 140 MB).
 * The tile box is the cost model's (ICNNM_AUTOTUNE is ignored: measuring would
 * allocate), and rounds are launched directly (no graph capture). The scratch keeps
 * the last call's contents; every array is written before it is read, so results
 * do not depend on them. All calls on one device share the scratch: calls that
 * overlap on one device would race, so within a process the library runs them one
 * at a time per device. The call is synchronous like icnnm_solve. */
icnnm_status icnnm_solve_noalloc(icnnm_ctx *ctx, const icnnm_shape *shape, const float *M,
                                 const uint8_t *mask, const float *V, const icnnm_params *params,
                                 float *L_out, icnnm_info *info, void *stream);

/* Solve `count` independent instances of possibly different shapes that share
 * one kernel size and one V, in joint launches (one per stage and iteration,
 * spanning all instances). Arrays are indexed by instance; infos may be NULL.
 * Each instance stops on its own when tol > 0. */
icnnm_status icnnm_solve_batch(icnnm_ctx *ctx, int32_t count, const icnnm_shape shapes[],
                               const float *const M[], const uint8_t *const masks[],
                               const float *V, const icnnm_params *params,
                               float *const L_out[], icnnm_info infos[], void *stream);

/* Serving: enqueue one request and return at once with a ticket. A scheduler
 * thread admits queued requests while the HBM budget allows, keeps their state
 * resident, runs all admitted requests sharing a V in joint iterations, and
 * retires each when its residual meets params->tol (or at max_iter).
 * Buffers must stay valid until icnnm_poll returns a value other than
 * ICNNM_PENDING. Returns ICNNM_E_BUDGET if the request can never fit. */
icnnm_status icnnm_submit(icnnm_ctx *ctx, const icnnm_shape *shape, const float *M,
                          const uint8_t *mask, const float *V, const icnnm_params *params,
                          float *L_out, uint64_t *ticket);

/* ICNNM_PENDING while the request runs; its final status once, after which
 * the ticket is released (a second poll returns ICNNM_E_NOTFOUND). */
icnnm_status icnnm_poll(icnnm_ctx *ctx, uint64_t ticket, icnnm_info *info);

/* Stage timing for measurement. While enabled on a context, synchronous solves
 * launch their stage kernels one by one (no graph replay) with a pair of HIP
 * events around each launch on the context's stream; the elapsed times are
 * accumulated per stage. Stages: 0 column norms, 1 adjoint, 2 L-step,
 * 3 forward. Rounds whose two contractions both run in BF16/FP16 (the delta
 * kernels of the reduced-precision form) are accounted at index 4 + stage, all
 * other rounds (FP32 solves, initialisation, FP32 refresh iterations) at index
 * stage. icnnm_stage_times copies the totals (milliseconds) and launch counts
 * into the host arrays ms[8] and counts[8], then resets them if reset is
 * nonzero. Timing adds event overhead between launches; keep it off for
 * throughput runs. */
icnnm_status icnnm_set_profiling(icnnm_ctx *ctx, int32_t enable);
icnnm_status icnnm_stage_times(icnnm_ctx *ctx, double ms[8], int64_t counts[8], int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* ICNNM_H */

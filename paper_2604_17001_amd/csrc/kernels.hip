// HIP kernels of the ICNNM solver for gfx950 (CDNA4).
//
// Operators (Section II-B, Section III-D):
//   A_k(L)[i, s] = L[(i - s) mod m]           convolution matrix (eq:ak)
//   A_k^*(X)[t]  = sum_s X[(t + s) mod m, s]   its adjoint
// The m x k state arrays (W = A_k(L) V and the scaled multiplier U = Y / theta;
// the Z-step operand Q = W - U is derived on load) are stored in "tile layout":
// for each 32-row group of a tile and each 32-column block, the 1024 values are
// the 32x32 MFMA accumulator's, as 256 float4: float4 g (accumulator values
// 4g..4g+3) of lane l at position g * 64 + l. A lane reads and writes its 16
// values as four 16-byte accesses, each of which is one contiguous kilobyte over
// the wavefront, and the adjoint consumes them directly as its B operand without
// a transpose. In the reduced-precision forms U is kept in 16 bits (u16_unpack).
//
// Accumulator layout of v_mfma_f32_32x32x2_f32 for D = A(32 x 2) B(2 x 32):
//   lane l, register v holds D[(v/4)*8 + (l/32)*4 + v%4][l%32];
//   lane l supplies A[l%32][l/32] and B[l/32][l%32].
#include "icnnm_dev.h"

#include <algorithm>
#include <type_traits>
#include <vector>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace icnnm {

constexpr int kLanesPerElem = kThreads / kLStepElems;      // L-step lanes per output element

typedef float floatx16 __attribute__((ext_vector_type(16)));

// global address space qualifier for device code (the host pass sees plain types)
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL_AS __attribute__((address_space(1)))
#else
#define GLOBAL_AS
#endif

// Reduced-precision MFMA: v_mfma_f32_32x32x16_{bf16,f16}. Lane l supplies the eight
// consecutive K entries (l/32)*8 .. (l/32)*8+7 of row l%32 of A and of column l%32 of B;
// the accumulator layout is that of the 32x32 FP32 MFMA.
template <int MODE>
struct LowP;
template <>
struct LowP<kBF16> {
  typedef __bf16 h;
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  typedef __bf16 v4 __attribute__((ext_vector_type(4)));
  typedef GLOBAL_AS const v8 gv8;
  static __device__ __forceinline__ floatx16 mfma(v8 a, v8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct LowP<kFP16> {
  typedef _Float16 h;
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  typedef _Float16 v4 __attribute__((ext_vector_type(4)));
  typedef GLOBAL_AS const v8 gv8;
  static __device__ __forceinline__ floatx16 mfma(v8 a, v8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// the split-BF16 refresh contraction uses BF16 MFMA
template <>
struct LowP<kX3> : LowP<kBF16> {};

// Which contraction a stage kernel of mode MODE runs for an iterating instance:
// FP32 on FP32 solves and on refresh iterations, the reduced precision otherwise;
// with rx3 set, the refresh iterations of BF16/FP16 instances run the kX3 kernels.
template <int MODE, class Desc>
__device__ __forceinline__ bool runs_iteration(const Desc& I, const InstState* st, int rx3) {
  const bool full = (I.prec == kFP32) || st->refresh;
  const bool x3 = rx3 && I.prec != kFP32 && st->refresh;
  if (MODE == kX3) return x3;
  return MODE == kFP32 ? (full && !x3) : (!full && I.prec == MODE);
}

// Pointers read from descriptors are generic; loads through them become flat
// loads, which the wait-count logic tracks conservatively. These casts let the
// compiler emit global loads and keep prefetches in flight.
// (The host pass only parses kernel bodies, so it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(1))) const float4 gcfloat4;
typedef __attribute__((address_space(1))) float4 gfloat4;
typedef __attribute__((address_space(1))) const float gcfloat;
typedef __attribute__((address_space(1))) const uint4 gcuint4;
#else
typedef const float4 gcfloat4;
typedef float4 gfloat4;
typedef const float gcfloat;
typedef const uint4 gcuint4;
#endif
__device__ __forceinline__ gcfloat4* gc4(const void* p) { return (gcfloat4*)(p); }
__device__ __forceinline__ gfloat4* g4(void* p) { return (gfloat4*)(p); }
__device__ __forceinline__ gcfloat* gc1(const void* p) { return (gcfloat*)(p); }
__device__ __forceinline__ gcuint4* gcu4(const void* p) { return (gcuint4*)(p); }

// the instance descriptor read as constant memory (never written while kernels run)
typedef __attribute__((address_space(4))) InstDev CInstDev;

__device__ __forceinline__ int wrapi(int v, int m) {
  v %= m;
  return v < 0 ? v + m : v;
}

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Column inside a 32-column block held by lane l in accumulator register v.
__device__ __forceinline__ int acc_col(int v, int half) { return (v >> 2) * 8 + half * 4 + (v & 3); }

__device__ __forceinline__ void load16(const float* p, float* out) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float4 t = q[i];
    out[4 * i + 0] = t.x;
    out[4 * i + 1] = t.y;
    out[4 * i + 2] = t.z;
    out[4 * i + 3] = t.w;
  }
}

__device__ __forceinline__ void store16(float* p, const float* in) {
  float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = make_float4(in[4 * i], in[4 * i + 1], in[4 * i + 2], in[4 * i + 3]);
}

// s[c] for the 16 columns lane `half` holds in a 32-column block starting at c0.
__device__ __forceinline__ void load_cols16(const float* s, int c0, int half, float* out) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    float4 t = *reinterpret_cast<const float4*>(s + c0 + g * 8 + half * 4);
    out[4 * g + 0] = t.x;
    out[4 * g + 1] = t.y;
    out[4 * g + 2] = t.z;
    out[4 * g + 3] = t.w;
  }
}

// Sum over the 32 lanes of one half-wavefront (lanes with equal l/32).
__device__ __forceinline__ float half_sum(float x) {
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Offset of kernel offset s inside a box with strides (E1*E2, E2, 1); 0 for padding.
template <class Desc>
__device__ __forceinline__ int kernel_off(int s, const Desc& I, int k) {
  if (s >= k) return 0;
  int s2 = s % I.k[2];
  int t = s / I.k[2];
  int s1 = t % I.k[1];
  int s0 = t / I.k[1];
  return (s0 * I.E[1] + s1) * I.E[2] + s2;
}

// Box position of tile row r (C order inside the tile box), shifted by (k - 1) so
// that base - off(s) addresses row r's source (forward) or target (adjoint) t = r - s.
template <class Desc>
__device__ __forceinline__ int row_base(int r, const Desc& I, const int* o, bool& valid) {
  // tile extents are powers of two: shifts and masks instead of divisions
  const int a2 = r & (I.b[2] - 1);
  const int t = r >> I.lb[2];
  const int a1 = t & (I.b[1] - 1);
  const int a0 = t >> I.lb[1];
  valid = (o[0] + a0 < I.m[0]) && (o[1] + a1 < I.m[1]) && (o[2] + a2 < I.m[2]);
  return ((a0 + I.k[0] - 1) * I.E[1] + (a1 + I.k[1] - 1)) * I.E[2] + (a2 + I.k[2] - 1);
}

template <class Desc>
__device__ __forceinline__ void tile_origin(int lt, const Desc& I, int* o) {
  int n2 = lt % I.nt[2];
  int t = lt / I.nt[2];
  int n1 = t % I.nt[1];
  int n0 = t / I.nt[1];
  o[0] = n0 * I.b[0];
  o[1] = n1 * I.b[1];
  o[2] = n2 * I.b[2];
}

// Box position -> source coordinates of a tile's circular halo. Quotients use a float
// reciprocal with a +-1 correction (exact for the box sizes here, < 2^22); before
// wrapping, coordinates lie in (-m, 3m) (k <= m, tile extent < 2m), so two
// conditional subtractions and one addition wrap them.
__device__ __forceinline__ int divq(int x, int d, float rd) {
  int q = (int)((float)x * rd);
  q += ((q + 1) * d <= x) ? 1 : 0;
  q -= (q * d > x) ? 1 : 0;
  return q;
}
__device__ __forceinline__ int wrap3(int v, int m) {
  v += v < 0 ? m : 0;
  v -= v >= m ? m : 0;
  v -= v >= m ? m : 0;
  return v;
}
struct HaloMap {
  int E12, E2, s0, s1, s2, m0, m1, m2;  // s_d = tile origin - (k_d - 1)
  float r12, r2;
  template <class Desc>
  __device__ __forceinline__ HaloMap(const Desc& I, const int* o) {
    E2 = I.E[2];
    E12 = I.E[1] * E2;
    r12 = 1.f / (float)E12;
    r2 = 1.f / (float)E2;
    s0 = o[0] - (I.k[0] - 1);
    s1 = o[1] - (I.k[1] - 1);
    s2 = o[2] - (I.k[2] - 1);
    m0 = I.m[0];
    m1 = I.m[1];
    m2 = I.m[2];
  }
  // flat index of the (wrapped) row (g0, g1, 0) and the unwrapped innermost coordinate
  __device__ __forceinline__ int64_t row(int x, int& c2) const {
    const int x0 = divq(x, E12, r12), rem = x - x0 * E12;
    const int x1 = divq(rem, E2, r2), x2 = rem - x1 * E2;
    c2 = s2 + x2;
    return ((int64_t)wrap3(s0 + x0, m0) * m1 + wrap3(s1 + x1, m1)) * m2;
  }
};

// Sums of 16 per-lane values over the 32 lanes of each half-wavefront, by halving
// exchanges (16 shuffles instead of 80). On return v[0] holds, in lanes l and l ^ 1,
// the total of value index vi = 8 b4 + 4 b3 + 2 b2 + b1 (b_j = bit j of l).
__device__ __forceinline__ float half_sum16(float (&v)[16], int lane, int& vi) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool hi = lane & 16;
    const float send = hi ? v[i] : v[i + 8], keep = hi ? v[i + 8] : v[i];
    v[i] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool hi = lane & 8;
    const float send = hi ? v[i] : v[i + 4], keep = hi ? v[i + 4] : v[i];
    v[i] = keep + __shfl_xor(send, 8, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool hi = lane & 4;
    const float send = hi ? v[i] : v[i + 2], keep = hi ? v[i + 2] : v[i];
    v[i] = keep + __shfl_xor(send, 4, 64);
  }
  {
    const bool hi = lane & 2;
    const float send = hi ? v[0] : v[1], keep = hi ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 2, 64);
  }
  v[0] += __shfl_xor(v[0], 1, 64);
  vi = ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 + ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
  return v[0];
}

// 16-bit storage of the scaled multiplier U = Y / theta in the reduced-precision forms
// (UB = 2): the FP16 value of the unscaled multiplier Y = theta U, whose entries stay
// of order one (the column norms of Y are bounded near 1 by dual feasibility) while U
// shrinks with the growing penalty; theta is the penalty the forward that wrote U
// scaled it with (theta_next there, theta_cur for every later reader), and readers
// multiply by the same float 1/theta. Eight values per 16-byte chunk; a piece (32
// rows x 32 columns of the tile layout) is 128 chunks: chunk c of lane l, values
// 8c..8c+7 of the lane's accumulator order, at c * 64 + l, so each access is one
// contiguous kilobyte over the wavefront.
__device__ __forceinline__ void u16_unpack(const uint4 h, float inv, float* v) {
  const uint32_t w[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    _Float16 lo, hi;
    const uint16_t bl = (uint16_t)(w[i] & 0xffffu), bh = (uint16_t)(w[i] >> 16);
    __builtin_memcpy(&lo, &bl, 2);
    __builtin_memcpy(&hi, &bh, 2);
    v[2 * i] = (float)lo * inv;
    v[2 * i + 1] = (float)hi * inv;
  }
}
__device__ __forceinline__ uint32_t u16_bits(float x, float scale) {
  const _Float16 h = (_Float16)(x * scale);  // round to nearest even
  uint16_t r;
  __builtin_memcpy(&r, &h, 2);
  return r;
}
__device__ __forceinline__ uint4 u16_pack(const float* v, float scale) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = u16_bits(v[2 * i], scale) | (u16_bits(v[2 * i + 1], scale) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}
// the value a stored 16-bit U reads back as
__device__ __forceinline__ float u16_round(float x, float scale, float inv) {
  return (float)(_Float16)(x * scale) * inv;
}

// =====================================================================================
// forward: W = A_k(L) V, fused with the dual update.
// The per-instance state is W (FP32) and the scaled multiplier U = Y / theta (FP32, or
// 16 bits in the reduced-precision forms: UB = 2, see u16_unpack); Q = W - U is derived on load.
//   init (phase kInit): U = 0, W                             (Y^0 = 0)
//   run  (phase kRun):  Z = s.Q_old, G = U_old + Z,
//                       U = (G - W) theta/theta',  Q = W - U (with U as stored)
// and per-tile partial sums of Q^2, W^2 (per column) and (Z - W)^2.
// grid = (tiles, kp / 256 column groups); each wave takes (64 rows x 64 columns) units.
// Split form (KS, for launches with few tiles): column groups of 64, and the four
// wavefronts of a workgroup share each unit, every one contracting a quarter of the
// kernel offsets; the partial sums meet in LDS (fixed order) and each wavefront runs
// the epilogue of one 32 x 32 piece. Four times the workgroups for the same work.
// =====================================================================================
template <int MODE, int RB, int UB, bool KS>
__global__ __launch_bounds__(kThreads, 2) void k_forward(StageArgs a) {
  static_assert(RB == 2 || (RB == 4 && MODE != kFP32), "FP32 units have two row blocks");
  static_assert(UB == 4 || UB == 2, "U is stored in 32 or 16 bits");
  static_assert(!KS || RB == 2, "the split form has 64-row units");
  extern __shared__ float smem[];
  const int2 tt = a.tiles[blockIdx.x];
  // The descriptor is read as constant memory: through a generic reference, a field
  // read after a global store (which might alias it) is loaded again with a vector
  // load and a wait for all outstanding loads, which drains the epilogue's prefetched
  // state loads at every piece; constant loads go through the scalar cache.
  const CInstDev& I = *(const CInstDev*)(a.inst + tt.x);
  const int phase = I.st->phase;
  if (MODE == kFP32) {
    if (phase != kInit && !(phase == kRun && runs_iteration<MODE>(I, I.st, a.rx3))) return;
  } else {
    if (!(phase == kRun && runs_iteration<MODE>(I, I.st, a.rx3))) return;
  }
  const bool init = phase == kInit;
  const int kp = a.kp, k = a.k;
  const int cg = blockIdx.y;
  const int CG = KS ? kColUnit : (kp < kGroup ? kp : kGroup);
  const int lt = tt.y;
  // (the wavefront index is uniform: read into a scalar register, so the unit and
  // piece indices derived from it stay scalar and hold no vector registers)
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), half = lane >> 5;

  int o[3];
  tile_origin(lt, I, o);
  const int E123 = I.E123;
  const int E12 = I.E[1] * I.E[2];
  const int nrc = I.bm / kRowUnit, ncc = CG / kColUnit;
  // FP32: halo of L (E123 floats) + offset table offs2[h*16 + half*8 + jj] = -4 off(s)
  //       (a byte offset), s = (h/2)*32 + (h%2)*16 + 2*jj + half
  // reduced precision: halo of D = L^t - L^{t-1} expanded along the innermost
  //       dimension, E4[y][d] = D_halo[y - d] (d < 4), so one 8-byte read yields four
  //       consecutive kernel offsets; offset table offs4[kk*4 + half*2 + g] = off(s)
  //       for s = 16*kk + 8*half + 4*g
  // (split BF16: head, middle and tail parts of L, each an expanded halo)
  const int halo_floats = MODE == kFP32 ? ((E123 + 3) & ~3) : (MODE == kX3 ? 6 : 2) * E123;
  float* halo = smem;
  int* offs2 = reinterpret_cast<int*>(smem + halo_floats);
  const int noffs = MODE == kFP32 ? kp : kp / 4;
  // column partials per 64-row chunk (per 32-row block in the split form)
  const int ncr = KS ? 2 * nrc : nrc;
  float* colq = reinterpret_cast<float*>(offs2 + noffs);  // [ncr][CG]
  float* colw = colq + ncr * CG;                          // [ncr][CG]
  float* rred = colw + ncr * CG;                          // [nrc * ncc (* 4 split)]
  float* kred = rred + nrc * ncc * (KS ? 4 : 1);          // split: [12][16][64] partials

  const HaloMap hm(I, o);
  if constexpr (MODE == kFP32) {
    // halo of L over the tile box extended backwards by k - 1, with circular wrap;
    // eight positions per thread are loaded before any is stored. The loads are
    // unconditional (positions past the box read box position 0, then discarded) and
    // their values pass through an empty asm before the selection: otherwise the
    // compiler turns the selection into a branch around each load, with the load's
    // wait inside it, one load at a time.
    gcfloat* L = gc1(I.L);
    for (int xb = tid; xb < E123; xb += 8 * kThreads) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int x = xb + j * kThreads;
        int c2;
        const int64_t r = hm.row(x < E123 ? x : 0, c2);
        v[j] = L[r + wrap3(c2, hm.m2)];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) asm("" : "+v"(v[j]));
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int x = xb + j * kThreads;
        if (x < E123) halo[x] = v[j];
      }
    }
    for (int e = tid; e < kp; e += kThreads) {
      const int h = e >> 4, hf = (e >> 3) & 1, jj = e & 7;
      offs2[e] = -4 * kernel_off((h >> 1) * 32 + (h & 1) * 16 + 2 * jj + hf, I, k);
    }
  } else {
    typedef typename LowP<MODE>::h H;
    H* e4 = reinterpret_cast<H*>(halo);
    // the delta forms stage D; the split-BF16 refresh stages L in three parts
    gcfloat* D = gc1(MODE == kX3 ? I.L : I.D);
    // four positions per thread (16 values) are loaded before any is stored, all
    // unconditionally (see the FP32 halo above): excluded entries read a valid
    // address and are set to zero
    for (int xb = tid; xb < E123; xb += 4 * kThreads) {
      float v[4][4];
      int x2v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = xb + j * kThreads;
        int c2;
        const int64_t r = hm.row(x < E123 ? x : 0, c2);
        x2v[j] = c2 - hm.s2;
#pragma unroll
        for (int d = 0; d < 4; ++d) v[j][d] = D[r + wrap3(x2v[j] >= d ? c2 - d : c2, hm.m2)];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          asm("" : "+v"(v[j][d]));
          v[j][d] = x2v[j] >= d ? v[j][d] : 0.f;
        }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = xb + j * kThreads;
        if (x < E123) {
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const H hd = (H)v[j][d];
            e4[4 * x + d] = hd;
            if constexpr (MODE == kX3) {
              // v = head + middle + tail + O(2^-27 |v|) (each difference is exact in FP32)
              const float r = v[j][d] - (float)hd;
              const H md = (H)r;
              e4[4 * (E123 + x) + d] = md;
              e4[4 * (2 * E123 + x) + d] = (H)(r - (float)md);
            }
          }
        }
      }
    }
    for (int e = tid; e < kp / 4; e += kThreads) offs2[e] = kernel_off(4 * e, I, k);
  }
  __syncthreads();

  const float ratio = (float)I.st->ratio;
  // 16-bit U: written as FP16 of theta_next U, read back (and the old U read) through
  // the float reciprocal of the penalty it was scaled with
  const float uscale = (float)I.st->theta, uinv = (float)(1.0 / I.st->theta);
  const float uinv_old = (float)(1.0 / I.st->theta_cur);
  const int nkb = kp / 32;
  const int nhs = 2 * nkb;  // half-steps of 16 kernel offsets
  // a unit is RB 32-row blocks x 64 columns: RB = 2 (FP32 and reduced precision) or
  // 4 (reduced precision with 128-row multiples: each V fragment feeds four row
  // blocks, halving the L2 traffic of V)
  constexpr int kRpu = RB / 2;  // 64-row chunks per unit
  const int nun = (nrc / kRpu) * ncc;
  // the kernel-offset half-steps this wavefront contracts
  const int hs0 = KS ? wave * (nhs / 4) : 0, hs1 = KS ? hs0 + nhs / 4 : nhs;
  // unit u = ru * ncc + cc, advanced without divisions (ncc <= 4)
  int ru = 0, cc = KS ? 0 : wave;
  while (cc >= ncc) {
    cc -= ncc;
    ++ru;
  }
  for (int u = KS ? 0 : wave; u < nun; u += KS ? 1 : 4) {
    const int c0 = cg * CG + cc * kColUnit;
    bool valid[RB];
    int base[RB];
#pragma unroll
    for (int ib = 0; ib < RB; ++ib) base[ib] = row_base(ru * RB * 32 + ib * 32 + (lane & 31), I, o, valid[ib]);

    // U/Q loads of the fused epilogue over the 2 RB 32x32 pieces (cb, ib) of the unit.
    // Reduced precision with 64-row units: all four pieces are loaded at the start of
    // the unit, so their HBM latency overlaps the contraction (the accumulators take
    // only 64 registers there). Otherwise a piece's loads are issued one or two pieces
    // ahead, overlapping the arithmetic and stores of the pieces before it.
    // Split form: the one piece the wavefront finishes is loaded before the contraction.
    constexpr int kPieces = 2 * RB;
    constexpr bool kDelta = MODE == kBF16 || MODE == kFP16;  // W^t = W^{t-1} + delta
    constexpr bool kEarly = kDelta && RB == 2 && !KS;
    constexpr int kAhead = KS ? 1 : (kEarly ? kPieces : (RB == 4 ? 1 : 2));  // pieces of U/Q loads in flight
    float rsum[kRpu];
#pragma unroll
    for (int r = 0; r < kRpu; ++r) rsum[r] = 0.f;
    // bw: W of a piece (four float4); bu: U (four float4 in FP32, two raw chunks in BF16)
    float4 bw[kAhead][4];
    typedef typename std::conditional<UB == 4, float4[4], uint4[2]>::type UPiece;
    UPiece bu[kAhead];
    auto load_piece = [&](int pc, int slot) {
      const int cb = pc / RB, ib = pc % RB;
      const size_t pidx = ((size_t)lt * (I.bm / 32) + ru * RB + ib) * nkb + c0 / 32 + cb;
      gcfloat4* Wp = gc4(I.W) + pidx * 256 + lane;
#pragma unroll
      for (int g = 0; g < 4; ++g) bw[slot][g] = Wp[g * 64];
      if constexpr (UB == 4) {
        gcfloat4* Up = gc4(I.U) + pidx * 256 + lane;
#pragma unroll
        for (int g = 0; g < 4; ++g) bu[slot][g] = Up[g * 64];
      } else {
        gcuint4* Up = gcu4(I.U) + pidx * 128 + lane;
        bu[slot][0] = Up[0];
        bu[slot][1] = Up[64];
      }
    };
    if constexpr (kEarly) {
#pragma unroll
      for (int i = 0; i < kPieces; ++i) load_piece(i, i);
    }
    if (KS && !init) load_piece(wave, 0);

    floatx16 acc[2][RB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < RB; ++j) acc[i][j] = (floatx16)(0.0f);

    if constexpr (MODE == kFP32) {
    // V fragments: per (column block, offset block) 16 floats per lane in k-step
    // order, consumed in half-steps of 8 k-steps (32 MFMAs). The loop is unrolled by
    // two with ping-pong operand registers: each half-step first issues the V loads
    // and halo reads of the next one and the offset-table read of the one after, then
    // runs its MFMAs on operands fetched a half-step earlier. A halo read costs one
    // add: lane byte address of the row block plus the pre-scaled table entry.
    gcfloat4* vf0 = gc4(a.Vf) + (size_t)(c0 / 32) * nkb * 256 + lane * 4;
    const size_t vstride = (size_t)nkb * 256;
    const char* hb = reinterpret_cast<const char*>(halo);
    const int rb0 = 4 * base[0], rb1 = 4 * base[1];
    const int* tp = offs2 + half * 8;
    float4 va[2][4];
    float bv[2][2][8];
    int4 tb0, tb1;
    auto fetch_v = [&](int h, float4 (&d)[4]) {
      const size_t q = (size_t)(h >> 1) * 256 + (h & 1) * 2;
      d[0] = vf0[q];
      d[1] = vf0[q + 1];
      d[2] = vf0[vstride + q];
      d[3] = vf0[vstride + q + 1];
    };
    auto fetch_t = [&](int h) {
      const int4* t = reinterpret_cast<const int4*>(tp + h * 16);
      tb0 = t[0];
      tb1 = t[1];
    };
    auto fetch_b = [&](float (&d)[2][8]) {
      const int ov[8] = {tb0.x, tb0.y, tb0.z, tb0.w, tb1.x, tb1.y, tb1.z, tb1.w};
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        d[0][jj] = *reinterpret_cast<const float*>(hb + (rb0 + ov[jj]));
        d[1][jj] = *reinterpret_cast<const float*>(hb + (rb1 + ov[jj]));
      }
    };
    auto mfma_half = [&](const float4 (&v)[4], const float (&b)[2][8]) {
      const float a0[8] = {v[0].x, v[0].y, v[0].z, v[0].w, v[1].x, v[1].y, v[1].z, v[1].w};
      const float a1[8] = {v[2].x, v[2].y, v[2].z, v[2].w, v[3].x, v[3].y, v[3].z, v[3].w};
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        acc[0][0] = mfma32(a0[jj], b[0][jj], acc[0][0]);
        acc[0][1] = mfma32(a0[jj], b[1][jj], acc[0][1]);
        acc[1][0] = mfma32(a1[jj], b[0][jj], acc[1][0]);
        acc[1][1] = mfma32(a1[jj], b[1][jj], acc[1][1]);
      }
    };
    // the range [hs0, hs1) has an even length (kp is a multiple of 64, of 128 in the
    // split form); fetches past its last half-step are clamped to it, which keeps the
    // body branch-free
    fetch_t(hs0);
    fetch_b(bv[0]);
    fetch_v(hs0, va[0]);
    fetch_t(hs0 + 1);
    // (the scheduling barriers keep the compiler from sinking the fetches below the
    // MFMAs that do not depend on them)
    for (int h = hs0; h < hs1; h += 2) {
      fetch_v(h + 1, va[1]);
      fetch_b(bv[1]);
      fetch_t(min(h + 2, hs1 - 1));
      __builtin_amdgcn_sched_barrier(0);
      mfma_half(va[0], bv[0]);
      __builtin_amdgcn_sched_barrier(0);
      fetch_v(min(h + 2, hs1 - 1), va[0]);
      fetch_b(bv[0]);
      fetch_t(min(h + 3, hs1 - 1));
      __builtin_amdgcn_sched_barrier(0);
      mfma_half(va[1], bv[1]);
      __builtin_amdgcn_sched_barrier(0);
    }
    } else {
    // reduced precision: one MFMA per (column block, row block) and 16 kernel offsets;
    // A = V (16 bytes per lane, prepacked), B = four-offset runs of D from the
    // expanded halo (two 8-byte LDS reads per row block)
    typedef typename LowP<MODE>::v8 V8;
    typedef typename LowP<MODE>::v4 V4;
    const V4* e4 = reinterpret_cast<const V4*>(halo);
    // The V fragments come from L2 with a latency of many k-steps (four MFMAs each):
    // they are loaded kPf steps ahead into a ring of registers; the LDS reads of D run
    // one step ahead. Each step issues its MFMAs first and then refills the ring slot
    // and the halo buffer it has just consumed, so the loads land in the registers
    // the step read (no copies, exact wait counts). The range [hs0, hs1) has a multiple
    // of kPf steps (kp is a multiple of 64, of 256 in the split form).
    // Split BF16 (kX3): L in three parts (l0 + l1 + l2), V in two (v0 + v1); five
    // MFMAs per step and block, the small terms first: l1 v1, l2 v0, l0 v1, l1 v0,
    // l0 v0 (dropped: l2 v1, 2^-27 relative). Splitting L in two parts only leaves a
    // 2^-18 relative error in each refresh that shows in the solution (W's trailing
    // eigendirections are small sums of large terms); V's 2^-18 is a fixed
    // perturbation of V and does not.
    constexpr bool kX = MODE == kX3;
    constexpr int kPf = (RB == 4 || kX) ? 2 : 4;  // eight (twenty) MFMAs per step
    typedef typename LowP<MODE>::gv8 GV8;
    GV8* vf0 = reinterpret_cast<GV8*>(gc4(kX ? a.Vf_x : a.Vf_lo)) + (size_t)(c0 / 32) * nhs * 64 + lane;
    GV8* vf1 = vf0 + (size_t)nhs * 64;
    const size_t vtail = (size_t)kp * kp / 8;  // the tails follow the heads (in V8)
    const V4* e4m = e4 + E123;                 // middle-part halo
    const V4* e4t = e4 + 2 * E123;             // tail halo
    V8 ra[kPf][2], rt[kX ? kPf : 1][2];
    V4 bn[2][RB][2];  // [step parity][row block][offset run]
    V4 bm[kX ? 2 : 1][RB][2], bt[kX ? 2 : 1][RB][2];
    auto load_d = [&](int kk, int slot) {
      const int2 ot = *reinterpret_cast<const int2*>(offs2 + kk * 4 + half * 2);
#pragma unroll
      for (int ib = 0; ib < RB; ++ib) {
        bn[slot][ib][0] = e4[base[ib] - ot.x];
        bn[slot][ib][1] = e4[base[ib] - ot.y];
        if constexpr (kX) {
          bm[slot][ib][0] = e4m[base[ib] - ot.x];
          bm[slot][ib][1] = e4m[base[ib] - ot.y];
          bt[slot][ib][0] = e4t[base[ib] - ot.x];
          bt[slot][ib][1] = e4t[base[ib] - ot.y];
        }
      }
    };
#pragma unroll
    for (int i = 0; i < kPf; ++i) {
      ra[i][0] = vf0[(size_t)(hs0 + i) * 64];
      ra[i][1] = vf1[(size_t)(hs0 + i) * 64];
      if constexpr (kX) {
        rt[i][0] = vf0[vtail + (size_t)(hs0 + i) * 64];
        rt[i][1] = vf1[vtail + (size_t)(hs0 + i) * 64];
      }
    }
    load_d(hs0, 0);
    for (int kb = hs0; kb < hs1; kb += kPf) {
#pragma unroll
      for (int i = 0; i < kPf; ++i) {
        const int kk = kb + i, cur = i & 1;
        V8 bv[RB], bmv[kX ? RB : 1], btv[kX ? RB : 1];
#pragma unroll
        for (int ib = 0; ib < RB; ++ib)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            bv[ib][j] = bn[cur][ib][0][j];
            bv[ib][4 + j] = bn[cur][ib][1][j];
            if constexpr (kX) {
              bmv[ib][j] = bm[cur][ib][0][j];
              bmv[ib][4 + j] = bm[cur][ib][1][j];
              btv[ib][j] = bt[cur][ib][0][j];
              btv[ib][4 + j] = bt[cur][ib][1][j];
            }
          }
        // the halo reads of the next step go to the other parity buffer
        load_d(min(kk + 1, hs1 - 1), cur ^ 1);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int ib = 0; ib < RB; ++ib) {
            if constexpr (kX) {
              acc[cb][ib] = LowP<MODE>::mfma(rt[i][cb], bmv[ib], acc[cb][ib]);
              acc[cb][ib] = LowP<MODE>::mfma(ra[i][cb], btv[ib], acc[cb][ib]);
              acc[cb][ib] = LowP<MODE>::mfma(rt[i][cb], bv[ib], acc[cb][ib]);
              acc[cb][ib] = LowP<MODE>::mfma(ra[i][cb], bmv[ib], acc[cb][ib]);
            }
            acc[cb][ib] = LowP<MODE>::mfma(ra[i][cb], bv[ib], acc[cb][ib]);
          }
        __builtin_amdgcn_sched_barrier(0);
        // unconditional (clamped) refill keeps the body branch-free; the last steps
        // reload the final fragments harmlessly
        const int kn = min(kk + kPf, hs1 - 1);
        ra[i][0] = vf0[(size_t)kn * 64];
        ra[i][1] = vf1[(size_t)kn * 64];
        if constexpr (kX) {
          rt[i][0] = vf0[vtail + (size_t)kn * 64];
          rt[i][1] = vf1[vtail + (size_t)kn * 64];
        }
      }
    }
    }

    if constexpr (KS) {
      // the partial sums of the pieces the wavefront does not finish go to LDS (slot
      // 3 pc + rank of the wavefront among the other three); the owner of piece pc
      // (wavefront pc) adds the four partials in wavefront order
#pragma unroll
      for (int pc = 0; pc < kPieces; ++pc)
        if (pc != wave) {
          float* d = kred + (3 * pc + (wave < pc ? wave : wave - 1)) * 1024 + lane;
#pragma unroll
          for (int v = 0; v < 16; ++v) d[v * 64] = acc[pc / RB][pc % RB][v];
        }
      __syncthreads();
#pragma unroll
      for (int pc = 0; pc < kPieces; ++pc)
        if (pc == wave) {
          floatx16 sum = (floatx16)(0.0f);
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            if (w == pc) {
              sum += acc[pc / RB][pc % RB];
            } else {
              const float* d = kred + (3 * pc + (w < pc ? w : w - 1)) * 1024 + lane;
#pragma unroll
              for (int v = 0; v < 16; ++v) sum[v] += d[v * 64];
            }
          }
          acc[pc / RB][pc % RB] = sum;
        }
    }

    // Two compiled forms of the same arithmetic: the first forward of a solve (U = 0,
    // Q = W, nothing loaded) and every later one. FP32: rows past the tensor's end
    // get W = 0; their U and Q are zero from the first forward on, so every value
    // derived from them is zero as well without further masking.
    auto epilogue = [&](auto init_c) {
      constexpr bool kFirst = decltype(init_c)::value;
      if constexpr (!kFirst && !kEarly && !KS) {
#pragma unroll
        for (int i = 0; i < kAhead; ++i) load_piece(i, i);
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        if (KS && cb != wave / RB) continue;  // split form: only the wavefront's own piece
        const int cblk = c0 / 32 + cb;
        float4 s4[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          s4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
          if constexpr (!kFirst) s4[g] = *gc4(I.s + cblk * 32 + g * 8 + half * 4);
        }
        float qs[16], ws[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) qs[v] = ws[v] = 0.f;
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) {
          if (KS && ib != wave % RB) continue;
          const int pc = cb * RB + ib, slot = KS ? 0 : pc % kAhead;
          // the piece's old U, unpacked from BF16 (UB = 2; FP32 U is read in place)
          float u16v[UB == 2 ? 16 : 1];
          float4 wo4[4], uo4[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) wo4[g] = uo4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
          if constexpr (!kFirst) {
#pragma unroll
            for (int g = 0; g < 4; ++g) wo4[g] = bw[slot][g];
            if constexpr (UB == 4) {
#pragma unroll
              for (int g = 0; g < 4; ++g) uo4[g] = bu[slot][g];
            } else {
              u16_unpack(bu[slot][0], uinv_old, u16v);
              u16_unpack(bu[slot][1], uinv_old, u16v + 8);
#pragma unroll
              for (int g = 0; g < 4; ++g) uo4[g] = make_float4(u16v[4 * g], u16v[4 * g + 1], u16v[4 * g + 2], u16v[4 * g + 3]);
            }
            if (!KS && pc + kAhead < kPieces) load_piece(pc + kAhead, slot);
          }
          const size_t pidx = ((size_t)lt * (I.bm / 32) + ru * RB + ib) * nkb + cblk;
          gfloat4* Wp = g4(I.W) + pidx * 256 + lane;
          gfloat4* Up4 = g4(I.U) + pidx * 256 + lane;
          float unv[UB == 2 ? 16 : 1];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const float4 u4 = uo4[g], w4 = wo4[g], sv4 = s4[g];
            const float uo[4] = {u4.x, u4.y, u4.z, u4.w}, wo[4] = {w4.x, w4.y, w4.z, w4.w};
            const float sv[4] = {sv4.x, sv4.y, sv4.z, sv4.w};
            float un[4], wn[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              // Q_old = W_old - U_old; Z = s.Q_old, U = (U_old + Z - W) ratio, Q = W - U;
              // residual (Z - W)^2
              const float qo = wo[e] - uo[e];
              float w, unew;
              if constexpr (kDelta) {
                // W^t = W^{t-1} + A_k(L^t - L^{t-1}) V; this form (masking after the
                // update) schedules better in the HBM-bound reduced-precision kernels
                w = acc[cb][ib][4 * g + e] + wo[e];
                if (!valid[ib]) {
                  w = 0.f;
                  unew = 0.f;
                } else {
                  const float z = sv[e] * qo;
                  unew = ((uo[e] + z) - w) * ratio;
                  const float d = z - w;
                  rsum[ib / 2] += d * d;
                }
              } else {
                w = valid[ib] ? acc[cb][ib][4 * g + e] : 0.f;
                if constexpr (kFirst) {
                  unew = 0.f;
                } else {
                  const float d = sv[e] * qo - w;
                  unew = (uo[e] + d) * ratio;
                  rsum[ib / 2] += d * d;
                }
              }
              // the column norms see Q as the next iteration will derive it
              if constexpr (UB == 2) {
                unew = u16_round(unew, uscale, uinv);
                unv[4 * g + e] = unew;
              }
              const float qnew = w - unew;
              un[e] = unew;
              wn[e] = w;
              qs[4 * g + e] += qnew * qnew;
              ws[4 * g + e] += w * w;
            }
            Wp[g * 64] = make_float4(wn[0], wn[1], wn[2], wn[3]);
            if constexpr (UB == 4) Up4[g * 64] = make_float4(un[0], un[1], un[2], un[3]);
          }
          if constexpr (UB == 2) {
            uint4* Up = reinterpret_cast<uint4*>(I.U) + pidx * 128 + lane;
            Up[0] = u16_pack(unv, uscale);
            Up[64] = u16_pack(unv + 8, uscale);
          }
          // FP32: one piece at a time (keeps the scheduler from hoisting the loads of
          // later pieces, which costs registers)
          if constexpr (!kDelta) __builtin_amdgcn_sched_barrier(0);
          if (KS || (ib & 1)) {  // column partials of one 64-row chunk (32-row block: split)
            int vi;
            const float q = half_sum16(qs, lane, vi);
            const float w = half_sum16(ws, lane, vi);
            if ((lane & 1) == 0) {
              const int col = cc * kColUnit + cb * 32 + acc_col(vi, half);
              const int rc = KS ? ru * RB + ib : ru * kRpu + ib / 2;
              colq[rc * CG + col] = q;
              colw[rc * CG + col] = w;
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) qs[v] = ws[v] = 0.f;
          }
        }
      }
    };
    if (MODE == kFP32 && init) {
      if constexpr (MODE == kFP32) epilogue(std::true_type{});
    } else {
      epilogue(std::false_type{});
    }
#pragma unroll
    for (int r = 0; r < kRpu; ++r) {
      const float rs = wave_sum(rsum[r]);
      if (lane == 0) rred[KS ? u * 4 + wave : (ru * kRpu + r) * ncc + cc] = rs;
    }
    if constexpr (KS) __syncthreads();  // the partial-sum slots are reused by the next unit
    cc += KS ? 1 : 4;
    while (cc >= ncc) {
      cc -= ncc;
      ++ru;
    }
  }
  __syncthreads();
  for (int c = tid; c < CG; c += kThreads) {
    float q = 0.f, w = 0.f;
    for (int rc = 0; rc < ncr; ++rc) {
      q += colq[rc * CG + c];
      w += colw[rc * CG + c];
    }
    // blocks of 64 columns, tile-major within a block: each workgroup writes whole
    // 256-byte runs (column-major over tiles made every value a partial-line write)
    const int C = cg * CG + c;
    const size_t pi = ((size_t)(C >> 6) * I.ntiles + lt) * 64 + (C & 63);
    I.qpart[pi] = q;
    I.wpart[pi] = w;
  }
  if (tid == 0) {
    float r = 0.f;
    for (int u = 0; u < nrc * ncc * (KS ? 4 : 1); ++u) r += rred[u];
    I.rpart[(size_t)lt * a.ncg + cg] = r;
  }
}

// =====================================================================================
// adjoint: T_partial = col2im(H), H = G V^T with G = U + s.Q (= (Y + theta Z)/theta).
// grid = (tiles, kp / 256 offset groups). The units of a workgroup (64 rows x 64
// offsets each, one per wavefront) are processed in rounds of four: each wavefront
// runs its unit's contraction on MFMA over all eigendirections and stores H^T in
// LDS; then every thread gathers, for the box positions it owns, the H entries that
// land on them (t = j - s), in a fixed order. No atomics: the result is
// deterministic and independent of how the work was scheduled.
// =====================================================================================
constexpr int kMaxOwned = 16;     // box positions per thread of the per-unit adjoint (E123 <= 4096)
constexpr int kMaxOwnedBig = 24;  // ... of the large-kernel adjoints (E123 <= 6144)

// col2im gather: thread-owned box position x (box coordinates) receives
// H[j = x - (k - 1) + s][s] for the staged kernel offsets s in [S0, S1) whose row j
// lies inside the tile; Hs[s - S0][row] holds the staged H^T. Fixed order.
template <int CAP, class Desc>
__device__ __forceinline__ void gather_round(const Desc& I, const float* Hs, int hstride, int S0, int S1,
                                             float* tacc) {
  const int k0 = I.k[0], k1 = I.k[1], k2 = I.k[2], k12 = k1 * k2;
  const int E123 = I.E123, E12 = I.E[1] * I.E[2];
#pragma unroll
  for (int i = 0; i < CAP; ++i) {
    const int x = threadIdx.x + i * kThreads;
    if (x >= E123) break;
    const int x0 = x / E12, rem = x - x0 * E12;
    const int x1 = rem / I.E[2], x2 = rem - x1 * I.E[2];
    // s_d in [lo_d, hi_d) keeps j_d = x_d - (k_d - 1) + s_d inside [0, b_d)
    const int lo0 = max(0, k0 - 1 - x0), hi0 = min(k0, k0 - 1 - x0 + I.b[0]);
    const int lo1 = max(0, k1 - 1 - x1), hi1 = min(k1, k1 - 1 - x1 + I.b[1]);
    const int lo2 = max(0, k2 - 1 - x2), hi2 = min(k2, k2 - 1 - x2 + I.b[2]);
    float sum = tacc[i];
    for (int p = max(lo0, S0 / k12); p < hi0 && p * k12 < S1; ++p) {
      const int j0 = x0 - (k0 - 1) + p;
      for (int q = lo1; q < hi1; ++q) {
        const int spq = (p * k1 + q) * k2;
        const int r0 = max(lo2, S0 - spq), r1 = min(hi2, S1 - spq);
        const int jrow = (j0 * I.b[1] + (x1 - (k1 - 1) + q)) * I.b[2] + (x2 - (k2 - 1));
        for (int r = r0; r < r1; ++r) sum += Hs[(spq + r - S0) * hstride + jrow + r];
      }
    }
    tacc[i] = sum;
  }
}

// Adjoint workgroup -> (global tile, offset group). Workgroup w runs on XCD w % 8; the
// nsg workgroups of one tile are placed consecutively on one XCD so that the tile's U
// and Q rows, read by each of them, come from HBM once and from that XCD's L2 after.
// The grid holds 8 * ceil(ntiles / 8) * nsg workgroups; the padding ones exit.
__device__ __forceinline__ bool adjoint_item(const StageArgs& a, int2& tt, int& sg) {
  const int w = blockIdx.x, n = w >> 3;
  sg = n % a.nsg;
  const int tile = (n / a.nsg) * 8 + (w & 7);
  if (tile >= a.ntiles) return false;
  tt = a.tiles[tile];
  return true;
}

// col2im gather specialised for an innermost kernel extent of 4 and an innermost
// tile extent of B2 rows: a thread owns whole box lines (x0, x1) and keeps all
// E2 = B2 + 3 positions of each line in registers. For every kernel pair (p, q) of
// the round whose rows (j0, j1) lie in the tile, the 4 x B2 block
// H[(j0, j1, j2)][(p, q, r)] (contiguous in j2, read as float4) is added along its
// anti-diagonals x2 = j2 + 3 - r. Every position receives its terms in the same
// (p, q, r) order as gather_round, so both give identical sums.
template <int B2, int LMAX, class Desc>
__device__ __forceinline__ void gather_lines(const Desc& I, const float* Hs, int hstride, int S0, int S1,
                                             float (&lacc)[LMAX][B2 + 3]) {
  const int k0 = I.k[0], k1 = I.k[1];
  const int E1 = I.E[1], nl = I.E[0] * E1;
  const int b0 = I.b[0], b1 = I.b[1];
  const int pq0 = S0 >> 2, pq1 = S1 >> 2;  // kernel pairs (p, q) staged this round
#pragma unroll
  for (int li = 0; li < LMAX; ++li) {
    const int l = threadIdx.x + li * kThreads;
    if (l >= nl) break;
    const int x0 = l / E1, x1 = l - x0 * E1;
    const int lo0 = max(0, k0 - 1 - x0), hi0 = min(k0, k0 - 1 - x0 + b0);
    const int lo1 = max(0, k1 - 1 - x1), hi1 = min(k1, k1 - 1 - x1 + b1);
    for (int p = max(lo0, pq0 / k1); p < hi0 && p * k1 < pq1; ++p) {
      const int j0 = x0 - (k0 - 1) + p;
      const int qa = max(lo1, pq0 - p * k1), qb = min(hi1, pq1 - p * k1);
      for (int q = qa; q < qb; ++q) {
        const int j1 = x1 - (k1 - 1) + q;
        const float* h = Hs + ((p * k1 + q) * 4 - S0) * hstride + (j0 * b1 + j1) * B2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int j = 0; j < B2; j += 4) {
            const float4 v = *reinterpret_cast<const float4*>(h + r * hstride + j);
            lacc[li][j + 3 - r] += v.x;
            lacc[li][j + 4 - r] += v.y;
            lacc[li][j + 5 - r] += v.z;
            lacc[li][j + 6 - r] += v.w;
          }
        }
      }
    }
  }
}

// Per-thread col2im accumulators of one adjoint workgroup. GV = 0: box positions, any
// geometry, CAP positions per thread (E123 <= 256 CAP); GV = 8: box lines for an
// innermost kernel extent of 4 and tile rows of 8 along the innermost dimension (at
// most 512 lines). The host picks GV per launch from the plans of the instances it
// covers.
template <int GV, int CAP = kMaxOwned>
struct GatherAcc;

template <int CAP>
struct GatherAcc<0, CAP> {
  float t[CAP];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < CAP; ++i) t[i] = 0.f;
  }
  template <class Desc>
  __device__ __forceinline__ void round(const Desc& I, const float* Hs, int hstride, int S0, int S1) {
    gather_round<CAP>(I, Hs, hstride, S0, S1, t);
  }
  template <class Desc>
  __device__ __forceinline__ void store(const Desc& I, float* dst) const {
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
      const int x = threadIdx.x + i * kThreads;
      if (x >= I.E123) break;
      dst[x] = t[i];
    }
  }
};

template <int CAP>
struct GatherAcc<8, CAP> {
  static constexpr int kLines = 2, kE2 = 8 + 3;
  float t[kLines][kE2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < kLines; ++i)
#pragma unroll
      for (int j = 0; j < kE2; ++j) t[i][j] = 0.f;
  }
  template <class Desc>
  __device__ __forceinline__ void round(const Desc& I, const float* Hs, int hstride, int S0, int S1) {
    gather_lines<8, kLines>(I, Hs, hstride, S0, S1, t);
  }
  template <class Desc>
  __device__ __forceinline__ void store(const Desc& I, float* dst) const {
    const int nl = I.E[0] * I.E[1];
#pragma unroll
    for (int i = 0; i < kLines; ++i) {
      const int l = threadIdx.x + i * kThreads;
      if (l >= nl) break;
#pragma unroll
      for (int j = 0; j < kE2; ++j) dst[l * kE2 + j] = t[i][j];
    }
  }
};

// Loads of the state for the adjoint's G: the eight values 8p..8p+7 of one lane (the
// float4 groups 2p and 2p + 1 of the tile layout) of W and of U for the piece at piece
// index pidx, kept as loaded (U in its stored width); split_uq8 then returns U and
// Q = W - U. The two steps are apart so that a prefetch's values are first used, and
// waited for, only where they are consumed, not right after the loads are issued.
template <int UB>
struct UQ8 {
  float4 w[2];
  typename std::conditional<UB == 4, float4[2], uint4>::type u;
};

template <int UB, class Desc>
__device__ __forceinline__ void load_uq8(const Desc& I, size_t pidx, int p, int lane, UQ8<UB>& r) {
  gcfloat4* W4 = gc4(I.W) + pidx * 256 + 2 * p * 64 + lane;
  r.w[0] = W4[0];
  r.w[1] = W4[64];
  if constexpr (UB == 4) {
    gcfloat4* U4 = gc4(I.U) + pidx * 256 + 2 * p * 64 + lane;
    r.u[0] = U4[0];
    r.u[1] = U4[64];
  } else {
    r.u = gcu4(I.U)[pidx * 128 + p * 64 + lane];
  }
}

template <int UB>
__device__ __forceinline__ void split_uq8(const UQ8<UB>& r, float uinv, float4 (&u)[2], float4 (&q)[2]) {
  if constexpr (UB == 4) {
    u[0] = r.u[0];
    u[1] = r.u[1];
  } else {
    float v[8];
    u16_unpack(r.u, uinv, v);
    u[0] = make_float4(v[0], v[1], v[2], v[3]);
    u[1] = make_float4(v[4], v[5], v[6], v[7]);
  }
  const float4 w0 = r.w[0], w1 = r.w[1];
  q[0] = make_float4(w0.x - u[0].x, w0.y - u[0].y, w0.z - u[0].z, w0.w - u[0].w);
  q[1] = make_float4(w1.x - u[1].x, w1.y - u[1].y, w1.z - u[1].z, w1.w - u[1].w);
}

template <int MODE, int GV, int UB, bool KS>
__global__ __launch_bounds__(kThreads, 2) void k_adjoint(StageArgs a) {
  extern __shared__ float smem[];
  int2 tt;
  int sg;
  if (!adjoint_item(a, tt, sg)) return;
  // constant descriptor (see k_forward) with the line gather; the position gather keeps
  // the generic one (with constant fields its per-thread accumulators spill)
  typedef typename std::conditional<GV == 8, const CInstDev, const InstDev>::type Desc;
  Desc& I = *(Desc*)(a.inst + tt.x);
  if (I.st->phase != kRun || !runs_iteration<MODE>(I, I.st, a.rx3)) return;
  const int kp = a.kp, k = a.k;
  const int SGW = KS ? kColUnit : (kp < kGroup ? kp : kGroup);
  const int lt = tt.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), half = lane >> 5;
  const int bm = I.bm;
  const int nrc = bm / kRowUnit, nsc = SGW / kColUnit;
  const int units = nrc * nsc;
  const int rounds = (units >= 4 && !KS) ? units / 4 : 1;  // four units per round (fewer when small)
  const int spr = (SGW / rounds);             // kernel offsets per round
  const int hstride = bm + 4;                 // LDS row stride of the staged H^T
  float* Hs = smem;                           // [spr][hstride]
  float* kred = Hs + spr * hstride;           // split: [12][16][64] partial sums

  // owned box positions and their valid kernel-offset ranges per dimension
  const int E123 = I.E123;
  GatherAcc<GV> gacc;
  gacc.zero();

  const int nkb = kp / 32;
  const int nhb = 2 * nkb;  // half column blocks of 8 MFMA k-steps
  const float* S = I.s;
  const float uinv = (float)(1.0 / I.st->theta_cur);  // 16-bit U: see u16_unpack
  // the eigendirection half blocks this wavefront contracts
  const int hb0 = KS ? wave * (nhb / 4) : 0, hb1 = KS ? hb0 + nhb / 4 : nhb;
  for (int rd = 0; rd < rounds; ++rd) {
    const int S0 = sg * SGW + rd * spr;      // first offset staged this round
    for (int ui = 0; ui < (KS ? nrc : 1); ++ui) {
    const int u = KS ? ui : rd * 4 + wave;
    const int rc = u % nrc, sc = u / nrc;    // a round covers whole offset chunks
    const int s0 = sg * SGW + sc * kColUnit;
    if (u < units) {
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = (floatx16)(0.0f);
    if constexpr (MODE == kFP32) {
    gcfloat4* va0 = gc4(a.Va) + (size_t)(s0 / 32) * nkb * 256 + lane * 4;
    gcfloat4* va1 = va0 + (size_t)nkb * 256;
    const size_t row0 = ((size_t)lt * (bm / 32) + rc * 2) * nkb;  // row group jb: (row0 + jb * nkb + cb)
    // operands of half block h (column block cb = h/2, part p = h%2); each iteration
    // consumes the loads of the previous one before issuing its own
    UQ8<UB> fr[2];
    float4 fs[2], fv[2][2];
    auto load = [&](int h) {
      const int cb = h >> 1, p = h & 1;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) load_uq8<UB>(I, row0 + (size_t)jb * nkb + cb, p, lane, fr[jb]);
      fs[0] = *gc4(S + cb * 32 + (2 * p) * 8 + half * 4);
      fs[1] = *gc4(S + cb * 32 + (2 * p + 1) * 8 + half * 4);
      const size_t ov = (size_t)cb * 256 + 2 * p;
      fv[0][0] = va0[ov];
      fv[0][1] = va0[ov + 1];
      fv[1][0] = va1[ov];
      fv[1][1] = va1[ov + 1];
    };
    load(hb0);
    for (int h = hb0; h < hb1; ++h) {
      float g[2][8];
      float4 fu[2][2], fq[2][2];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) split_uq8<UB>(fr[jb], uinv, fu[jb], fq[jb]);
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          g[jb][4 * t + 0] = fu[jb][t].x + fs[t].x * fq[jb][t].x;
          g[jb][4 * t + 1] = fu[jb][t].y + fs[t].y * fq[jb][t].y;
          g[jb][4 * t + 2] = fu[jb][t].z + fs[t].z * fq[jb][t].z;
          g[jb][4 * t + 3] = fu[jb][t].w + fs[t].w * fq[jb][t].w;
        }
      }
      const float v0[8] = {fv[0][0].x, fv[0][0].y, fv[0][0].z, fv[0][0].w,
                           fv[0][1].x, fv[0][1].y, fv[0][1].z, fv[0][1].w};
      const float v1[8] = {fv[1][0].x, fv[1][0].y, fv[1][0].z, fv[1][0].w,
                           fv[1][1].x, fv[1][1].y, fv[1][1].z, fv[1][1].w};
      if (h + 1 < hb1) load(h + 1);
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        acc[0][0] = mfma32(v0[jj], g[0][jj], acc[0][0]);
        acc[0][1] = mfma32(v0[jj], g[1][jj], acc[0][1]);
        acc[1][0] = mfma32(v1[jj], g[0][jj], acc[1][0]);
        acc[1][1] = mfma32(v1[jj], g[1][jj], acc[1][1]);
      }
    }
    } else {
    // reduced precision: the contraction runs on the change of G since the previous
    // iteration, dG = G^t - G^{t-1} = (s - 1) Q - U / ratio_prev, and the L-step adds
    // it to the running A_k^*(G V^T)
    typedef typename LowP<MODE>::v8 V8;
    const float rp = (float)(1.0 / I.st->ratio_prev);
    gcuint4* va0 = gcu4(a.Va_lo) + (size_t)(s0 / 32) * nkb * 128 + lane;
    gcuint4* va1 = va0 + (size_t)nkb * 128;
    const size_t row0 = ((size_t)lt * (bm / 32) + rc * 2) * nkb;
    UQ8<UB> fr[2];
    float4 fs[2];
    uint4 fv0, fv1;
    auto load = [&](int h) {
      const int cb = h >> 1, p = h & 1;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) load_uq8<UB>(I, row0 + (size_t)jb * nkb + cb, p, lane, fr[jb]);
      fs[0] = *gc4(S + cb * 32 + (2 * p) * 8 + half * 4);
      fs[1] = *gc4(S + cb * 32 + (2 * p + 1) * 8 + half * 4);
      fv0 = va0[(size_t)h * 64];
      fv1 = va1[(size_t)h * 64];
    };
    load(hb0);
    for (int h = hb0; h < hb1; ++h) {
      V8 g[2];
      float4 fu[2][2], fq[2][2];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) split_uq8<UB>(fr[jb], uinv, fu[jb], fq[jb]);
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          g[jb][4 * t + 0] = (fs[t].x - 1.f) * fq[jb][t].x - fu[jb][t].x * rp;
          g[jb][4 * t + 1] = (fs[t].y - 1.f) * fq[jb][t].y - fu[jb][t].y * rp;
          g[jb][4 * t + 2] = (fs[t].z - 1.f) * fq[jb][t].z - fu[jb][t].z * rp;
          g[jb][4 * t + 3] = (fs[t].w - 1.f) * fq[jb][t].w - fu[jb][t].w * rp;
        }
      }
      V8 v0, v1;
      __builtin_memcpy(&v0, &fv0, 16);
      __builtin_memcpy(&v1, &fv1, 16);
      if (h + 1 < hb1) load(h + 1);
      acc[0][0] = LowP<MODE>::mfma(v0, g[0], acc[0][0]);
      acc[0][1] = LowP<MODE>::mfma(v0, g[1], acc[0][1]);
      acc[1][0] = LowP<MODE>::mfma(v1, g[0], acc[1][0]);
      acc[1][1] = LowP<MODE>::mfma(v1, g[1], acc[1][1]);
    }
    }
    if constexpr (KS) {
      // partial sums of the pieces (sb, jb) = (pc / 2, pc % 2) the wavefront does not
      // stage go to LDS; the owner (wavefront pc) adds the four in wavefront order
#pragma unroll
      for (int pc = 0; pc < 4; ++pc)
        if (pc != wave) {
          float* d = kred + (3 * pc + (wave < pc ? wave : wave - 1)) * 1024 + lane;
#pragma unroll
          for (int v = 0; v < 16; ++v) d[v * 64] = acc[pc / 2][pc % 2][v];
        }
      __syncthreads();
#pragma unroll
      for (int pc = 0; pc < 4; ++pc)
        if (pc == wave) {
          floatx16 sum = (floatx16)(0.0f);
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            if (w == pc) {
              sum += acc[pc / 2][pc % 2];
            } else {
              const float* d = kred + (3 * pc + (w < pc ? w : w - 1)) * 1024 + lane;
#pragma unroll
              for (int v = 0; v < 16; ++v) sum[v] += d[v * 64];
            }
          }
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int sl = s0 + (pc / 2) * 32 + acc_col(v, half) - S0;
            Hs[sl * hstride + rc * 64 + (pc % 2) * 32 + (lane & 31)] = sum[v];
          }
        }
      __syncthreads();  // the partial-sum slots are reused by the next unit
    } else {
    // stage H^T of this unit: Hs[s - S0][row]
#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int sl = s0 + sb * 32 + acc_col(v, half) - S0;
          Hs[sl * hstride + rc * 64 + jb * 32 + (lane & 31)] = acc[sb][jb][v];
        }
    }
    }
    }
    __syncthreads();
    gacc.round(I, Hs, hstride, S0, min(S0 + spr, k));
    __syncthreads();
  }
  gacc.store(I, I.part + ((size_t)lt * a.nsg + sg) * E123);
}

// =====================================================================================
// adjoint for large kernels (kp >= 512): the same contraction and col2im, tiled for
// operand reuse. A workgroup computes H^T for 128 tile rows x 256 kernel offsets over
// all eigendirections; chunks of 16 eigendirections of G (formed from U, Q, s) and of
// V are staged cooperatively in LDS (double buffered) and each wavefront computes
// 64 rows x 128 offsets (eight 32x32 accumulators), so every G element is fetched once
// per workgroup and every V element once per workgroup. The col2im then runs in two
// rounds of 128 offsets through the shared gather.
// =====================================================================================
constexpr int kBigChunk = 16;            // eigendirections per staged chunk
constexpr int kBigPad = kBigChunk + 1;   // LDS row stride (odd: conflict-free columns)

template <int GV, int UB>
__global__ __launch_bounds__(kThreads, 2) void k_adjoint_big(StageArgs a) {
  extern __shared__ float smem[];
  int2 tt;
  int sg;
  if (!adjoint_item(a, tt, sg)) return;
  // constant descriptor (see k_forward) with the line gather; the position gather keeps
  // the generic one (with constant fields its per-thread accumulators spill)
  typedef typename std::conditional<GV == 8, const CInstDev, const InstDev>::type Desc;
  Desc& I = *(Desc*)(a.inst + tt.x);
  if (I.st->phase != kRun || !runs_iteration<kFP32>(I, I.st, a.rx3)) return;
  const int kp = a.kp, k = a.k;
  const int lt = tt.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), half = lane >> 5;
  const int nkb = kp / 32;
  const int rw = wave & 1, sh = wave >> 1;             // row chunk, offset half
  float* Gs = smem;                                    // [2][128][kBigPad]
  float* Vs = smem + 2 * 128 * kBigPad;                // [2][256][kBigPad]
  GatherAcc<GV, kMaxOwnedBig> gacc;
  gacc.zero();

  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (floatx16)(0.0f);

  // cooperative share of a chunk: thread t stages G for (row group t/64, lane t%64)
  // of the tile layout (8 values) and V row s = t of this offset group (16 values)
  const int rg = tid >> 6, hf = (tid >> 5) & 1;
  const float uinv = (float)(1.0 / I.st->theta_cur);  // 16-bit U: see u16_unpack
  const float* vrow = a.Vp + (size_t)(sg * kGroup + tid) * kp;
  // two register slots: the loads of chunk q + 2 are issued while chunk q is
  // contracted, so each chunk's global loads have two contraction phases to land
  UQ8<UB> cr[2];
  float4 cs[2][2], cv[2][4];  // [slot][...]
  auto coop_load = [&](int q, int sl) {
    const int cb = q >> 1, p = q & 1;
    load_uq8<UB>(I, ((size_t)lt * 4 + rg) * nkb + cb, p, lane, cr[sl]);
    cs[sl][0] = *gc4(I.s + cb * 32 + (2 * p) * 8 + hf * 4);
    cs[sl][1] = *gc4(I.s + cb * 32 + (2 * p + 1) * 8 + hf * 4);
    gcfloat4* vp = gc4(vrow + q * kBigChunk);
#pragma unroll
    for (int i = 0; i < 4; ++i) cv[sl][i] = vp[i];
  };
  auto coop_store = [&](int buf, int sl) {
    // G values of v = 8p..8p+7 sit at chunk columns (v%8/4)*8 + hf*4 + v%4
    float* gd = Gs + ((size_t)buf * 128 + rg * 32 + (lane & 31)) * kBigPad + hf * 4;
    float4 cu[2], cq[2];
    split_uq8<UB>(cr[sl], uinv, cu, cq);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      gd[8 * t + 0] = cu[t].x + cs[sl][t].x * cq[t].x;
      gd[8 * t + 1] = cu[t].y + cs[sl][t].y * cq[t].y;
      gd[8 * t + 2] = cu[t].z + cs[sl][t].z * cq[t].z;
      gd[8 * t + 3] = cu[t].w + cs[sl][t].w * cq[t].w;
    }
    float* vd = Vs + ((size_t)buf * 256 + tid) * kBigPad;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      vd[4 * i + 0] = cv[sl][i].x;
      vd[4 * i + 1] = cv[sl][i].y;
      vd[4 * i + 2] = cv[sl][i].z;
      vd[4 * i + 3] = cv[sl][i].w;
    }
  };
  const int nq = kp / kBigChunk;  // even (kp is a multiple of 256)
  coop_load(0, 0);
  coop_load(1, 1);
  coop_store(0, 0);
  __syncthreads();
  for (int q0 = 0; q0 < nq; q0 += 2) {
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int q = q0 + sl;
      // slot sl held chunk q, already in LDS: refill it with chunk q + 2 (clamped, so
      // the body stays branch-free; the last chunks reload harmlessly)
      coop_load(min(q + 2, nq - 1), sl);
      const float* gb = Gs + ((size_t)sl * 128 + rw * 64 + (lane & 31)) * kBigPad + half;
      const float* vb = Vs + ((size_t)sl * 256 + sh * 128 + (lane & 31)) * kBigPad + half;
#pragma unroll
      for (int kk = 0; kk < kBigChunk / 2; ++kk) {
        const float g0 = gb[2 * kk], g1 = gb[32 * kBigPad + 2 * kk];
        float v[4];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) v[sb] = vb[sb * 32 * kBigPad + 2 * kk];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
          acc[sb][0] = mfma32(v[sb], g0, acc[sb][0]);
          acc[sb][1] = mfma32(v[sb], g1, acc[sb][1]);
        }
      }
      if (q + 1 < nq) coop_store(sl ^ 1, sl ^ 1);
      __syncthreads();
    }
  }
  const int hstride = 128 + 4;
  float* Hs = smem;
  for (int rd = 0; rd < 2; ++rd) {
    const int S0 = sg * kGroup + rd * 128;
    if (sh == rd) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
          for (int v = 0; v < 16; ++v)
            Hs[(sb * 32 + acc_col(v, half)) * hstride + rw * 64 + jb * 32 + (lane & 31)] = acc[sb][jb][v];
    }
    __syncthreads();
    gacc.round(I, Hs, hstride, S0, min(S0 + 128, k));
    __syncthreads();
  }
  gacc.store(I, I.part + ((size_t)lt * a.nsg + sg) * I.E123);
}

// Reduced-precision variant of the tiled large-kernel adjoint: chunks of 32
// eigendirections, dG = (s - 1) Q - U / ratio_prev converted to BF16/FP16 when
// staged, V read from its zero-padded BF16/FP16 copy, 32x32x16 MFMA (two k-steps per
// chunk) with FP32 accumulation. LDS rows are 40 halves (80 bytes): 16-byte vector
// reads of eight consecutive rows then fall on distinct banks.
constexpr int kBigLpChunk = 32;
constexpr int kBigLpPad = kBigLpChunk + 8;
// floats of LDS before the shrink factors: the staging buffers or the staged H^T
constexpr int kBigLpStage = (2 * (128 + 256) * kBigLpPad / 2 > 128 * (128 + 4)) ? 2 * (128 + 256) * kBigLpPad / 2
                                                                                  : 128 * (128 + 4);
// split-BF16 refresh (MODE kX3): G = U + s.Q formed in FP32 and staged in three BF16
// parts (g0 + g1 + g2), V in two (v0 + v1); five MFMAs per product, the small terms
// first: g1 v1, g2 v0, g0 v1, g1 v0, g0 v0 (one workgroup per compute unit)
// (single-buffered: two workgroups per CU)
constexpr int kBigX3Stage = ((3 * 128 + 2 * 256) * kBigLpPad / 2 > 128 * (128 + 4)) ? (3 * 128 + 2 * 256) * kBigLpPad / 2
                                                                                    : 128 * (128 + 4);

template <int MODE, int GV>
__global__ __launch_bounds__(kThreads, 2) void k_adjoint_big_lp(StageArgs a) {
  typedef typename LowP<MODE>::h H;
  typedef typename LowP<MODE>::v8 V8;
  typedef typename LowP<MODE>::v4 V4;
  extern __shared__ float smem[];
  int2 tt;
  int sg;
  if (!adjoint_item(a, tt, sg)) return;
  // constant descriptor (see k_forward) with the line gather; the position gather keeps
  // the generic one (with constant fields its per-thread accumulators spill)
  typedef typename std::conditional<GV == 8, const CInstDev, const InstDev>::type Desc;
  Desc& I = *(Desc*)(a.inst + tt.x);
  if (I.st->phase != kRun || !runs_iteration<MODE>(I, I.st, a.rx3)) return;
  const int kp = a.kp, k = a.k;
  const int lt = tt.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), half = lane >> 5;
  const int nkb = kp / 32;
  const int rw = wave & 1, sh = wave >> 1;
  constexpr bool kX = MODE == kX3;
  constexpr int kNB = kX ? 1 : 2;                      // staging buffers
  H* Gs = reinterpret_cast<H*>(smem);                  // [kNB][128][kBigLpPad]
  H* Vs = Gs + kNB * 128 * kBigLpPad;                  // [kNB][256][kBigLpPad]
  H* Gm = Vs + kNB * 256 * kBigLpPad;                  // kX3: G middle parts [1][128][kBigLpPad]
  H* Gt = Gm + kNB * 128 * kBigLpPad;                  //      G tails [1][128][kBigLpPad]
  H* Vt = Gt + kNB * 128 * kBigLpPad;                  //      V tails [1][256][kBigLpPad]
  float* Ss = smem + (kX ? kBigX3Stage : kBigLpStage);  // shrink factors [kp]
  for (int c = threadIdx.x; c < kp; c += kThreads) Ss[c] = I.s[c];
  GatherAcc<GV, kMaxOwnedBig> gacc;
  gacc.zero();
  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (floatx16)(0.0f);

  const float rp = (float)(1.0 / I.st->ratio_prev);
  const float uinv = (float)(1.0 / I.st->theta_cur);  // 16-bit U: see u16_unpack
  const int rg = tid >> 6, hf = (tid >> 5) & 1;
  // thread t stages G of (row group t/64, lane t%64) of the tile layout (16 values)
  // and a quarter (16 bytes) of four V rows of this offset group: instruction i of
  // wavefront w covers rows w * 64 + 16 i .. + 15 whole, 64 contiguous bytes each
  const int vr = wave * 64 + (lane >> 2), vf = lane & 3;
  gcfloat4* vrow = gc4(kX ? a.Vp_x : a.Vp_lo) + (size_t)(sg * kGroup + vr) * (kp / 8) + vf;
  const size_t vstep = (size_t)16 * (kp / 8);
  const size_t vtail = (size_t)kp * kp / 8;  // kX3: the tails follow the heads (in float4)
  // G (from HBM) is prefetched two chunks ahead in two register slots, V (mostly from
  // L2) one chunk ahead: chunk q + 2's state is loaded while chunk q is contracted
  UQ8<2> cr[2][2];  // [slot][part]
  float4 cv0, cv1, cv2, cv3, ct0, ct1, ct2, ct3;  // ct: kX3 tails
  auto load_g = [&](int cb, int sl) {
    const size_t pidx = ((size_t)lt * 4 + rg) * nkb + cb;
    load_uq8<2>(I, pidx, 0, lane, cr[sl][0]);
    load_uq8<2>(I, pidx, 1, lane, cr[sl][1]);
  };
  auto load_v = [&](int cb) {
    cv0 = vrow[cb * 4];
    cv1 = vrow[vstep + cb * 4];
    cv2 = vrow[2 * vstep + cb * 4];
    cv3 = vrow[3 * vstep + cb * 4];
    if constexpr (kX) {
      ct0 = vrow[vtail + cb * 4];
      ct1 = vrow[vtail + vstep + cb * 4];
      ct2 = vrow[vtail + 2 * vstep + cb * 4];
      ct3 = vrow[vtail + 3 * vstep + cb * 4];
    }
  };
  auto coop_store = [&](int buf, int cb, int sl) {
    // value v = 4g + e of the tile layout sits at column acc_col(v, hf) = 8g + 4hf + e
    if constexpr (kX) buf = 0;
    H* gd = Gs + ((size_t)buf * 128 + rg * 32 + (lane & 31)) * kBigLpPad + hf * 4;
    float4 cu[4], cq[4];
    split_uq8<2>(cr[sl][0], uinv, reinterpret_cast<float4(&)[2]>(cu[0]), reinterpret_cast<float4(&)[2]>(cq[0]));
    split_uq8<2>(cr[sl][1], uinv, reinterpret_cast<float4(&)[2]>(cu[2]), reinterpret_cast<float4(&)[2]>(cq[2]));
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 sv = *reinterpret_cast<const float4*>(Ss + cb * 32 + g * 8 + hf * 4);
      V4 t;
      if constexpr (kX) {
        const float gv[4] = {cu[g].x + sv.x * cq[g].x, cu[g].y + sv.y * cq[g].y, cu[g].z + sv.z * cq[g].z,
                             cu[g].w + sv.w * cq[g].w};
        V4 tm4, tt4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          t[e] = (H)gv[e];
          const float r = gv[e] - (float)t[e];
          tm4[e] = (H)r;
          tt4[e] = (H)(r - (float)tm4[e]);
        }
        *reinterpret_cast<V4*>(gd + (Gm - Gs) + 8 * g) = tm4;
        *reinterpret_cast<V4*>(gd + (Gt - Gs) + 8 * g) = tt4;
      } else {
        t[0] = (H)((sv.x - 1.f) * cq[g].x - cu[g].x * rp);
        t[1] = (H)((sv.y - 1.f) * cq[g].y - cu[g].y * rp);
        t[2] = (H)((sv.z - 1.f) * cq[g].z - cu[g].z * rp);
        t[3] = (H)((sv.w - 1.f) * cq[g].w - cu[g].w * rp);
      }
      *reinterpret_cast<V4*>(gd + 8 * g) = t;
    }
    float4* vd = reinterpret_cast<float4*>(Vs + ((size_t)buf * 256 + vr) * kBigLpPad) + vf;
    const int rs = 16 * kBigLpPad / 8;  // float4s per 16 rows
    vd[0] = cv0;
    vd[rs] = cv1;
    vd[2 * rs] = cv2;
    vd[3 * rs] = cv3;
    if constexpr (kX) {
      float4* vtd = vd + (Vt - Vs) / 8;
      vtd[0] = ct0;
      vtd[rs] = ct1;
      vtd[2 * rs] = ct2;
      vtd[3 * rs] = ct3;
    }
  };
  load_g(0, 0);
  load_v(0);
  load_g(min(1, nkb - 1), 1);
  __syncthreads();
  coop_store(0, 0, 0);
  __syncthreads();
  // nkb is even (kp is a multiple of 256): chunk q lives in LDS buffer and G slot q & 1
  for (int q0 = 0; q0 < nkb; q0 += 2) {
#pragma unroll
    for (int buf = 0; buf < 2; ++buf) {
      const int q = q0 + buf;
      // unconditional (indices clamped; the last chunks reload harmlessly): loads under
      // a condition would leave the wait counts path-dependent, and the compiler then
      // waits for every outstanding load, this prefetch included
      load_v(min(q + 1, nkb - 1));
      // (V first: loads complete in issue order, so the wait for V(q + 1) before the
      // end-of-step store must not also wait for the G loads of chunk q + 2)
      __builtin_amdgcn_sched_barrier(0);
      load_g(min(q + 2, nkb - 1), buf);  // slot buf held chunk q, already in LDS
      const int lb = kX ? 0 : buf;  // LDS buffer of chunk q
      const H* gb = Gs + ((size_t)lb * 128 + rw * 64 + (lane & 31)) * kBigLpPad + 8 * half;
      const H* vb = Vs + ((size_t)lb * 256 + sh * 128 + (lane & 31)) * kBigLpPad + 8 * half;
#pragma unroll
      for (int kk = 0; kk < kBigLpChunk / 16; ++kk) {
        const V8 g0 = *reinterpret_cast<const V8*>(gb + 16 * kk);
        const V8 g1 = *reinterpret_cast<const V8*>(gb + 32 * kBigLpPad + 16 * kk);
        V8 v[4];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) v[sb] = *reinterpret_cast<const V8*>(vb + sb * 32 * kBigLpPad + 16 * kk);
        if constexpr (kX) {
          const H* gmb = gb + (Gm - Gs);
          const H* gtb = gb + (Gt - Gs);
          const H* vtb = vb + (Vt - Vs);
          const V8 m0 = *reinterpret_cast<const V8*>(gmb + 16 * kk);
          const V8 m1 = *reinterpret_cast<const V8*>(gmb + 32 * kBigLpPad + 16 * kk);
          const V8 t0 = *reinterpret_cast<const V8*>(gtb + 16 * kk);
          const V8 t1 = *reinterpret_cast<const V8*>(gtb + 32 * kBigLpPad + 16 * kk);
#pragma unroll
          for (int sb = 0; sb < 4; ++sb) {
            const V8 vt = *reinterpret_cast<const V8*>(vtb + sb * 32 * kBigLpPad + 16 * kk);
            acc[sb][0] = LowP<MODE>::mfma(vt, m0, acc[sb][0]);
            acc[sb][1] = LowP<MODE>::mfma(vt, m1, acc[sb][1]);
            acc[sb][0] = LowP<MODE>::mfma(v[sb], t0, acc[sb][0]);
            acc[sb][1] = LowP<MODE>::mfma(v[sb], t1, acc[sb][1]);
            acc[sb][0] = LowP<MODE>::mfma(vt, g0, acc[sb][0]);
            acc[sb][1] = LowP<MODE>::mfma(vt, g1, acc[sb][1]);
            acc[sb][0] = LowP<MODE>::mfma(v[sb], m0, acc[sb][0]);
            acc[sb][1] = LowP<MODE>::mfma(v[sb], m1, acc[sb][1]);
          }
        }
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
          acc[sb][0] = LowP<MODE>::mfma(v[sb], g0, acc[sb][0]);
          acc[sb][1] = LowP<MODE>::mfma(v[sb], g1, acc[sb][1]);
        }
      }
      if constexpr (kX) __syncthreads();  // single buffer: every wavefront is done with it
      if (q + 1 < nkb) coop_store(buf ^ 1, q + 1, buf ^ 1);
      __syncthreads();
    }
  }
  const int hstride = 128 + 4;
  float* Hs = smem;
  for (int rd = 0; rd < 2; ++rd) {
    const int S0 = sg * kGroup + rd * 128;
    if (sh == rd) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
          for (int v = 0; v < 16; ++v)
            Hs[(sb * 32 + acc_col(v, half)) * hstride + rw * 64 + jb * 32 + (lane & 31)] = acc[sb][jb][v];
    }
    __syncthreads();
    gacc.round(I, Hs, hstride, S0, min(S0 + 128, k));
    __syncthreads();
  }
  gacc.store(I, I.part + ((size_t)lt * a.nsg + sg) * I.E123);
}

// =====================================================================================
// lstep: T[t] = sum of the halo partials covering t;  L-step of Section III-D.
//   init (phase kInit): L = P_Omega(M), partial sums of ||P_Omega M||^2
//   run: lambda = inf: L = M on Omega, T/k elsewhere;
//        finite lambda: L = (theta T/k + lambda M)/(lambda + theta) on Omega, T/k elsewhere
//        partial sums of ||L_new - L_old||^2
// =====================================================================================
template <int KG>
__global__ __launch_bounds__(kThreads) void k_lstep(StageArgs a) {
  // Workgroup w runs on XCD w % 8; the blocks are dealt so that each XCD takes one
  // contiguous run of them, in order: neighbouring output blocks read adjacent rows of
  // the same tiles' halo partials, so a cache line one block fetches is in that XCD's
  // L2 for the next (results do not depend on the order).
  const int nb8 = (a.nlblocks + 7) >> 3;
  const int lbi = (int)(blockIdx.x & 7) * nb8 + (int)(blockIdx.x >> 3);
  if (lbi >= a.nlblocks) return;
  const int2 lb = a.lblocks[lbi];
  const CInstDev& I = *(const CInstDev*)(a.inst + lb.x);  // constant: see k_forward
  const int phase = I.st->phase;
  if (phase != kInit && phase != kRun) return;
  // kLanesPerElem lanes share one output element; each sums every kLanesPerElem-th
  // covering partial in a fixed order and the lanes combine by shuffles
  const int sub = threadIdx.x & (kLanesPerElem - 1);
  const int64_t t = (int64_t)lb.y * kLStepElems + (threadIdx.x / kLanesPerElem);
  double acc = 0.0, pen = 0.0;
  const bool in = t < I.mtot;
  float T = 0.f;
  int t0 = 0, t1 = 0, t2 = 0;
  if (in) {
    if (I.mtot < (int64_t(1) << 31)) {
      const int t32 = (int)t, r = t32 / I.m[2];
      t2 = t32 - r * I.m[2];
      t0 = r / I.m[1];
      t1 = r - t0 * I.m[1];
    } else {
      t2 = (int)(t % I.m[2]);
      const int64_t r = t / I.m[2];
      t1 = (int)(r % I.m[1]);
      t0 = (int)(r / I.m[1]);
    }
  }
  // the element's own inputs are loaded first, so that their latency overlaps the
  // gather (lanes past the tensor read element 0 and discard it)
  const int64_t tc = in ? t : 0;
  const bool obs = I.mask[tc] != 0;
  const float mv = I.M[tc];
  const float lold = I.L[tc];
  float tprev = 0.f;
  if (I.prec != kFP32) tprev = I.T[tc];
  if (in && phase == kRun) {
    // partials of this iteration's adjoint: the full A_k^*(G V^T), or on a reduced
    // precision iteration its change since the previous one
    const int32_t* g0 = I.gtab + I.goff[0] + t0 * I.C[0];
    const int32_t* g1 = I.gtab + I.goff[1] + t1 * I.C[1];
    const int32_t* g2 = I.gtab + I.goff[2] + t2 * I.C[2];
    const int nsg = a.nsg;
    // lane `sub` takes the (c0, c1) pairs congruent to it modulo kLanesPerElem and
    // sums all c2 and offset groups of each, in a fixed order. The partials come from
    // other workgroups' writes (not in this XCD's L2), so the loads of a pair are all
    // issued before any is summed.
    const int C1 = I.C[1], C2 = I.C[2];
    const int npair = I.C[0] * C1;
    const int gsh = I.gshift, gmask = (1 << gsh) - 1;  // entry = (tile << gsh) | position
    // fast path: C2 <= 4, <= 4 pairs per lane, <= KG offset groups (1, or 4 for
    // launches with several); same summation order as the general loop below
    constexpr int kC2 = 4, kPr = 4, kG = KG;
    if (C2 <= kC2 && nsg <= kG && npair <= kPr * kLanesPerElem) {
      int e2v[kC2];
#pragma unroll
      for (int c2 = 0; c2 < kC2; ++c2) e2v[c2] = c2 < C2 ? g2[c2] : -1;
      int e0v[kPr], e1v[kPr];
#pragma unroll
      for (int j = 0; j < kPr; ++j) {
        const int pr = sub + j * kLanesPerElem;
        e0v[j] = e1v[j] = -1;
        if (pr < npair) {
          const int c0 = pr / C1, c1 = pr - c0 * C1;
          e0v[j] = g0[c0];
          e1v[j] = g1[c1];
        }
      }
      float v[kPr][kC2][kG];
#pragma unroll
      for (int j = 0; j < kPr; ++j) {
        const int e0 = e0v[j], e1 = e1v[j];
        const bool okp = (e0 | e1) >= 0;
        const int tb = ((e0 >> gsh) * I.nt[1] + (e1 >> gsh)) * I.nt[2];
        const int pb = ((e0 & gmask) * I.E[1] + (e1 & gmask)) * I.E[2];
#pragma unroll
        for (int c2 = 0; c2 < kC2; ++c2) {
          const int e2 = e2v[c2];
          const float* pp = I.part + ((size_t)(tb + (e2 >> gsh)) * nsg) * I.E123 + pb + (e2 & gmask);
#pragma unroll
          for (int g = 0; g < kG; ++g) {
            v[j][c2][g] = 0.f;
            if (okp && e2 >= 0 && g < nsg) v[j][c2][g] = pp[(size_t)g * I.E123];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kPr; ++j)
#pragma unroll
        for (int c2 = 0; c2 < kC2; ++c2)
#pragma unroll
          for (int g = 0; g < kG; ++g) T += v[j][c2][g];
    } else if (C2 <= kC2 && nsg <= kG) {
      // any number of pairs, one at a time: the pair's table entries, then all of its
      // (c2, offset group) partials at once (two memory latencies per pair instead of
      // one per partial); same summation order
      int e2v[kC2];
#pragma unroll
      for (int c2 = 0; c2 < kC2; ++c2) e2v[c2] = c2 < C2 ? g2[c2] : -1;
      for (int pr = sub; pr < npair; pr += kLanesPerElem) {
        const int c0 = pr / C1, c1 = pr - c0 * C1;
        const int e0 = g0[c0], e1 = g1[c1];
        const bool okp = (e0 | e1) >= 0;
        const int tb = ((e0 >> gsh) * I.nt[1] + (e1 >> gsh)) * I.nt[2];
        const int pb = ((e0 & gmask) * I.E[1] + (e1 & gmask)) * I.E[2];
        float v[kC2][kG];
#pragma unroll
        for (int c2 = 0; c2 < kC2; ++c2) {
          const int e2 = e2v[c2];
          const float* pp = I.part + ((size_t)(tb + (e2 >> gsh)) * nsg) * I.E123 + pb + (e2 & gmask);
#pragma unroll
          for (int g = 0; g < kG; ++g) {
            v[c2][g] = 0.f;
            if (okp && e2 >= 0 && g < nsg) v[c2][g] = pp[(size_t)g * I.E123];
          }
        }
#pragma unroll
        for (int c2 = 0; c2 < kC2; ++c2)
#pragma unroll
          for (int g = 0; g < kG; ++g) T += v[c2][g];
      }
    } else {
      for (int pr = sub; pr < npair; pr += kLanesPerElem) {
        const int c0 = pr / C1, c1 = pr - c0 * C1;
        const int e0 = g0[c0], e1 = g1[c1];
        if ((e0 | e1) < 0) continue;
        const int tb = ((e0 >> gsh) * I.nt[1] + (e1 >> gsh)) * I.nt[2];
        const int pb = ((e0 & gmask) * I.E[1] + (e1 & gmask)) * I.E[2];
        for (int c2 = 0; c2 < C2; ++c2) {
          const int e2 = g2[c2];
          if (e2 < 0) break;
          const float* pp = I.part + ((size_t)(tb + (e2 >> gsh)) * nsg) * I.E123 + pb + (e2 & gmask);
          for (int g = 0; g < nsg; ++g) T += pp[(size_t)g * I.E123];
        }
      }
    }
  }
#pragma unroll
  for (int o = 1; o < kLanesPerElem; o <<= 1) T += __shfl_xor(T, o, 64);
  if (in && sub == 0) {
    if (phase == kInit) {
      const float lv = obs ? mv : 0.f;
      I.L[t] = lv;
      acc = (double)lv * (double)lv;
    } else {
      float tk = T / (float)a.kt;
      if (I.prec != kFP32) {
        if (!I.st->refresh) tk += tprev;
        I.T[t] = tk;
      }
      float lv;
      if (!obs) {
        lv = tk;
      } else if (I.lam > 1e300) {
        lv = mv;
      } else {
        const double th = I.st->theta_cur;
        lv = (float)((th * (double)tk + I.lam * (double)mv) / (I.lam + th));
      }
      const float old = lold;
      I.L[t] = lv;
      if (I.prec != kFP32) I.D[t] = lv - old;
      const double d = (double)lv - (double)old;
      acc = d * d;
      // penalized program (finite lambda): ||P_Omega(L - M)||^2 of its objective
      if (obs && I.lam <= 1e300) {
        const double e = (double)lv - (double)mv;
        pen = e * e;
      }
    }
  }
  // block reductions in FP64, fixed order
  __shared__ double red[2][kThreads / 64];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    acc += __shfl_xor(acc, o, 64);
    pen += __shfl_xor(pen, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = acc;
    red[1][threadIdx.x >> 6] = pen;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    I.dlpart[2 * lb.y] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    I.dlpart[2 * lb.y + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// =====================================================================================
// colnorm, two launches. k_colnorm_reduce: block b of an instance reduces, in FP64,
// one tile range of one 64-column block (a lane per column, fixed order) and a share
// of the scalar partials. k_colnorm_finish (one block per instance): the ranges'
// column sums in range order, column norms -> shrink factors (Z-step), penalty
// schedule, residuals of the previous iteration, stopping decision, phase changes. The kernel boundary orders
// the two, so no device-scope fences or counters are needed.
// =====================================================================================
__global__ __launch_bounds__(kThreads) void k_colnorm_reduce(StageArgs a) {
  const int2 sl = a.slices[blockIdx.x];
  const CInstDev& I = *(const CInstDev*)(a.inst + sl.x);  // constant: see k_forward
  const int phase = I.st->phase;
  if (phase != kInit && phase != kRun) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kp = a.kp;
  const int nt = I.ntiles;
  double* colpart = I.slice;             // [kColRanges][kp][2]: sums of Q^2, W^2 per tile range
  double* scal = I.slice + 2 * kColRanges * kp;  // [nslice][3]: (Z - W)^2, ||dL||^2, ||P_Omega(L - M)||^2
  {
    // the kp / 4 blocks of an instance: 64-column block cb, tile range r (kColRanges
    // ranges per column block); lane = column, each wavefront a quarter of the range,
    // reading whole 256-byte runs of the partials [c / 64][tile][c % 64]
    const int ncb = kp >> 6;
    const int cb = sl.y % ncb, r = sl.y / ncb;
    const int rch = (nt + kColRanges - 1) / kColRanges, wch = (rch + 3) / 4;
    const int t0 = min(nt, r * rch + wave * wch), t1 = min(min(nt, (r + 1) * rch), t0 + wch);
    const float* qp = I.qpart + ((size_t)cb * nt) * 64 + lane;
    const float* wp = I.wpart + ((size_t)cb * nt) * 64 + lane;
    double q = 0.0, w = 0.0;
#pragma unroll 4
    for (int t = t0; t < t1; ++t) {
      q += (double)qp[(size_t)t * 64];
      w += (double)wp[(size_t)t * 64];
    }
    __shared__ double cred[2][kThreads / 64][64];
    cred[0][wave][lane] = q;
    cred[1][wave][lane] = w;
    __syncthreads();
    if (wave == 0) {
      double* d = colpart + 2 * ((size_t)r * kp + cb * 64 + lane);
      d[0] = ((cred[0][0][lane] + cred[0][1][lane]) + cred[0][2][lane]) + cred[0][3][lane];
      d[1] = ((cred[1][0][lane] + cred[1][1][lane]) + cred[1][2][lane]) + cred[1][3][lane];
    }
  }
  __shared__ double red[3][kThreads / 64];
  const int nr = nt * a.ncg;
  const int rch = (nr + I.nslice - 1) / I.nslice, lch = (I.nlblk + I.nslice - 1) / I.nslice;
  double r = 0.0, dl = 0.0, pn = 0.0;
  for (int i = sl.y * rch + tid; i < min(nr, (sl.y + 1) * rch); i += kThreads) r += (double)I.rpart[i];
  for (int i = sl.y * lch + tid; i < min(I.nlblk, (sl.y + 1) * lch); i += kThreads) {
    dl += I.dlpart[2 * i];
    pn += I.dlpart[2 * i + 1];
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    r += __shfl_xor(r, o, 64);
    dl += __shfl_xor(dl, o, 64);
    pn += __shfl_xor(pn, o, 64);
  }
  if (lane == 0) {
    red[0][wave] = r;
    red[1][wave] = dl;
    red[2][wave] = pn;
  }
  __syncthreads();
  if (tid == 0) {
    scal[3 * sl.y] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    scal[3 * sl.y + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    scal[3 * sl.y + 2] = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
  }
}

__global__ __launch_bounds__(kThreads) void k_colnorm_finish(StageArgs a) {
  const CInstDev& I = *(const CInstDev*)(a.inst + blockIdx.x);  // constant: see k_forward
  InstState* st = I.st;
  const int phase = st->phase;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (phase == kDone) return;
  if (phase == kNew) {
    if (tid == 0) st->phase = kInit;
    return;
  }
  const int kp = a.kp;
  // column sums: the tile ranges' partials added in range order (the sums land in the
  // first range's slots, read again below by the thread that wrote them)
  double* colsum = I.slice;
  const double* scal = I.slice + 2 * kColRanges * kp;
  __shared__ double sh_obj[kThreads / 64], sh_max[kThreads / 64], sh_rs[kThreads / 64], sh_ds[kThreads / 64],
      sh_pn[kThreads / 64];
  __shared__ double sh_sc[3];
  double obj = 0.0, mx = 0.0, rs = 0.0, ds = 0.0, pn = 0.0;
  for (int c = tid; c < kp; c += kThreads) {
    double q = 0.0, w = 0.0;
    for (int r = 0; r < kColRanges; ++r) {
      q += colsum[2 * ((size_t)r * kp + c)];
      w += colsum[2 * ((size_t)r * kp + c) + 1];
    }
    colsum[2 * c] = q;
    colsum[2 * c + 1] = w;
    obj += sqrt(w);
    mx = fmax(mx, sqrt(q));
  }
  // slice partials of the residual sums: strided over the block, fixed tree
  for (int j = tid; j < I.nslice; j += kThreads) {
    rs += scal[3 * j];
    ds += scal[3 * j + 1];
    pn += scal[3 * j + 2];
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    obj += __shfl_xor(obj, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    rs += __shfl_xor(rs, o, 64);
    ds += __shfl_xor(ds, o, 64);
    pn += __shfl_xor(pn, o, 64);
  }
  if (lane == 0) {
    sh_obj[wave] = obj;
    sh_max[wave] = mx;
    sh_rs[wave] = rs;
    sh_ds[wave] = ds;
    sh_pn[wave] = pn;
  }
  __syncthreads();
  if (tid == 0) {
    sh_sc[0] = ((sh_rs[0] + sh_rs[1]) + sh_rs[2]) + sh_rs[3];
    sh_sc[1] = ((sh_ds[0] + sh_ds[1]) + sh_ds[2]) + sh_ds[3];
    sh_sc[2] = ((sh_pn[0] + sh_pn[1]) + sh_pn[2]) + sh_pn[3];
  }
  __shared__ int go_on;
  if (tid == 0) {
    // ||A_k(L)V||_{2,1} (eq:InductiveCNNM); the penalized program (eq:admm) adds
    // (lambda k / 2) ||P_Omega(L - M)||_F^2 (zero at initialisation, L = P_Omega M)
    double objective = ((sh_obj[0] + sh_obj[1]) + sh_obj[2]) + sh_obj[3];
    if (I.lam <= 1e300) objective += 0.5 * I.lam * (double)a.kt * sh_sc[2];
    const double maxn = fmax(fmax(sh_max[0], sh_max[1]), fmax(sh_max[2], sh_max[3]));
    int go = 1;
    if (phase == kInit) {
      const double dn = sqrt(sh_sc[1]);
      st->denom = dn > 0.0 ? dn : 1.0;
      if (!(st->theta > 0.0)) st->theta = I.theta0 > 0.0 ? I.theta0 : (maxn > 0.0 ? 1.25 / maxn : 1.0);
      st->objective = objective;
      st->iters = 0;
      st->phase = kRun;
      if (I.max_iter <= 0) {
        st->phase = kDone;
        go = 0;
      }
    } else {
      const double kk = (double)a.kt;
      st->r_primal = sqrt(sh_sc[0]) / (sqrt(kk) * st->denom);
      st->r_change = sqrt(sh_sc[1]) / st->denom;
      st->objective = objective;
      st->iters += 1;
      if (!isfinite(st->r_primal) || !isfinite(st->r_change) || !isfinite(objective)) {
        st->status = -5;
        st->phase = kDone;
        go = 0;
      } else if (I.tol > 0.0 && fmax(st->r_primal, st->r_change) <= I.tol) {
        st->converged = 1;
        st->phase = kDone;
        go = 0;
      } else if (st->iters >= I.max_iter) {
        st->phase = kDone;
        go = 0;
      }
    }
    if (go) {
      const double th = st->theta;
      const double thn = fmin(I.rho * th, I.theta_max);
      st->theta_cur = th;
      st->ratio_prev = st->ratio;
      st->ratio = th / thn;
      st->theta = thn;
      st->refresh = (I.refresh_every <= 1) || (st->iters % I.refresh_every == 0) ||
                    (st->iters + 1 >= I.max_iter);
    }
    go_on = go;
  }
  __syncthreads();
  if (!go_on) return;
  const double th = st->theta_cur;
  for (int c = tid; c < kp; c += kThreads) {
    const double n = sqrt(colsum[2 * c]);
    const double sc = n > 0.0 ? fmax(0.0, 1.0 - 1.0 / (th * n)) : 0.0;
    I.s[c] = (float)sc;
  }
}

// =====================================================================================
// Operand layouts of V (kp x kp, zero padded), built once per solve.
//   Vf[((cb * nkb + sb) * 64 + l) * 16 + j] = V[sb*32 + 2j + l/32][cb*32 + l%32]
//   Va[((sb * nkb + cb) * 64 + l) * 16 + v] = V[sb*32 + l%32][cb*32 + acc_col(v, l/32)]
// =====================================================================================
__global__ void k_prep_v(const float* V, int k, int kp, float* Vf, float* Va, float* Vp) {
  const int nkb = kp / 32;
  const int64_t n = (int64_t)kp * kp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    {  // plain zero-padded kp x kp
      const int s = (int)(e / kp), c = (int)(e % kp);
      Vp[e] = (s < k && c < k) ? V[(int64_t)s * k + c] : 0.f;
    }
    const int j = (int)(e & 15);
    const int l = (int)((e >> 4) & 63);
    const int64_t blk = e >> 10;
    const int b2 = (int)(blk % nkb), b1 = (int)(blk / nkb);
    {  // forward: b1 = column block, b2 = offset block
      const int s = b2 * 32 + 2 * j + (l >> 5), c = b1 * 32 + (l & 31);
      Vf[e] = (s < k && c < k) ? V[(int64_t)s * k + c] : 0.f;
    }
    {  // adjoint: b1 = offset block, b2 = column block
      const int s = b1 * 32 + (l & 31), c = b2 * 32 + acc_col(j, l >> 5);
      Va[e] = (s < k && c < k) ? V[(int64_t)s * k + c] : 0.f;
    }
  }
}

//   Vf_lo[((cb * nhs + kk) * 64 + l) * 8 + j] = V[16*kk + 8*(l/32) + j][cb*32 + l%32]
//   Va_lo[(((sb * nkb + cb) * 2 + p) * 64 + l) * 8 + j] = V[sb*32 + l%32][cb*32 + acc_col(8p + j, l/32)]
//   Vp_lo[s * kp + c] = V[s][c] (zero-padded)
template <int MODE>
__global__ void k_prep_v_lp(const float* V, int k, int kp, void* Vf_lo, void* Va_lo, void* Vp_lo) {
  typedef typename LowP<MODE>::h H;
  H* vf = reinterpret_cast<H*>(Vf_lo);
  H* va = reinterpret_cast<H*>(Va_lo);
  H* vp = reinterpret_cast<H*>(Vp_lo);
  const int nkb = kp / 32, nhs = kp / 16;
  const int64_t n = (int64_t)kp * kp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    {
      const int s = (int)(e / kp), c = (int)(e % kp);
      vp[e] = (H)((s < k && c < k) ? V[(int64_t)s * k + c] : 0.f);
    }
    const int j = (int)(e & 7);
    const int l = (int)((e >> 3) & 63);
    const int64_t blk = e >> 9;
    {
      const int kk = (int)(blk % nhs), cb = (int)(blk / nhs);
      const int s = 16 * kk + 8 * (l >> 5) + j, c = cb * 32 + (l & 31);
      vf[e] = (H)((s < k && c < k) ? V[(int64_t)s * k + c] : 0.f);
    }
    {
      const int p = (int)(blk & 1);
      const int64_t sc = blk >> 1;
      const int cb = (int)(sc % nkb), sb = (int)(sc / nkb);
      const int s = sb * 32 + (l & 31), c = cb * 32 + acc_col(8 * p + j, l >> 5);
      va[e] = (H)((s < k && c < k) ? V[(int64_t)s * k + c] : 0.f);
    }
  }
}

// Split-BF16 copies for the kX3 kernels: V = head + tail + O(2^-18 |V|), head = BF16(V),
// tail = BF16(V - head); the same layouts as Vf_lo and Vp_lo, each array kp x kp heads
// followed by kp x kp tails.
__global__ void k_prep_v_x3(const float* V, int k, int kp, __bf16* vf, __bf16* vp) {
  const int nhs = kp / 16;
  const int64_t n = (int64_t)kp * kp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    {
      const int s = (int)(e / kp), c = (int)(e % kp);
      const float v = (s < k && c < k) ? V[(int64_t)s * k + c] : 0.f;
      const __bf16 h = (__bf16)v;
      vp[e] = h;
      vp[n + e] = (__bf16)(v - (float)h);
    }
    const int j = (int)(e & 7);
    const int l = (int)((e >> 3) & 63);
    const int64_t blk = e >> 9;
    const int kk = (int)(blk % nhs), cb = (int)(blk / nhs);
    const int s = 16 * kk + 8 * (l >> 5) + j, c = cb * 32 + (l & 31);
    const float v = (s < k && c < k) ? V[(int64_t)s * k + c] : 0.f;
    const __bf16 h = (__bf16)v;
    vf[e] = h;
    vf[n + e] = (__bf16)(v - (float)h);
  }
}

// max_{i,j} |(V^T V - I)_{ij}| with FP64 dot products.
__global__ void k_check_v(const float* V, int k, float* out) {
  __shared__ float red[kThreads];
  float mx = 0.f;
  const int64_t n = (int64_t)k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    double d = 0.0;
    for (int s = 0; s < k; ++s) d += (double)V[(int64_t)s * k + i] * (double)V[(int64_t)s * k + j];
    if (i == j) d -= 1.0;
    mx = fmaxf(mx, (float)fabs(d));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<int*>(out), __float_as_int(red[0]));
}

// =====================================================================================
// Gram accumulation for learning V (Definition 3, eq:A), in FP64.
// sum_i A_k(L)[i,s] A_k(L)[i,s'] = sum_x L[x] L[x + s - s'] = R(s - s'), the circular
// autocorrelation at lag d = s - s' in the box [-(k-1), k-1]. A block stages a tile of
// L with its circular halo (the tile extended by k - 1 on both sides) in LDS and every
// thread accumulates kAcLpt lags over the tile's positions (products of FP32 values are
// exact in FP64); blocks loop over tiles, so each leaves one partial per lag, and a
// second kernel sums the partials of all blocks in a fixed order: deterministic.
// =====================================================================================
constexpr int kAcLpt = 16;

__global__ __launch_bounds__(kThreads) void k_autocorr_tiled(const float* L, AcGeom g, double* part) {
  extern __shared__ float halo[];
  const int k0 = g.k[0], k1 = g.k[1], k2 = g.k[2];
  const int D1 = 2 * k1 - 1, D2 = 2 * k2 - 1;
  const int h1 = g.h[1], h2 = g.h[2], hsz = g.h[0] * h1 * h2;
  const int lag0 = blockIdx.y * kThreads * kAcLpt;
  int off[kAcLpt];
  double acc[kAcLpt];
#pragma unroll
  for (int i = 0; i < kAcLpt; ++i) {
    // lags past the last one read lag 0 (an in-box address) and are never stored, which
    // keeps the inner loop free of branches
    const int l = min(lag0 + (int)threadIdx.x + i * kThreads, g.nlags - 1);
    const int d2 = l % D2 - (k2 - 1), d1 = (l / D2) % D1 - (k1 - 1), d0 = l / (D1 * D2) - (k0 - 1);
    off[i] = (d0 * h1 + d1) * h2 + d2;
    acc[i] = 0.0;
  }
  const int nown = min(kAcLpt, max(0, (g.nlags - lag0 - (int)threadIdx.x + kThreads - 1) / kThreads));
  const int h0 = g.h[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int tile = blockIdx.x; tile < g.ntiles; tile += gridDim.x) {
    const int n2 = tile % g.nt[2], r = tile / g.nt[2];
    const int n1 = r % g.nt[1], n0 = r / g.nt[1];
    const int o0 = n0 * g.t[0], o1 = n1 * g.t[1], o2 = n2 * g.t[2];
    __syncthreads();  // the previous tile's reads are done
    // one halo line (i0, i1) per wavefront pass, its i2 over the lanes; source
    // coordinates o - (k - 1) + i lie in (-m, 3m) (tile and kernel extents <= m), so
    // three conditional steps wrap them
    for (int row = wave; row < h0 * h1; row += kThreads / 64) {
      const int i0 = row / h1, i1 = row - i0 * h1;
      const int y0 = wrap3(o0 - (k0 - 1) + i0, g.m[0]), y1 = wrap3(o1 - (k1 - 1) + i1, g.m[1]);
      const float* src = L + ((int64_t)y0 * g.m[1] + y1) * g.m[2];
      float* dst = halo + (size_t)row * h2;
      for (int i2 = lane; i2 < h2; i2 += 64) dst[i2] = src[wrap3(o2 - (k2 - 1) + i2, g.m[2])];
    }
    __syncthreads();
    const int e0 = min(g.t[0], g.m[0] - o0), e1 = min(g.t[1], g.m[1] - o1), e2 = min(g.t[2], g.m[2] - o2);
    for (int p0 = 0; p0 < e0; ++p0)
      for (int p1 = 0; p1 < e1; ++p1) {
        const int rowb = ((p0 + k0 - 1) * h1 + (p1 + k1 - 1)) * h2 + (k2 - 1);
        for (int p2 = 0; p2 < e2; ++p2) {
          const int b = rowb + p2;
          const double lx = (double)halo[b];
#pragma unroll
          for (int i = 0; i < kAcLpt; ++i) acc[i] = fma(lx, (double)halo[b + off[i]], acc[i]);
        }
      }
  }
#pragma unroll
  for (int i = 0; i < kAcLpt; ++i) {
    const int l = lag0 + threadIdx.x + i * kThreads;
    if (i < nown) part[(size_t)blockIdx.x * g.nlags + l] = acc[i];
  }
}

// R[l] += sum over the nblk partials of lag l, in block order
__global__ void k_autocorr_reduce(const double* part, int nblk, int nlags, double* R) {
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nlags; l += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * nlags + l];
    R[l] += s;
  }
}

__global__ void k_gram_expand(const double* R, int k0, int k1, int k2, double* G) {
  const int k = k0 * k1 * k2;
  const int D1 = 2 * k1 - 1, D2 = 2 * k2 - 1;
  const int64_t n = (int64_t)k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(e / k), t = (int)(e % k);
    const int s2 = s % k2, s1 = (s / k2) % k1, s0 = s / (k1 * k2);
    const int t2 = t % k2, t1 = (t / k2) % k1, t0 = t / (k1 * k2);
    const int di = ((s0 - t0 + k0 - 1) * D1 + (s1 - t1 + k1 - 1)) * D2 + (s2 - t2 + k2 - 1);
    G[e] = R[di];
  }
}

__global__ void k_copy_f32(const float* src, float* dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// V of the kernel (k0, k1, k2) into the bank of the kernel (k0, k1, k2p), k2p >= k2:
// out[s'][i] = V[s][i] for the offset s' = (s0, s1, s2) with s2 < k2 and i < kt, else 0
__global__ void k_pad_v(const float* V, int k0, int k1, int k2, int k2p, float* out) {
  const int kt = k0 * k1 * k2, kc = k0 * k1 * k2p;
  const int64_t n = (int64_t)kc * kc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int sp = (int)(e / kc), i = (int)(e - (int64_t)sp * kc);
    const int s2 = sp % k2p, s01 = sp / k2p;
    out[e] = (s2 < k2 && i < kt) ? V[(int64_t)(s01 * k2 + s2) * kt + i] : 0.f;
  }
}

__global__ void k_fill_f32(float* dst, float v, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = v;
}

// ------------------------------------------------------------------------------------ launchers
static inline int grid_for(int64_t n, int cap = 65536) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

void launch_colnorm(const StageArgs& a, int nslices_total, int ninst, hipStream_t st) {
  hipLaunchKernelGGL(k_colnorm_reduce, dim3(nslices_total), dim3(kThreads), 0, st, a);
  hipLaunchKernelGGL(k_colnorm_finish, dim3(ninst), dim3(kThreads), 0, st, a);
}

template <int GV>
static void launch_adjoint_big_gv(const StageArgs& a, int ntiles_total, int mode, hipStream_t st) {
  const dim3 g(((ntiles_total + 7) / 8) * 8 * a.nsg), b(kThreads);
  if (mode == kFP32) {
    const int lds = std::max(2 * (128 + 256) * kBigPad, 128 * (128 + 4));
    if (a.u16)
      hipLaunchKernelGGL((k_adjoint_big<GV, 2>), g, b, lds * 4, st, a);
    else
      hipLaunchKernelGGL((k_adjoint_big<GV, 4>), g, b, lds * 4, st, a);
  } else if (mode == kX3) {
    const int lds = kBigX3Stage + a.kp;
    hipLaunchKernelGGL((k_adjoint_big_lp<kX3, GV>), g, b, lds * 4, st, a);
  } else {
    const int lds = kBigLpStage + a.kp;
    if (mode == kBF16) hipLaunchKernelGGL((k_adjoint_big_lp<kBF16, GV>), g, b, lds * 4, st, a);
    if (mode == kFP16) hipLaunchKernelGGL((k_adjoint_big_lp<kFP16, GV>), g, b, lds * 4, st, a);
  }
}

size_t adjoint_big_x3_lds_bytes(int kp) { return (size_t)(kBigX3Stage + kp) * 4; }

void launch_adjoint_big(const StageArgs& a, int ntiles_total, int mode, int gv, hipStream_t st) {
  if (gv == 8)
    launch_adjoint_big_gv<8>(a, ntiles_total, mode, st);
  else
    launch_adjoint_big_gv<0>(a, ntiles_total, mode, st);
}

template <int GV, bool KS>
static void launch_adjoint_gv(const StageArgs& a, int ntiles_total, int lds_floats, int mode, hipStream_t st) {
  const dim3 g(((ntiles_total + 7) / 8) * 8 * a.nsg), b(kThreads);
  if (mode == kBF16)
    hipLaunchKernelGGL((k_adjoint<kBF16, GV, 2, KS>), g, b, lds_floats * 4, st, a);
  else if (mode == kFP16)
    hipLaunchKernelGGL((k_adjoint<kFP16, GV, 2, KS>), g, b, lds_floats * 4, st, a);
  else if (a.u16)
    hipLaunchKernelGGL((k_adjoint<kFP32, GV, 2, KS>), g, b, lds_floats * 4, st, a);
  else
    hipLaunchKernelGGL((k_adjoint<kFP32, GV, 4, KS>), g, b, lds_floats * 4, st, a);
}

void launch_adjoint(const StageArgs& a, int ntiles_total, int lds_floats, int mode, int gv, hipStream_t st) {
  if (gv == 8)
    a.split ? launch_adjoint_gv<8, true>(a, ntiles_total, lds_floats, mode, st)
            : launch_adjoint_gv<8, false>(a, ntiles_total, lds_floats, mode, st);
  else
    a.split ? launch_adjoint_gv<0, true>(a, ntiles_total, lds_floats, mode, st)
            : launch_adjoint_gv<0, false>(a, ntiles_total, lds_floats, mode, st);
}

void launch_lstep(const StageArgs& a, int nlblocks_total, hipStream_t st) {
  // the four-group paths (more registers) only for launches with several offset
  // groups (the split form; kp of 512 and more)
  StageArgs b = a;
  b.nlblocks = nlblocks_total;
  const dim3 g(((nlblocks_total + 7) / 8) * 8);
  if (a.nsg > 1)
    hipLaunchKernelGGL(k_lstep<4>, g, dim3(kThreads), 0, st, b);
  else
    hipLaunchKernelGGL(k_lstep<1>, g, dim3(kThreads), 0, st, b);
}

template <bool KS>
static void launch_forward_ks(const StageArgs& a, int ntiles_total, int lds_floats, int mode, int rb,
                              hipStream_t st) {
  const dim3 g(ntiles_total, a.ncg), b(kThreads);
  const size_t lds = (size_t)lds_floats * 4;
  if (mode == kX3) {
    if constexpr (!KS) hipLaunchKernelGGL((k_forward<kX3, 2, 2, false>), g, b, lds, st, a);
  } else if (mode == kBF16) {
    if (rb == 4 && !KS)
      hipLaunchKernelGGL((k_forward<kBF16, 4, 2, false>), g, b, lds, st, a);
    else
      hipLaunchKernelGGL((k_forward<kBF16, 2, 2, KS>), g, b, lds, st, a);
  } else if (mode == kFP16) {
    if (rb == 4 && !KS)
      hipLaunchKernelGGL((k_forward<kFP16, 4, 2, false>), g, b, lds, st, a);
    else
      hipLaunchKernelGGL((k_forward<kFP16, 2, 2, KS>), g, b, lds, st, a);
  } else if (a.u16) {
    hipLaunchKernelGGL((k_forward<kFP32, 2, 2, KS>), g, b, lds, st, a);
  } else {
    hipLaunchKernelGGL((k_forward<kFP32, 2, 4, KS>), g, b, lds, st, a);
  }
}

void launch_forward(const StageArgs& a, int ntiles_total, int lds_floats, int mode, int rb, hipStream_t st) {
  if (a.split)
    launch_forward_ks<true>(a, ntiles_total, lds_floats, mode, rb, st);
  else
    launch_forward_ks<false>(a, ntiles_total, lds_floats, mode, rb, st);
}

void launch_prep_v(const float* V, int k, int kp, float* Vf, float* Va, float* Vp, void* Vf_lo, void* Va_lo,
                   void* Vp_lo, int prec, hipStream_t st) {
  const dim3 g(grid_for((int64_t)kp * kp, 4096)), b(kThreads);
  hipLaunchKernelGGL(k_prep_v, g, b, 0, st, V, k, kp, Vf, Va, Vp);
  if (prec == kBF16) hipLaunchKernelGGL(k_prep_v_lp<kBF16>, g, b, 0, st, V, k, kp, Vf_lo, Va_lo, Vp_lo);
  if (prec == kFP16) hipLaunchKernelGGL(k_prep_v_lp<kFP16>, g, b, 0, st, V, k, kp, Vf_lo, Va_lo, Vp_lo);
}

void launch_prep_v_x3(const float* V, int k, int kp, void* Vf_x, void* Vp_x, hipStream_t st) {
  hipLaunchKernelGGL(k_prep_v_x3, dim3(grid_for((int64_t)kp * kp, 4096)), dim3(kThreads), 0, st, V, k, kp,
                     reinterpret_cast<__bf16*>(Vf_x), reinterpret_cast<__bf16*>(Vp_x));
}

void launch_check_v(const float* V, int k, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_check_v, dim3(grid_for((int64_t)k * k, 1024)), dim3(kThreads), 0, st, V, k, out);
}

AcGeom autocorr_geometry(const int32_t* m, const int32_t* k) {
  // the tile box with the most positions per staged halo value that fits the LDS
  // budget (t_d powers of two or the whole dimension)
  AcGeom g{};
  for (int d = 0; d < 3; ++d) {
    g.m[d] = m[d];
    g.k[d] = k[d];
  }
  g.nlags = (2 * k[0] - 1) * (2 * k[1] - 1) * (2 * k[2] - 1);
  auto cands = [](int md) {
    std::vector<int> c;
    for (int t = 1; t < md && t <= 4096; t <<= 1) c.push_back(t);
    c.push_back(md);
    return c;
  };
  double best = -1.0;
  for (int t0 : cands(m[0]))
    for (int t1 : cands(m[1]))
      for (int t2 : cands(m[2])) {
        const int64_t h = (int64_t)(t0 + 2 * k[0] - 2) * (t1 + 2 * k[1] - 2) * (t2 + 2 * k[2] - 2);
        const int64_t pos = (int64_t)t0 * t1 * t2;
        if (h > kAcHaloFloats || pos > (1 << 16)) continue;
        const double score = (double)pos / (double)h + 1e-9 * (double)pos;
        if (score > best) {
          best = score;
          g.t[0] = t0;
          g.t[1] = t1;
          g.t[2] = t2;
        }
      }
  g.ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    g.h[d] = g.t[d] + 2 * k[d] - 2;
    g.nt[d] = (m[d] + g.t[d] - 1) / g.t[d];
    g.ntiles *= g.nt[d];
  }
  return g;
}

size_t autocorr_part_doubles(const int32_t* k) {
  return (size_t)kAcBlocks * (2 * k[0] - 1) * (2 * k[1] - 1) * (2 * k[2] - 1);
}

void launch_autocorr(const float* L, const int32_t* m, const int32_t* k, double* R, double* part, hipStream_t st) {
  // the smallest tile's halo is the lag box, prod(2 k_d - 1) < 8 prod(k_d) <= 32768
  // floats, so a tile box always fits
  const AcGeom g = autocorr_geometry(m, k);
  const int nchunks = (g.nlags + kThreads * kAcLpt - 1) / (kThreads * kAcLpt);
  const int nblk = std::min(kAcBlocks, g.ntiles);
  const size_t lds = (size_t)g.h[0] * g.h[1] * g.h[2] * 4;
  hipLaunchKernelGGL(k_autocorr_tiled, dim3(nblk, nchunks), dim3(kThreads), lds, st, L, g, part);
  hipLaunchKernelGGL(k_autocorr_reduce, dim3((g.nlags + kThreads - 1) / kThreads), dim3(kThreads), 0, st, part,
                     nblk, g.nlags, R);
}

void launch_gram_expand(const double* R, const int32_t* k, double* G, hipStream_t st) {
  const int64_t kk = (int64_t)k[0] * k[1] * k[2];
  hipLaunchKernelGGL(k_gram_expand, dim3(grid_for(kk * kk, 8192)), dim3(kThreads), 0, st, R, k[0], k[1], k[2], G);
}

void launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n, 8192)), dim3(kThreads), 0, st, src, dst, n);
}

void launch_pad_v(const float* V, const int* kd, const int* kdp, float* out, hipStream_t st) {
  const int64_t kc = (int64_t)kdp[0] * kdp[1] * kdp[2];
  hipLaunchKernelGGL(k_pad_v, dim3(grid_for(kc * kc, 8192)), dim3(kThreads), 0, st, V, kd[0], kd[1], kd[2], kdp[2], out);
}

void launch_fill_f32(float* dst, float v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 8192)), dim3(kThreads), 0, st, dst, v, n);
}

}  // namespace icnnm

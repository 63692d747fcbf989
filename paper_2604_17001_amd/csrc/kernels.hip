// HIP kernels of the ICNNM solver for gfx950 (CDNA4).
//
// Operators (Section II-B, Section III-D):
//   A_k(L)[i, s] = L[(i - s) mod m]           convolution matrix (eq:ak)
//   A_k^*(X)[t]  = sum_s X[(t + s) mod m, s]   its adjoint
// The m x k state arrays (scaled dual U and Q = W - U) are stored in "tile
// layout": for each 32-row group of a tile and each 32-column block, the 1024
// values sit in the order of the 32x32 MFMA accumulator, lane-major, so a lane
// reads and writes its 16 values as four 16-byte accesses and the adjoint
// consumes them directly as its B operand without a transpose.
//
// Accumulator layout of v_mfma_f32_32x32x2_f32 for D = A(32 x 2) B(2 x 32):
//   lane l, register v holds D[(v/4)*8 + (l/32)*4 + v%4][l%32];
//   lane l supplies A[l%32][l/32] and B[l/32][l%32].
#include "icnnm_dev.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace icnnm {

typedef float floatx16 __attribute__((ext_vector_type(16)));

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
__device__ __forceinline__ int kernel_off(int s, const InstDev& I, int k) {
  if (s >= k) return 0;
  int s2 = s % I.k[2];
  int t = s / I.k[2];
  int s1 = t % I.k[1];
  int s0 = t / I.k[1];
  return (s0 * I.E[1] + s1) * I.E[2] + s2;
}

// Box position of tile row r (C order inside the tile box), shifted by (k - 1) so
// that base - off(s) addresses row r's source (forward) or target (adjoint) t = r - s.
__device__ __forceinline__ int row_base(int r, const InstDev& I, const int* o, bool& valid) {
  int a2 = r % I.b[2];
  int t = r / I.b[2];
  int a1 = t % I.b[1];
  int a0 = t / I.b[1];
  valid = (o[0] + a0 < I.m[0]) && (o[1] + a1 < I.m[1]) && (o[2] + a2 < I.m[2]);
  return ((a0 + I.k[0] - 1) * I.E[1] + (a1 + I.k[1] - 1)) * I.E[2] + (a2 + I.k[2] - 1);
}

__device__ __forceinline__ void tile_origin(int lt, const InstDev& I, int* o) {
  int n2 = lt % I.nt[2];
  int t = lt / I.nt[2];
  int n1 = t % I.nt[1];
  int n0 = t / I.nt[1];
  o[0] = n0 * I.b[0];
  o[1] = n1 * I.b[1];
  o[2] = n2 * I.b[2];
}

// =====================================================================================
// forward: W = A_k(L) V, fused with the dual update and the next Q.
//   init (phase kInit): U = 0, Q = W                      (Y^0 = 0)
//   run  (phase kRun):  Z = s.Q_old, G = U_old + Z,
//                       U = (G - W) theta/theta',  Q = W - U
// and per-tile partial sums of Q^2, W^2 (per column) and (Z - W)^2.
// grid = (tiles, kp / 256 column groups); each wave takes (64 rows x 64 columns) units.
// =====================================================================================
__global__ __launch_bounds__(kThreads) void k_forward(StageArgs a) {
  extern __shared__ float smem[];
  const int2 tt = a.tiles[blockIdx.x];
  const InstDev& I = a.inst[tt.x];
  const int phase = I.st->phase;
  if (phase != kInit && phase != kRun) return;
  const bool init = phase == kInit;
  const int kp = a.kp, k = a.k;
  const int cg = blockIdx.y;
  const int CG = kp < kGroup ? kp : kGroup;
  const int lt = tt.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5;

  int o[3];
  tile_origin(lt, I, o);
  const int E123 = I.E123;
  float* halo = smem;                                   // E123
  int* offs = reinterpret_cast<int*>(halo + E123);      // kp
  const int nrc = I.bm / kRowUnit, ncc = CG / kColUnit;
  float* colq = reinterpret_cast<float*>(offs + kp);    // [nrc][CG]
  float* colw = colq + nrc * CG;                        // [nrc][CG]
  float* rred = colw + nrc * CG;                        // [nrc * ncc]

  // halo of L over the tile box extended backwards by k - 1, with circular wrap
  const float* L = I.L;
  const int E12 = I.E[1] * I.E[2];
  for (int x = tid; x < E123; x += kThreads) {
    int x0 = x / E12, rem = x - x0 * E12;
    int x1 = rem / I.E[2], x2 = rem - x1 * I.E[2];
    int g0 = wrapi(o[0] - (I.k[0] - 1) + x0, I.m[0]);
    int g1 = wrapi(o[1] - (I.k[1] - 1) + x1, I.m[1]);
    int g2 = wrapi(o[2] - (I.k[2] - 1) + x2, I.m[2]);
    halo[x] = L[((int64_t)g0 * I.m[1] + g1) * I.m[2] + g2];
  }
  for (int s = tid; s < kp; s += kThreads) offs[s] = kernel_off(s, I, k);
  __syncthreads();

  const float ratio = (float)I.st->ratio;
  const int nkb = kp / 32;
  for (int u = wave; u < nrc * ncc; u += 4) {
    const int rc = u / ncc, cc = u % ncc;
    const int c0 = cg * CG + cc * kColUnit;
    bool valid[2];
    int base[2];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) base[ib] = row_base(rc * 64 + ib * 32 + (lane & 31), I, o, valid[ib]);

    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = (floatx16)(0.0f);

    const float* vf0 = a.Vf + ((size_t)(c0 / 32) * nkb) * 1024 + lane * 16;
    const float* vf1 = vf0 + (size_t)nkb * 1024;
    for (int sb = 0; sb < nkb; ++sb) {
      float av0[16], av1[16];
      load16(vf0 + (size_t)sb * 1024, av0);
      load16(vf1 + (size_t)sb * 1024, av1);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int off = offs[sb * 32 + 2 * j + half];
        const float b0 = halo[base[0] - off];
        const float b1 = halo[base[1] - off];
        acc[0][0] = mfma32(av0[j], b0, acc[0][0]);
        acc[0][1] = mfma32(av0[j], b1, acc[0][1]);
        acc[1][0] = mfma32(av1[j], b0, acc[1][0]);
        acc[1][1] = mfma32(av1[j], b1, acc[1][1]);
      }
    }

    // fused epilogue
    float rsum = 0.f;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int cblk = c0 / 32 + cb;
      float sv[16];
      if (!init) load_cols16(I.s, cblk * 32, half, sv);
      float qs[16], ws[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) qs[v] = ws[v] = 0.f;
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) {
        const size_t sidx = ((((size_t)lt * (I.bm / 32) + rc * 2 + ib) * nkb + cblk) * 64 + lane) * 16;
        float uo[16], qo[16], un[16], qn[16];
        if (!init) {
          load16(I.U + sidx, uo);
          load16(I.Q + sidx, qo);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float w = acc[cb][ib][v];
          float unew, qnew;
          if (!valid[ib]) {
            w = 0.f;
            unew = 0.f;
            qnew = 0.f;
          } else if (init) {
            unew = 0.f;
            qnew = w;
          } else {
            const float z = sv[v] * qo[v];
            const float g = uo[v] + z;
            unew = (g - w) * ratio;
            qnew = w - unew;
            const float d = z - w;
            rsum += d * d;
          }
          un[v] = unew;
          qn[v] = qnew;
          qs[v] += qnew * qnew;
          ws[v] += w * w;
        }
        store16(I.U + sidx, un);
        store16(I.Q + sidx, qn);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float q = half_sum(qs[v]);
        const float w = half_sum(ws[v]);
        if ((lane & 31) == 0) {
          const int col = cc * kColUnit + cb * 32 + acc_col(v, half);
          colq[rc * CG + col] = q;
          colw[rc * CG + col] = w;
        }
      }
    }
    rsum = wave_sum(rsum);
    if (lane == 0) rred[u] = rsum;
  }
  __syncthreads();
  for (int c = tid; c < CG; c += kThreads) {
    float q = 0.f, w = 0.f;
    for (int rc = 0; rc < nrc; ++rc) {
      q += colq[rc * CG + c];
      w += colw[rc * CG + c];
    }
    I.qpart[(size_t)lt * kp + cg * CG + c] = q;
    I.wpart[(size_t)lt * kp + cg * CG + c] = w;
  }
  if (tid == 0) {
    float r = 0.f;
    for (int u = 0; u < nrc * ncc; ++u) r += rred[u];
    I.rpart[(size_t)lt * a.ncg + cg] = r;
  }
}

// =====================================================================================
// adjoint: T_partial = col2im(H), H = G V^T with G = U + s.Q (= (Y + theta Z)/theta).
// grid = (tiles, kp / 256 offset groups). Each wave computes H^T for (64 offsets x 64
// rows) units over the whole reduction over eigendirections, then scatters
// H[j, s] onto box position base(j) - off(s) with LDS float atomics.
// =====================================================================================
__global__ __launch_bounds__(kThreads) void k_adjoint(StageArgs a) {
  extern __shared__ float smem[];
  const int2 tt = a.tiles[blockIdx.x];
  const InstDev& I = a.inst[tt.x];
  if (I.st->phase != kRun) return;
  const int kp = a.kp, k = a.k;
  const int sg = blockIdx.y;
  const int SGW = kp < kGroup ? kp : kGroup;
  const int lt = tt.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5;
  int o[3];
  tile_origin(lt, I, o);
  const int E123 = I.E123;
  float* box = smem;
  int* offs = reinterpret_cast<int*>(box + E123);
  for (int x = tid; x < E123; x += kThreads) box[x] = 0.f;
  for (int s = tid; s < kp; s += kThreads) offs[s] = kernel_off(s, I, k);
  __syncthreads();

  const int nrc = I.bm / kRowUnit, nsc = SGW / kColUnit;
  const int nkb = kp / 32;
  for (int u = wave; u < nrc * nsc; u += 4) {
    const int rc = u / nsc, sc = u % nsc;
    const int s0 = sg * SGW + sc * kColUnit;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = (floatx16)(0.0f);
    const float* va0 = a.Va + ((size_t)(s0 / 32) * nkb) * 1024 + lane * 16;
    const float* va1 = va0 + (size_t)nkb * 1024;
    for (int cb = 0; cb < nkb; ++cb) {
      float sv[16];
      load_cols16(I.s, cb * 32, half, sv);
      float g[2][16];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const size_t sidx = ((((size_t)lt * (I.bm / 32) + rc * 2 + jb) * nkb + cb) * 64 + lane) * 16;
        float uo[16], qo[16];
        load16(I.U + sidx, uo);
        load16(I.Q + sidx, qo);
#pragma unroll
        for (int v = 0; v < 16; ++v) g[jb][v] = uo[v] + sv[v] * qo[v];
      }
      float va[2][16];
      load16(va0 + (size_t)cb * 1024, va[0]);
      load16(va1 + (size_t)cb * 1024, va[1]);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[0][0] = mfma32(va[0][v], g[0][v], acc[0][0]);
        acc[0][1] = mfma32(va[0][v], g[1][v], acc[0][1]);
        acc[1][0] = mfma32(va[1][v], g[0][v], acc[1][0]);
        acc[1][1] = mfma32(va[1][v], g[1][v], acc[1][1]);
      }
    }
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      bool valid;
      const int base = row_base(rc * 64 + jb * 32 + (lane & 31), I, o, valid);
#pragma unroll
      for (int sb = 0; sb < 2; ++sb) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int s = s0 + sb * 32 + acc_col(v, half);
          if (s < k) atomicAdd(&box[base - offs[s]], acc[sb][jb][v]);
        }
      }
    }
  }
  __syncthreads();
  float* dst = I.part + ((size_t)lt * a.nsg + sg) * E123;
  for (int x = tid; x < E123; x += kThreads) dst[x] = box[x];
}

// =====================================================================================
// lstep: T[t] = sum of the halo partials covering t;  L-step of Section III-D.
//   init (phase kInit): L = P_Omega(M), partial sums of ||P_Omega M||^2
//   run: lambda = inf: L = M on Omega, T/k elsewhere;
//        finite lambda: L = (theta T/k + lambda M)/(lambda + theta) on Omega, T/k elsewhere
//        partial sums of ||L_new - L_old||^2
// =====================================================================================
__global__ __launch_bounds__(kThreads) void k_lstep(StageArgs a) {
  const int2 lb = a.lblocks[blockIdx.x];
  const InstDev& I = a.inst[lb.x];
  const int phase = I.st->phase;
  if (phase != kInit && phase != kRun) return;
  const int64_t t = (int64_t)lb.y * kThreads + threadIdx.x;
  double acc = 0.0;
  if (t < I.mtot) {
    const bool obs = I.mask[t] != 0;
    const float mv = I.M[t];
    if (phase == kInit) {
      const float lv = obs ? mv : 0.f;
      I.L[t] = lv;
      acc = (double)lv * (double)lv;
    } else {
      const int t2 = (int)(t % I.m[2]);
      const int64_t r = t / I.m[2];
      const int t1 = (int)(r % I.m[1]);
      const int t0 = (int)(r / I.m[1]);
      const int32_t* g0 = I.gtab + I.goff[0] + t0 * I.C[0];
      const int32_t* g1 = I.gtab + I.goff[1] + t1 * I.C[1];
      const int32_t* g2 = I.gtab + I.goff[2] + t2 * I.C[2];
      const int nsg = a.nsg;
      float T = 0.f;
      for (int c0 = 0; c0 < I.C[0]; ++c0) {
        const int e0 = g0[c0];
        if (e0 < 0) break;
        for (int c1 = 0; c1 < I.C[1]; ++c1) {
          const int e1 = g1[c1];
          if (e1 < 0) break;
          for (int c2 = 0; c2 < I.C[2]; ++c2) {
            const int e2 = g2[c2];
            if (e2 < 0) break;
            const int tile = ((e0 >> 16) * I.nt[1] + (e1 >> 16)) * I.nt[2] + (e2 >> 16);
            const int pos = ((e0 & 0xffff) * I.E[1] + (e1 & 0xffff)) * I.E[2] + (e2 & 0xffff);
            const float* p = I.part + (size_t)tile * nsg * I.E123 + pos;
            for (int g = 0; g < nsg; ++g) T += p[(size_t)g * I.E123];
          }
        }
      }
      const float tk = T / (float)a.k;
      float lv;
      if (!obs) {
        lv = tk;
      } else if (I.lam > 1e300) {
        lv = mv;
      } else {
        const double th = I.st->theta_cur;
        lv = (float)((th * (double)tk + I.lam * (double)mv) / (I.lam + th));
      }
      const float old = I.L[t];
      I.L[t] = lv;
      const double d = (double)lv - (double)old;
      acc = d * d;
    }
  }
  // block reduction in FP64, fixed order
  __shared__ double red[kThreads / 64];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) I.dlpart[lb.y] = red[0] + red[1] + red[2] + red[3];
}

// =====================================================================================
// colnorm: FP64 reduction of the per-tile partials in slices, the last arriving block
// of an instance finishes: column norms -> shrink factors, penalty schedule,
// residuals of the previous iteration, stopping decision.
// =====================================================================================
__global__ __launch_bounds__(kThreads) void k_colnorm(StageArgs a) {
  const int2 sl = a.slices[blockIdx.x];
  const InstDev& I = a.inst[sl.x];
  InstState* st = I.st;
  const int phase = st->phase;
  const int tid = threadIdx.x;
  if (phase == kDone) return;
  // a new instance only moves to initialisation; the move is made by the last
  // arriving block so that no block of this launch sees the new phase
  if (phase == kNew) {
    if (tid == 0) {
      __threadfence();
      if (atomicAdd(&st->counter, 1u) == (unsigned)I.nslice - 1u) {
        st->counter = 0u;
        st->phase = kInit;
      }
    }
    return;
  }
  const int kp = a.kp;
  const int stride = 2 * kp + 2;
  double* out = I.slice + (size_t)sl.y * stride;
  const int tb = sl.y * a.tiles_per_slice;
  const int te = min(I.ntiles, tb + a.tiles_per_slice);
  for (int c = tid; c < kp; c += kThreads) {
    double q = 0.0, w = 0.0;
    for (int tI = tb; tI < te; ++tI) {
      q += (double)I.qpart[(size_t)tI * kp + c];
      w += (double)I.wpart[(size_t)tI * kp + c];
    }
    out[c] = q;
    out[kp + c] = w;
  }
  // scalars: (Z - W)^2 over the slice's tiles and this slice's share of L-step blocks
  __shared__ double red[2][kThreads / 64];
  double r = 0.0, dl = 0.0;
  for (int i = tb * a.ncg + tid; i < te * a.ncg; i += kThreads) r += (double)I.rpart[i];
  const int lpb = (I.nlblk + I.nslice - 1) / I.nslice;
  const int lb0 = sl.y * lpb, lb1 = min(I.nlblk, lb0 + lpb);
  for (int i = lb0 + tid; i < lb1; i += kThreads) dl += I.dlpart[i];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    r += __shfl_xor(r, o, 64);
    dl += __shfl_xor(dl, o, 64);
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = r;
    red[1][tid >> 6] = dl;
  }
  __syncthreads();
  if (tid == 0) {
    out[2 * kp] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    out[2 * kp + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
  // last-arriving block of this instance finishes
  __shared__ int last;
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(&st->counter, 1u);
    last = (prev == (unsigned)I.nslice - 1u);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();

  __shared__ double sh_obj[kThreads / 64], sh_max[kThreads / 64], sh_sc[2];
  double obj = 0.0, mx = 0.0;
  for (int c = tid; c < kp; c += kThreads) {
    double w = 0.0, q = 0.0;
    for (int j = 0; j < I.nslice; ++j) {
      q += I.slice[(size_t)j * stride + c];
      w += I.slice[(size_t)j * stride + kp + c];
    }
    obj += sqrt(w);
    mx = fmax(mx, sqrt(q));
    I.slice[c] = q;  // slice 0 row now holds the column sums (read back below by the same thread)
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    obj += __shfl_xor(obj, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  if ((tid & 63) == 0) {
    sh_obj[tid >> 6] = obj;
    sh_max[tid >> 6] = mx;
  }
  if (tid == 0) {
    double rs = 0.0, ds = 0.0;
    for (int j = 0; j < I.nslice; ++j) {
      rs += I.slice[(size_t)j * stride + 2 * kp];
      ds += I.slice[(size_t)j * stride + 2 * kp + 1];
    }
    sh_sc[0] = rs;
    sh_sc[1] = ds;
  }
  __syncthreads();
  __shared__ int go_on;
  if (tid == 0) {
    st->counter = 0u;
    const double objective = sh_obj[0] + sh_obj[1] + sh_obj[2] + sh_obj[3];
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
      const double kk = (double)a.k;
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
    const double n = sqrt(I.slice[c]);
    const double sc = n > 0.0 ? fmax(0.0, 1.0 - 1.0 / (th * n)) : 0.0;
    I.s[c] = (float)sc;
  }
}

// =====================================================================================
// Operand layouts of V (kp x kp, zero padded), built once per solve.
//   Vf[((cb * nkb + sb) * 64 + l) * 16 + j] = V[sb*32 + 2j + l/32][cb*32 + l%32]
//   Va[((sb * nkb + cb) * 64 + l) * 16 + v] = V[sb*32 + l%32][cb*32 + acc_col(v, l/32)]
// =====================================================================================
__global__ void k_prep_v(const float* V, int k, int kp, float* Vf, float* Va) {
  const int nkb = kp / 32;
  const int64_t n = (int64_t)kp * kp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
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
// autocorrelation at lag d = s - s' in the box [-(k-1), k-1]. One block per lag.
// =====================================================================================
__global__ __launch_bounds__(kThreads) void k_autocorr(const float* L, int m0, int m1, int m2, int k0,
                                                        int k1, int k2, double* R) {
  const int D1 = 2 * k1 - 1, D2 = 2 * k2 - 1;
  const int di = blockIdx.x;
  const int d2 = di % D2 - (k2 - 1);
  const int d1 = (di / D2) % D1 - (k1 - 1);
  const int d0 = di / (D1 * D2) - (k0 - 1);
  double acc = 0.0;
  const int rows = m0 * m1;
  for (int row = threadIdx.x / 64; row < rows; row += kThreads / 64) {
    const int x0 = row / m1, x1 = row % m1;
    const int y0 = (x0 + d0 + m0) % m0, y1 = (x1 + d1 + m1) % m1;
    const float* a = L + ((int64_t)x0 * m1 + x1) * m2;
    const float* b = L + ((int64_t)y0 * m1 + y1) * m2;
    for (int x2 = threadIdx.x & 63; x2 < m2; x2 += 64) {
      int y2 = x2 + d2;
      y2 += (y2 < 0) ? m2 : 0;
      y2 -= (y2 >= m2) ? m2 : 0;
      acc += (double)a[x2] * (double)b[y2];
    }
  }
  __shared__ double red[kThreads / 64];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) R[di] += red[0] + red[1] + red[2] + red[3];
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

// ------------------------------------------------------------------------------------ launchers
static inline int grid_for(int64_t n, int cap = 65536) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

void launch_colnorm(const StageArgs& a, int nslices_total, hipStream_t st) {
  hipLaunchKernelGGL(k_colnorm, dim3(nslices_total), dim3(kThreads), 0, st, a);
}

void launch_adjoint(const StageArgs& a, int ntiles_total, int lds_floats, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint, dim3(ntiles_total, a.nsg), dim3(kThreads), lds_floats * 4, st, a);
}

void launch_lstep(const StageArgs& a, int nlblocks_total, hipStream_t st) {
  hipLaunchKernelGGL(k_lstep, dim3(nlblocks_total), dim3(kThreads), 0, st, a);
}

void launch_forward(const StageArgs& a, int ntiles_total, int lds_floats, hipStream_t st) {
  hipLaunchKernelGGL(k_forward, dim3(ntiles_total, a.ncg), dim3(kThreads), lds_floats * 4, st, a);
}

void launch_prep_v(const float* V, int k, int kp, float* Vf, float* Va, void*, void*, int, hipStream_t st) {
  hipLaunchKernelGGL(k_prep_v, dim3(grid_for((int64_t)kp * kp, 4096)), dim3(kThreads), 0, st, V, k, kp, Vf, Va);
}

void launch_check_v(const float* V, int k, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_check_v, dim3(grid_for((int64_t)k * k, 1024)), dim3(kThreads), 0, st, V, k, out);
}

void launch_autocorr(const float* L, const int32_t* m, const int32_t* k, double* R, hipStream_t st) {
  const int nd = (2 * k[0] - 1) * (2 * k[1] - 1) * (2 * k[2] - 1);
  hipLaunchKernelGGL(k_autocorr, dim3(nd), dim3(kThreads), 0, st, L, m[0], m[1], m[2], k[0], k[1], k[2], R);
}

void launch_gram_expand(const double* R, const int32_t* k, double* G, hipStream_t st) {
  const int64_t kk = (int64_t)k[0] * k[1] * k[2];
  hipLaunchKernelGGL(k_gram_expand, dim3(grid_for(kk * kk, 8192)), dim3(kThreads), 0, st, R, k[0], k[1], k[2], G);
}

void launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n, 8192)), dim3(kThreads), 0, st, src, dst, n);
}

}  // namespace icnnm
